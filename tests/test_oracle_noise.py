"""Pins of the depolarizing-channel oracle (App. A, DEPOLARIZING CHANNEL).

Closed forms: certain insertions (a probability of 1) and the bit-flip
Markov chain, whose mean <Qz> after G gates is (1 - (1 - 2 p_x)^G) / 2."""
import math

import numpy as np

from oracle import core as O
from oracle import noise as Nz


def test_no_noise_is_the_circuit():
    circ = [("H", (0,), ()), ("CNOT", (0, 1), ()), ("T", (2,), ())]
    u = np.random.default_rng(0).random(len(circ) * 3)
    assert Nz.expand(circ, 3, 0.0, 0.0, 0.0, u) == circ


def test_certain_x_after_every_gate():
    # X on every qubit after H 0: X^n H|0...0> = |+> on qubit 0, |1> on the others
    n = 4
    u = np.zeros(n)
    psi = O.run(O.zero_state(n), n, Nz.expand([("H", (0,), ())], n, 1.0, 0.0, 0.0, u))
    want = np.zeros(1 << n, dtype=complex)
    want[0b1110] = want[0b1111] = 1 / math.sqrt(2)
    assert np.max(np.abs(psi - want)) < 1e-15


def test_certain_y_and_z():
    # Y|0> = i|1> (App. A matrix of Y), Z leaves |0> alone and flips the sign of |1>
    n = 1
    psi = O.run(O.zero_state(n), n, Nz.expand([("I", (0,), ())], n, 0.0, 1.0, 0.0, [0.5]))
    assert abs(psi[1] - 1j) < 1e-15 and psi[0] == 0
    psi = O.run(O.zero_state(n), n, Nz.expand([("X", (0,), ())], n, 0.0, 0.0, 1.0, [0.5]))
    assert abs(psi[1] + 1) < 1e-15


def test_draw_thresholds():
    circ = [("I", (0,), ())]
    for u, want in ((0.05, "X"), (0.15, "Y"), (0.25, "Z"), (0.35, None)):
        out = Nz.expand(circ, 1, 0.1, 0.1, 0.1, [u])
        assert (out[1][0] if len(out) > 1 else None) == want


def test_bit_flip_chain_mean():
    # G identity gates on |0>, p_x only: P(flipped) = (1 - (1 - 2 p)^G) / 2
    n, G, p, T = 2, 12, 0.05, 3000
    rng = np.random.default_rng(11)
    qz = np.zeros(n)
    for _ in range(T):
        u = rng.random(G * n)
        psi = O.run(O.zero_state(n), n, Nz.expand([("I", (0,), ())] * G, n, p, 0.0, 0.0, u))
        qz += O.expect_q(psi, n)[2]
    want = (1 - (1 - 2 * p) ** G) / 2
    sigma = math.sqrt(want * (1 - want) / T)
    assert np.all(np.abs(qz / T - want) < 4 * sigma)

"""Pins of the oracle's projection layer (App. A: M, CLEAR, SET) and of its
sampler (GENERATE EVENTS) on the CPU.

The App. B error-correction example fixes everything: its syndrome
measurements have certain outcomes, so the printed expectation values after
the corrections, CLEAR and SET do not depend on the random draws.  The
projection itself is checked against the projector |v><v| built as a dense
matrix, and the measurement rule against its threshold definition.  The
sampler is checked against closed forms (uniform, basis and GHZ states) and
a brute-force scan of the running sum."""
import json
import math
import os

import numpy as np
import pytest

from oracle import core as O
from oracle import dense as D


def rand_state(rng, n):
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return psi / np.linalg.norm(psi)


def program(fx, variant):
    to = lambda lst: [(g[0], tuple(g[1]), ()) for g in lst]
    return to(fx["prepare"]), to(fx["errors"][variant]) + to(fx["correct"])


@pytest.mark.parametrize("variant,syndrome", [("i", [0, 0]), ("ii", [1, 1]), ("iii", [0, 1])])
def test_appendix_b_error_correction(golden_dir, variant, syndrome):
    fx = json.load(open(os.path.join(golden_dir, "appB_error_correction.json")))
    n, d = fx["n_qubits"], fx["digits"]
    prep, rest = program(fx, variant)
    for draws in ([0.5, 0.5], [0.0, 0.999999]):
        psi = O.run(O.zero_state(n), n, prep)
        for got, key in zip(O.expect_q(psi, n), ("Qx", "Qy", "Qz")):
            assert np.all(np.round(got, d) == np.array(fx["first"][key])), (key, got)
        outcomes = O.run_program(psi, n, rest, draws)
        # the syndrome bits (q0 xor q1, q0 xor q2) of the injected errors
        assert outcomes == syndrome
        assert abs(O.norm2(psi, n) - 1.0) < 1e-14
        for got, key in zip(O.expect_q(psi, n), ("Qx", "Qy", "Qz")):
            assert np.all(np.round(got, d) == np.array(fx["final"][variant][key])), (variant, key, got)
    # closed forms behind 0.146 and 0.854: (1 -+ cos(pi/4)) / 2
    qz = O.expect_q(psi, n)[2]
    want = (1 - math.cos(math.pi / 4)) / 2 if variant != "iii" else (1 + math.cos(math.pi / 4)) / 2
    assert np.allclose(qz[:3], want, atol=1e-15) and qz[3] == 0.0 and abs(qz[4] - 1.0) < 1e-15


@pytest.mark.parametrize("q,v", [(0, 0), (0, 1), (2, 1), (4, 0)])
def test_project_is_the_normalised_projector(q, v):
    rng = np.random.default_rng(10 * q + v)
    n = 5
    psi = rand_state(rng, n)
    proj = np.zeros((2, 2), dtype=complex)
    proj[v, v] = 1.0
    ref = D.full_matrix(n, [q], [], proj) @ psi
    p_ref = float(np.vdot(ref, ref).real)
    ref /= math.sqrt(p_ref)
    got = psi.copy()
    p = O.project(got, n, q, v)
    assert abs(p - p_ref) < 1e-15
    assert np.max(np.abs(got - ref)) < 1e-15
    # projecting again is the identity (p = 1), the other value gives zero
    again = got.copy()
    assert abs(O.project(again, n, q, v) - 1.0) < 1e-15 and np.max(np.abs(again - got)) < 1e-15
    other = got.copy()
    assert O.project(other, n, q, 1 - v) == 0.0 and np.array_equal(other, got)


def test_measure_follows_the_threshold_rule():
    # one qubit rotated so that p1 = sin^2(0.6); u below p0 gives 0, at or above gives 1
    n = 3
    c, s = math.cos(0.6), math.sin(0.6)
    base = O.run(O.zero_state(n), n, [("MAT1", (1,), (c, 0, -s, 0, s, 0, c, 0)), ("H", (0,), ())])
    p1 = s * s
    for u, want in ((0.0, 0), (1 - p1 - 1e-9, 0), (1 - p1 + 1e-9, 1), (0.999999, 1)):
        psi = base.copy()
        out, p1_got = O.measure(psi, n, 1, u)
        assert out == want and abs(p1_got - p1) < 1e-15
        assert np.all(psi[((np.arange(1 << n) >> 1) & 1) != out] == 0)
        assert abs(O.norm2(psi, n) - 1.0) < 1e-15
    # on a grid of draws the outcome frequency is p1 to the grid's resolution
    grid = (np.arange(10000) + 0.5) / 10000
    ones = sum(O.measure(base.copy(), n, 1, u)[0] for u in grid)
    assert abs(ones / len(grid) - p1) <= 1e-4


def test_projection_onto_zero_amplitude_fails():
    n = 3
    psi = O.zero_state(n)
    assert O.project(psi, n, 1, 1) == 0.0 and psi[0] == 1.0
    with pytest.raises(ValueError):
        O.run_program(psi, n, [("SET", (2,), ())])
    # certain outcome whatever the draw
    for u in (0.0, 0.5, 0.999999):
        assert O.measure(O.zero_state(n), n, 2, u) == (0, 0.0)


def test_compact_projection_of_uniform_state_is_exact():
    # H on every qubit, then SET on qubit 3: half the amplitudes become
    # 2^(-(N-1)/2), all moduli equal, so the two-byte code is exact (range
    # r0 == r1, every kept code -127, every dropped code -128)
    n = 8
    st = O.CompactState.encode(O.uniform_state(n), n)
    p = st.project(3, 1)
    assert abs(p - 0.5) < 1e-15
    kept = ((np.arange(1 << n) >> 3) & 1) == 1
    assert np.all(st.b0[kept] == -127) and np.all(st.b0[~kept] == -128) and np.all(st.b1 == 0)
    assert st.rng[0] == st.rng[1] and abs(st.rng[0] - 2.0 ** (-(n - 1) / 2)) < 1e-16
    amp = st.decode()
    assert np.max(np.abs(amp[kept] - 2.0 ** (-(n - 1) / 2))) < 1e-16 and np.all(amp[~kept] == 0)


# -- GENERATE EVENTS (App. A): inverse-CDF sampling with the caller's draws --

def test_sample_uniform_state_is_floor_of_u():
    # p_i = 2^-N exactly, so the cumulative sums are exact and event = floor(u 2^N)
    n = 10
    u = np.concatenate([[0.0, 1 - 2.0 ** -40, 0.25, 0.5, 0.75], np.random.default_rng(1).random(500)])
    got = O.sample(O.uniform_state(n), n, u)
    assert np.array_equal(got, np.floor(u * 2 ** n).astype(np.uint64))


def test_sample_basis_and_ghz_states():
    n = 7
    u = np.random.default_rng(2).random(200)
    assert np.all(O.sample(O.basis_state(n, 77), n, u) == 77)
    ghz = O.run(O.zero_state(n), n, [("H", (0,), ())] + [("CNOT", (q, q + 1), ()) for q in range(n - 1)])
    u = u[np.abs(u - 0.5) > 1e-9]
    got = O.sample(ghz, n, u)
    assert np.array_equal(got, np.where(u < 0.5, 0, (1 << n) - 1).astype(np.uint64))


def test_sample_is_the_first_index_past_the_target():
    # brute force: scan the running sum in index order
    rng = np.random.default_rng(3)
    n = 6
    psi = rand_state(rng, n)
    psi[rng.random(1 << n) < 0.3] = 0  # zero-probability states are never drawn
    u = rng.random(300)
    got = O.sample(psi, n, u)
    p = psi.real * psi.real + psi.imag * psi.imag
    total = 0.0
    for x in p:
        total = total + x
    for k in range(len(u)):
        t, c = u[k] * total, 0.0
        for i in range(1 << n):
            c = c + p[i]
            if c > t:
                break
        assert got[k] == i and p[i] > 0
    # frequencies on a fine grid of draws are the probabilities
    grid = (np.arange(20000) + 0.5) / 20000
    counts = np.bincount(O.sample(psi, n, grid).astype(np.int64), minlength=1 << n)
    assert np.max(np.abs(counts / len(grid) - p / p.sum())) <= 1.0 / len(grid)

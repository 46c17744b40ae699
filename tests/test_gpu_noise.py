"""GPU parity of the depolarizing channel (App. A, DEPOLARIZING CHANNEL)
through the C ABI: jq_apply_circuit_noisy against the oracle's explicit
expansion run by its C core, on the same draws."""
import math

import numpy as np
import pytest

from oracle import core as O
from oracle import noise as Nz
from paper_1805_04708_amd import jq
from paper_1805_04708_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = {"c128": 1e-12, "c64": 2e-6}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    jq.lib()


@pytest.mark.parametrize("enc", ["c128", "c64"])
@pytest.mark.parametrize("n,fusion", [(6, 0), (12, 0), (12, 1)])
def test_noisy_circuit_matches_oracle(enc, n, fusion):
    circ = W.random_circuit(n, 80, seed=70 + n) + [("I", (0,), ())]
    u = np.random.default_rng(n).random(len(circ) * n)
    px, py, pz = 0.03, 0.02, 0.04
    ref = O.run(O.zero_state(n), n, Nz.expand(circ, n, px, py, pz, u))
    with jq.State(n, enc) as s:
        s.apply_circuit_noisy(circ, px, py, pz, u, fusion=fusion)
        assert O.rel_l2(s.amplitudes(), ref) < TOL[enc] * 3


def test_noisy_two_byte_code_matches_oracle():
    n = 10
    circ = W.random_circuit(n, 60, seed=3)
    u = np.random.default_rng(4).random(len(circ) * n)
    px, py, pz = 0.02, 0.02, 0.02
    exp = Nz.expand(circ, n, px, py, pz, u)
    st = O.CompactState.encode(O.zero_state(n), n).run(exp)
    with jq.State(n, "compact") as s:
        s.apply_circuit_noisy(circ, px, py, pz, u)
        b0, b1, rng = s.codes()
        amps = s.amplitudes()
    d0 = np.abs(b0.astype(int) - st.b0.astype(int))
    d1 = np.abs(((b1.astype(int) - st.b1.astype(int)) + 128) % 256 - 128)
    assert int(np.sum((d0 != 0) | (d1 != 0))) <= max(2, 0.01 * d0.size)
    exact = O.run(O.zero_state(n), n, exp)
    assert 1 - O.fidelity(amps, exact) <= 2 * (1 - O.fidelity(st.decode(), exact)) + 1e-12


def test_zero_probabilities_equal_the_plain_circuit():
    n = 11
    circ = W.random_circuit(n, 100, seed=8)
    u = np.random.default_rng(1).random(len(circ) * n)
    with jq.State(n, "c128") as a, jq.State(n, "c128") as b:
        a.apply_circuit(circ)
        b.apply_circuit_noisy(circ, 0.0, 0.0, 0.0, u)
        assert np.array_equal(a.amplitudes(), b.amplitudes())


def test_certain_x_after_every_gate():
    n = 5
    with jq.State(n, "c128") as s:
        s.apply_circuit_noisy([("H", (0,), ())], 1.0, 0.0, 0.0, np.zeros(n))
        want = np.zeros(1 << n, dtype=complex)
        want[0b11110] = want[0b11111] = 1 / math.sqrt(2)
        assert np.max(np.abs(s.amplitudes() - want)) < 1e-15


def test_bit_flip_chain_mean_over_trajectories():
    n, G, p, T = 2, 12, 0.05, 600
    rng = np.random.default_rng(21)
    qz = np.zeros(n)
    circ = [("I", (0,), ())] * G
    with jq.State(n, "c128") as s:
        for _ in range(T):
            s.init(jq.JQ_INIT_ZERO)
            s.apply_circuit_noisy(circ, p, 0.0, 0.0, rng.random(G * n))
            qz += s.expectations()[2]
    want = (1 - (1 - 2 * p) ** G) / 2
    sigma = math.sqrt(want * (1 - want) / T)
    assert np.all(np.abs(qz / T - want) < 4 * sigma)


def test_noisy_argument_errors_leave_state():
    n = 4
    circ = [("H", (1,), ())]
    with jq.State(n, "c128") as s:
        s.apply_circuit([("H", (0,), ())])
        before = s.amplitudes()
        for px, py, pz, u in ((0.6, 0.6, 0.0, np.zeros(n)), (-0.1, 0, 0, np.zeros(n)),
                              (0.1, 0, 0, np.full(n, 1.0)), (0.1, 0, 0, np.full(n, np.nan))):
            with pytest.raises(jq.JqError) as e:
                s.apply_circuit_noisy(circ, px, py, pz, u)
            assert e.value.code == jq.JQ_EINVAL
        with pytest.raises(jq.JqError):
            s.apply_circuit_noisy(circ, 0.1, 0, 0, np.zeros(n + 1))
        assert np.array_equal(s.amplitudes(), before)

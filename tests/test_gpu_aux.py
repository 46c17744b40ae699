"""GPU parity of the auxiliary-variable amplitudes (Sec. 4.2) through the C
ABI: jq_aux_amplitudes against the oracle's Eq. appa7 sum and against state
vectors; a 48-qubit case, far beyond any state vector, against a closed form
that factorises over independent qubit pairs."""
import math

import numpy as np
import pytest

from oracle import aux as A
from oracle import core as O
from paper_1805_04708_amd import jq
from paper_1805_04708_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    jq.lib()


def mixed_circuit(n, n_single, n_pairs, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_single + n_pairs):
        if i % 3 != 2 or n_pairs == 0:
            q = int(rng.integers(n))
            out.append(("MAT1", (q,), W.haar_u2(rng)) if rng.random() < 0.5 else ("H", (q,), ()))
        else:
            n_pairs -= 1
            a, b = (int(x) for x in rng.permutation(n)[:2])
            out.append([("CNOT", (a, b), ()), ("CZ", (a, b), ()), ("U", (a, b), (int(rng.integers(1, 6)),)),
                        ("CP", (a, b), (float(rng.uniform(-3, 3)),)), ("T", (a,), ()), ("X", (b,), ())][
                int(rng.integers(6))])
    return out


@pytest.mark.parametrize("n,pairs,seed", [(3, 0, 1), (5, 4, 2), (8, 8, 3)])
def test_matches_oracle_sum(n, pairs, seed):
    circ = mixed_circuit(n, 3 * n, pairs, seed)
    ref = A.amplitudes(circ, n, range(1 << n))
    got = jq.aux_amplitudes(n, circ, np.arange(1 << n))
    assert np.max(np.abs(got - ref)) < 1e-12


@pytest.mark.parametrize("n,pairs", [(14, 12), (20, 16)])
def test_matches_state_vector(n, pairs):
    circ = mixed_circuit(n, 2 * n, pairs, n)
    idx = np.random.default_rng(n).integers(0, 1 << n, 40).astype(np.uint64)
    got = jq.aux_amplitudes(n, circ, idx)
    with jq.State(n, "c128") as s:
        s.apply_circuit(circ)
        amp = s.amplitudes()
    assert np.max(np.abs(got - amp[idx.astype(np.int64)])) < 1e-10
    # against the oracle's state vector too (not only the GPU's)
    ref = O.run(O.zero_state(n), n, circ)
    assert np.max(np.abs(got - ref[idx.astype(np.int64)])) < 1e-10


def test_48_qubits_factorised_pairs():
    # 24 independent pairs (2p, 2p+1): H H, CZ, Haar U(2) on the second, T on
    # the first: the state is a product of two-qubit states, so every
    # amplitude is a product of 24 two-qubit amplitudes
    n = 48
    rng = np.random.default_rng(48)
    circ, pair_states = [], []
    for p in range(n // 2):
        a, b = 2 * p, 2 * p + 1
        u = W.haar_u2(rng)
        g = [("H", (a,), ()), ("H", (b,), ()), ("CZ", (a, b), ()), ("MAT1", (b,), u), ("T", (a,), ())]
        circ += g
        loc = [(x[0], tuple(0 if q == a else 1 for q in x[1]), x[2]) for x in g]
        pair_states.append(O.run(O.zero_state(2), 2, loc))
    idx = rng.integers(0, 1 << 62, 64, dtype=np.uint64) & np.uint64((1 << n) - 1)
    idx[0] = 0
    want = np.ones(len(idx), dtype=complex)
    for p in range(n // 2):
        two = ((idx >> np.uint64(2 * p)) & np.uint64(3)).astype(np.int64)
        want *= pair_states[p][two]
    got = jq.aux_amplitudes(n, circ, idx)
    assert np.allclose(got, want, rtol=1e-9, atol=1e-20)


def test_aux_errors():
    for circ in ([("SWAP", (0, 1), ())], [("TOFFOLI", (0, 1, 2), ())], [("H", (0,), (), (1,))]):
        with pytest.raises(jq.JqError) as e:
            jq.aux_amplitudes(4, circ, [0])
        assert e.value.code == jq.JQ_EUNSUPPORTED
    with pytest.raises(jq.JqError) as e:
        jq.aux_amplitudes(42, [("CZ", (q, q + 1), ()) for q in range(41)], [0])
    assert e.value.code == jq.JQ_EUNSUPPORTED
    with pytest.raises(jq.JqError) as e:
        jq.aux_amplitudes(4, [("H", (0,), ())], [16])
    assert e.value.code == jq.JQ_EINVAL

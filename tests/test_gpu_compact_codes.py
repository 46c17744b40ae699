"""GPU checks of the fused code-domain passes of the two-byte code with
per-gate quantisation (the default compact mode).  Permutations and
modulus-preserving phase shifts by a non-tie integer are exact on the codes,
so runs of them execute as one tile pass; the codes must be bit-identical to
running every gate through its own per-gate kernel (fusion=1), which the
parity tests compare with the oracle."""
import numpy as np
import pytest

from paper_1805_04708_amd import jq
from paper_1805_04708_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    jq.lib()


def run_both(n, circ, init=None, codes=None, search=jq.JQ_SEARCH_AUTO):
    out = []
    for fusion in (0, 1):
        with jq.State(n, "compact") as s:
            if init is not None:
                s.init(init)
            if codes is not None:
                s.write_codes(*codes)
            s.apply_circuit(circ, fusion=fusion, search=search)
            out.append(s.codes())
    return out


def assert_same(a, b):
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("search", [jq.JQ_SEARCH_AUTO, jq.JQ_SEARCH_ON])
@pytest.mark.parametrize("n", [8, 12, 15])
def test_rz_cnot_chain_bit_identical(n, search):
    # with the search forced on: the code passes a 2^29-code state gets
    layers = 3 if search == jq.JQ_SEARCH_AUTO else 12
    fused, single = run_both(n, W.rz_cnot_chain(n, layers, seed=n), init=jq.JQ_INIT_UNIFORM, search=search)
    assert_same(fused, single)


@pytest.mark.parametrize("n", [12, 16])
def test_random_circuit_with_dense_gates_bit_identical(n):
    # dense gates (H, Haar U(2)) break the code runs and keep their place
    fused, single = run_both(n, W.random_circuit(n, 200, seed=300 + n))
    assert_same(fused, single)


def test_controls_ties_and_every_code_op():
    n = 13
    rng = np.random.default_rng(5)
    circ = [("H", (q,), ()) for q in range(n)]
    for _ in range(120):
        q = [int(x) for x in rng.permutation(n)[:4]]
        kind = int(rng.integers(12))
        circ.append([("X", (q[0],), ()), ("CNOT", (q[0], q[1]), ()), ("TOFFOLI", (q[0], q[1], q[2]), ()),
                     ("X", (q[0],), (), (q[1], q[2], q[3])), ("Z", (q[0],), ()), ("S", (q[0],), ()),
                     ("T+", (q[0],), ()), ("CZ", (q[0], q[1]), ()), ("R", (q[0],), (int(rng.integers(1, 11)),)),
                     ("U", (q[0], q[1]), (int(rng.integers(1, 11)),)), ("SWAP", (q[0], q[1]), ()),
                     ("SWAP", (q[0], q[1]), (), (q[2],))][kind])
    # random codes (canonical: zero amplitudes carry phase code 0)
    b0 = rng.integers(-127, 127, 1 << n).astype(np.int8)
    b1 = rng.integers(-128, 128, 1 << n).astype(np.int8)
    b0[rng.random(1 << n) < 0.1] = -128
    b1[b0 == -128] = 0
    for search in (jq.JQ_SEARCH_AUTO, jq.JQ_SEARCH_ON):
        fused, single = run_both(n, circ, codes=(b0, b1, (0.01, 0.3)), search=search)
        assert_same(fused, single)
    order, blen, fused_flags = jq.plan_schedule(n, "compact", circ)
    assert fused_flags.any()


def test_full_size_layer_bit_identical():
    n = 28
    fused, single = run_both(n, W.rz_cnot_chain(n, 2, seed=28), init=jq.JQ_INIT_UNIFORM)
    assert_same(fused, single)


@pytest.mark.parametrize("fusion", [0, 3, 4, 5, 6, 7])
def test_qubit0_controls_selectors_and_targets(fusion):
    # two codes share a register in the code pass (qubit 0 picks the half):
    # controls and selectors on qubit 0 act on one half of every register,
    # a target on qubit 0 swaps the halves; every tile depth K
    n = 16
    rng = np.random.default_rng(70 + fusion)
    circ = [("H", (q,), ()) for q in range(n)]
    for _ in range(150):
        t = int(rng.integers(1, n))
        u = int(rng.choice([q for q in range(1, n) if q != t]))
        circ.append([("CNOT", (0, t), ()), ("TOFFOLI", (0, u, t), ()), ("CNOT", (t, 0), ()),
                     ("X", (0,), (), (t,)), ("CZ", (0, t), ()), ("CP", (0, t), (float(rng.uniform(-3, 3)),)),
                     ("RZ", (0,), (float(rng.uniform(0, 6.2)),)), ("U1", (t,), (float(rng.uniform(-3, 3)),), (0,)),
                     ("CP", (t, u), (float(rng.uniform(-3, 3)),)), ("X", (t,), (), (0, u))][int(rng.integers(10))])
    b0 = rng.integers(-127, 127, 1 << n).astype(np.int8)
    b1 = rng.integers(-128, 128, 1 << n).astype(np.int8)
    b0[rng.random(1 << n) < 0.2] = -128
    b1[b0 == -128] = 0
    out = []
    for fu in (fusion, 1):
        with jq.State(n, "compact") as s:
            s.write_codes(b0, b1, (0.01, 0.3))
            s.apply_circuit(circ, fusion=fu)
            out.append(s.codes())
    assert_same(out[0], out[1])
    if fusion != 1:
        _, blen, fused = jq.plan_schedule(n, "compact", circ, fusion=fusion)
        assert fused.any()

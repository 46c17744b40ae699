"""jq_apply_circuit_noalloc (fused ops staged in the library's fixed per-GPU
workspace) against jq_apply_circuit, through the C ABI.

Both calls run the same plan through the same kernels, so the results must
be identical bit for bit: amplitudes for complex128 / complex64, both code
planes and the (r0, r1) range for the two-byte code.  Each case makes two
calls in a row on the shared workspace, the second with a smaller state and
a shorter circuit; the complex128 result is also held to the oracle
(relative L2 <= 1e-12).
"""
import ctypes

import numpy as np
import pytest

from oracle import core as O
from paper_1805_04708_amd import jq
from paper_1805_04708_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    try:
        import torch
        ok = torch.cuda.is_available()
    except Exception:
        ok = False
    if not ok:
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    jq.lib()


def _noalloc(state, circuit, compact_mode, search):
    arr, cnt = jq.gates(circuit)
    opts = jq.exec_opts(0, compact_mode, 0, search)
    return jq.lib().jq_apply_circuit_noalloc(state.h, arr, cnt, ctypes.byref(opts))


def _result(state, enc):
    if enc == "compact":
        b0, b1, rng = state.codes()
        return b0.copy(), b1.copy(), np.asarray(rng, dtype=np.float64).copy()
    return (state.amplitudes(),)


def _same(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        assert x.shape == y.shape
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))


CASES = [
    ("c128", jq.JQ_COMPACT_PER_GATE),
    ("c64", jq.JQ_COMPACT_PER_GATE),
    ("compact", jq.JQ_COMPACT_PER_GATE),
    ("compact", jq.JQ_COMPACT_PER_BLOCK),
]


@pytest.mark.parametrize("enc,mode", CASES)
def test_noalloc_matches_apply_circuit_twice(enc, mode):
    # first call: 17 qubits, 8 layered Haar-U(2) + CZ layers and 200 random
    # gates with the large-state planner on (a few hundred fused ops);
    # second call: 11 qubits, 60 gates (fewer ops over the same workspace)
    calls = [
        (17, W.layered_u2_cz(17, 8, 31) + W.random_circuit(17, 200, 32), jq.JQ_SEARCH_ON),
        (11, W.random_circuit(11, 60, 33), jq.JQ_SEARCH_AUTO),
    ]
    for n, circ, search in calls:
        print(f"noalloc case enc={enc} mode={mode} n={n} gates={len(circ)}", flush=True)
        with jq.State(n, enc) as ref, jq.State(n, enc) as got:
            ref.apply_circuit(circ, compact_mode=mode, search=search)
            rc = _noalloc(got, circ, mode, search)
            assert rc == jq.JQ_OK, jq.lib().jq_last_error().decode()
            r_ref, r_got = _result(ref, enc), _result(got, enc)
            _same(r_ref, r_got)
            if enc == "c128":
                exact = O.run(O.zero_state(n), n, circ)
                assert O.rel_l2(r_got[0], exact) <= 1e-12


def test_noalloc_rejects_a_plan_larger_than_the_workspace():
    # 7000 CNOTs on a 12-qubit state plan as 7000 fused ops (704 bytes
    # each): more than the 4 MiB workspace holds
    n = 12
    rng = np.random.default_rng(7)
    circ = []
    for _ in range(7000):
        a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
        circ.append(("CNOT", (a, b), ()))
    steps = jq.plan_steps(n, "c128", circ)
    assert sum(s["n_ops"] for s in steps if s["fused"]) * 704 > 4 << 20
    start = W.random_circuit(n, 40, 8)
    with jq.State(n, "c128") as s:
        s.apply_circuit(start)
        before = s.amplitudes()
        rc = _noalloc(s, circ, jq.JQ_COMPACT_PER_GATE, jq.JQ_SEARCH_AUTO)
        assert rc == jq.JQ_EINVAL
        assert "workspace" in jq.lib().jq_last_error().decode()
        assert np.array_equal(s.amplitudes(), before)
        # the workspace is still usable after the rejection
        rc = _noalloc(s, start, jq.JQ_COMPACT_PER_GATE, jq.JQ_SEARCH_AUTO)
        assert rc == jq.JQ_OK
        with jq.State(n, "c128") as r:
            r.apply_circuit(start)
            r.apply_circuit(start)
            assert np.array_equal(r.amplitudes(), s.amplitudes())


def test_noalloc_rejects_an_invalid_gate_without_touching_the_state():
    n = 9
    with jq.State(n, "c128") as s:
        s.apply_circuit(W.random_circuit(n, 30, 9))
        before = s.amplitudes()
        rc = _noalloc(s, [("H", (0,), ()), ("CNOT", (3, 3), ())], jq.JQ_COMPACT_PER_GATE, jq.JQ_SEARCH_AUTO)
        assert rc == jq.JQ_EINVAL
        assert np.array_equal(s.amplitudes(), before)

"""GPU parity of the two-byte code in per-block quantisation mode: each fused
pass decodes once, applies its gates in FP64 and encodes once (range pass,
then encode pass).  The oracle runs the same blocks in the same order, taken
from the planner's host-only schedule (jq_plan_schedule), with its own
gate-by-gate FP64 arithmetic.  The GPU multiplies merged gate matrices, so a
code may differ where a value sits within rounding of a code boundary:
codes are compared by mismatch rate, the range to 1e-12 relative, and the
accuracy against the exact state as in the per-gate tests."""
import numpy as np
import pytest

from oracle import core as O
from paper_1805_04708_amd import jq
from paper_1805_04708_amd import workloads as W

pytestmark = pytest.mark.gpu
PER_BLOCK = jq.JQ_COMPACT_PER_BLOCK


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    jq.lib()


def code_diffs(b0, b1, o0, o1):
    d0 = np.abs(b0.astype(int) - o0.astype(int))
    d1 = np.abs(((b1.astype(int) - o1.astype(int)) + 128) % 256 - 128)
    return d0, d1


def oracle_blocks(n, circ, start, fusion=0, search=jq.JQ_SEARCH_AUTO):
    order, blen, fused = jq.plan_schedule(n, "compact", circ, fusion=fusion, compact_mode=PER_BLOCK, search=search)
    st = start.run([circ[i] for i in order], blocks=[int(b) for b in blen])
    return st, fused


def gpu_blocks(n, circ, fusion=0, init=None, codes=None, search=jq.JQ_SEARCH_AUTO):
    with jq.State(n, "compact") as s:
        if init is not None:
            s.init(init)
        if codes is not None:
            s.write_codes(*codes)
        s.apply_circuit(circ, fusion=fusion, compact_mode=PER_BLOCK, search=search)
        b0, b1, rng = s.codes()
        amps = s.amplitudes()
    return b0, b1, rng, amps


@pytest.mark.parametrize("n,fusion", [(8, 0), (10, 0), (12, 2), (12, 3), (13, 0), (16, 0)])
def test_per_block_random_circuit_matches_oracle(n, fusion):
    circ = W.random_circuit(n, 120, seed=500 + n)
    st, fused = oracle_blocks(n, circ, O.CompactState.encode(O.zero_state(n), n), fusion)
    assert fused.any()
    b0, b1, rng, amps = gpu_blocks(n, circ, fusion)
    d0, d1 = code_diffs(b0, b1, st.b0, st.b1)
    assert int(np.sum((d0 != 0) | (d1 != 0))) <= max(2, 0.01 * d0.size)
    exact = O.run(O.zero_state(n), n, circ)
    f_gpu, f_or = O.fidelity(amps, exact), O.fidelity(st.decode(), exact)
    assert 1 - f_gpu <= 2 * (1 - f_or) + 1e-12, (f_gpu, f_or)


@pytest.mark.parametrize("search", [jq.JQ_SEARCH_AUTO, jq.JQ_SEARCH_ON])
@pytest.mark.parametrize("n", [10, 14])
def test_per_block_haar_layers_codes_identical(n, search):
    # Haar U(2) and CZ: no value is placed on a rounding tie on purpose; with
    # the search forced on, the blocks are those a 2^29-amplitude state gets
    circ = W.layered_u2_cz(n, 3 if search == jq.JQ_SEARCH_AUTO else 8, seed=n)
    st, fused = oracle_blocks(n, circ, O.CompactState.encode(O.zero_state(n), n), search=search)
    assert fused.any()
    b0, b1, rng, amps = gpu_blocks(n, circ, search=search)
    d0, d1 = code_diffs(b0, b1, st.b0, st.b1)
    assert np.mean((d0 == 0) & (d1 == 0)) >= 1 - 1e-4
    assert np.allclose(rng, st.rng, rtol=1e-12, atol=0)


def test_per_block_one_block_from_random_codes():
    # a single fused block from identical codes: one decode, five gates, one
    # range, one encode
    n = 12
    rng = np.random.default_rng(9)
    b0 = rng.integers(-127, 127, 1 << n).astype(np.int8)
    b1 = rng.integers(-128, 128, 1 << n).astype(np.int8)
    b0[rng.random(1 << n) < 0.1] = -128
    b1[b0 == -128] = 0
    circ = [("MAT1", (7,), W.haar_u2(rng)), ("H", (1,), ()), ("CZ", (1, 7), ()),
            ("RZ", (3,), (0.7,)), ("MAT1", (1,), W.haar_u2(rng), (9,))]
    r = (0.01, 0.3)
    order, blen, fused = jq.plan_schedule(n, "compact", circ, compact_mode=PER_BLOCK)
    assert list(blen) == [5] and fused[0]
    st = O.CompactState(n, b0.copy(), b1.copy(), *r).run([circ[i] for i in order], blocks=[5])
    g0, g1, grng, _ = gpu_blocks(n, circ, codes=(b0, b1, r))
    assert np.allclose(grng, st.rng, rtol=1e-12, atol=0)
    d0, d1 = code_diffs(g0, g1, st.b0, st.b1)
    assert d0.max() <= 1 and d1.max() <= 1
    assert int(np.sum((d0 != 0) | (d1 != 0))) <= max(2, 1e-3 * d0.size)


def test_per_block_modulus_preserving_blocks_keep_the_range():
    # uniform start, RZ layer and CNOT chain: every block keeps all moduli,
    # so (r0, r1) stays 2^(-N/2) and every modulus code stays -127
    n = 14
    circ = W.rz_cnot_chain(n, 2, seed=8)
    st, fused = oracle_blocks(n, circ, O.CompactState.encode(O.uniform_state(n), n))
    assert fused.any()
    b0, b1, rng, _ = gpu_blocks(n, circ, init=jq.JQ_INIT_UNIFORM)
    assert np.all(b0 == -127) and np.array_equal(b0, st.b0)
    assert rng[0] == rng[1] == 2.0 ** (-n / 2) and np.array_equal(rng, st.rng)
    d1 = np.abs(((b1.astype(int) - st.b1.astype(int)) + 128) % 256 - 128)
    assert d1.max() <= 1 and np.mean(d1 == 0) >= 1 - 1e-3


def test_per_block_is_more_accurate_than_per_gate():
    # fewer quantisation steps: less accumulated code error
    n = 14
    circ = W.layered_u2_cz(n, 4, seed=3)
    exact = O.run(O.zero_state(n), n, circ)
    with jq.State(n, "compact") as s:
        s.apply_circuit(circ)
        f_gate = O.fidelity(s.amplitudes(), exact)
    _, _, _, amps = gpu_blocks(n, circ)
    f_block = O.fidelity(amps, exact)
    assert 1 - f_block < 1 - f_gate, (f_block, f_gate)


def test_per_block_small_state_equals_per_gate():
    # below one tile (N < 8) every block is a single gate
    n = 7
    circ = W.random_circuit(n, 80, seed=77)
    order, blen, fused = jq.plan_schedule(n, "compact", circ, compact_mode=PER_BLOCK)
    assert not fused.any()
    with jq.State(n, "compact") as s:
        s.apply_circuit(circ)
        ref = s.codes()
    b0, b1, rng, _ = gpu_blocks(n, circ)
    assert np.array_equal(b0, ref[0]) and np.array_equal(b1, ref[1]) and np.array_equal(rng, ref[2])

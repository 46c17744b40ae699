"""GPU parity of the batched persistent launch (many small circuits in one
kernel) against the CPU oracle, and batch-vs-alone bitwise equality."""
import math

import numpy as np
import pytest

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


def mixed_circuit(n, gates, rng):
    out = []
    for _ in range(gates):
        q = [int(x) for x in rng.permutation(n)]
        r = rng.random()
        if r < 0.35 or n < 2:
            out.append(("MAT1", (q[0],), W.haar_u2(rng)))
        elif r < 0.5:
            out.append(("CNOT", (q[0], q[1]), ()))
        elif r < 0.65:
            out.append(("CP", (q[0], q[1]), (float(rng.uniform(0, 6)),)))
        elif r < 0.75:
            out.append(("RZ", (q[0],), (float(rng.uniform(0, 6)),)))
        elif r < 0.82:
            out.append(("SWAP", (q[0], q[1]), ()))
        elif r < 0.9 and n >= 3:
            out.append(("TOFFOLI", (q[0], q[1], q[2]), ()))
        elif n >= 2:
            out.append(("MAT1", (q[0],), W.haar_u2(rng), (q[1],)))
    return out


def oracle_state(n, circ):
    return O.run(O.zero_state(n), n, circ)


@pytest.mark.parametrize("enc,tol", [("c128", 1e-12), ("c64", 5e-6)])
@pytest.mark.parametrize("fusion", [0, 1, 2, 3, 4])
def test_batch_matches_oracle(enc, tol, fusion):
    rng = np.random.default_rng(17 + fusion)
    inst = []
    for i in range(120):
        n = int(rng.integers(1, 15))
        inst.append((n, mixed_circuit(n, int(rng.integers(0, 50)), rng)))
    b = jq.Batch(inst, enc, fusion=fusion)
    b.run()
    for i, (n, circ) in enumerate(inst):
        got = b.amplitudes(i)
        ref = oracle_state(n, circ)
        assert O.rel_l2(got, ref) <= tol, (i, n, O.rel_l2(got, ref))
    b.close()


@pytest.mark.parametrize("enc", ["c128", "c64"])
def test_batch_workload_sizes_and_alone_equality(enc):
    # N in 8..16 with the random 100-gate circuits of the small-circuit workload
    inst = W.batch_instances(48, base_seed=900)
    b = jq.Batch(inst, enc)
    b.run()
    first = [b.amplitudes(i) for i in range(len(inst))]
    b.run()  # a second run resets every state and gives identical bits
    for i in range(len(inst)):
        assert np.array_equal(first[i], b.amplitudes(i))
    for i in range(0, len(inst), 6):
        n, circ = inst[i]
        ref = oracle_state(n, circ)
        assert O.rel_l2(first[i], ref) <= (1e-12 if enc == "c128" else 5e-6)
        alone = jq.Batch([inst[i]], enc)
        alone.run()
        assert np.array_equal(alone.amplitudes(i - i), first[i]), i
        alone.close()
    b.close()


@pytest.mark.parametrize("enc,tol", [("c128", 1e-12), ("c64", 5e-6)])
def test_batch_tile_mode_large_states(enc, tol):
    # states too large for LDS (N 13..16) in tile mode (depth 4): the
    # planner's register/lane passes run by one workgroup per circuit (SWAPs
    # included); a circuit with a general two-qubit dense gate falls back to
    # blocks.  Every state against the oracle, and alone against in the
    # batch, bit for bit
    rng = np.random.default_rng(4)
    inst = []
    for i in range(24):
        n = 13 + i % 4
        circ = mixed_circuit(n, 60, rng)
        if i % 6 == 0:
            q, _ = np.linalg.qr(rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4)))
            flat = [float(v) for x in q.ravel() for v in (x.real, x.imag)]
            circ.insert(30, ("MAT2", (1, n - 1), tuple(flat)))
        inst.append((n, circ))
    b = jq.Batch(inst, enc, fusion=4)
    b.run()
    for i, (n, circ) in enumerate(inst):
        got = b.amplitudes(i)
        assert O.rel_l2(got, oracle_state(n, circ)) <= tol, (i, n)
        if i % 5 == 0:
            alone = jq.Batch([inst[i]], enc, fusion=4)
            alone.run()
            assert np.array_equal(alone.amplitudes(0), got), i
            alone.close()
    # the same circuits in block mode agree to rounding
    blk = jq.Batch(inst, enc, fusion=3)
    blk.run()
    for i in range(len(inst)):
        assert O.rel_l2(blk.amplitudes(i), b.amplitudes(i)) <= tol
    blk.close()
    b.close()


def support_growth_circuits(n, rng):
    """Circuits whose passes widen the set of qubits the state may occupy a
    few at a time, with controls, selectors and diagonals on qubits outside
    it (tile mode then visits only part of the later passes' tiles)."""
    low = list(range(10))
    high = list(range(10, n))
    a = [("H", (q,), ()) for q in low]
    # controls and a phase selector on qubits the state does not occupy yet
    a += [("MAT1", (3,), W.haar_u2(rng), (high[-1],)), ("CP", (high[0], 5), (0.7,)), ("RZ", (high[1],), (1.1,))]
    # spread to one high qubit at a time, with dense gates in between
    for k, h in enumerate(high):
        a.append(("CNOT", (low[k % 10], h), ()))
        a.append(("MAT1", (low[(3 * k) % 10],), W.haar_u2(rng)))
        if k % 2:
            a.append(("CP", (h, high[(k + 1) % len(high)]), (0.3 + k,)))
    a += [("MAT1", (h,), W.haar_u2(rng)) for h in high[::2]]
    a += mixed_circuit(n, 30, rng)
    # only the low qubits: one pass, the rest of the state stays exactly zero
    b = [("H", (q,), ()) for q in low] + [("CNOT", (0, 9), ()), ("T", (4,), ())]
    # only diagonals outside the first pass's qubits
    c = [("H", (0,), ()), ("RZ", (high[0],), (0.4,)), ("CP", (high[-1], high[0]), (1.3,)), ("Z", (high[1],), ())]
    return [a, b, c, []]


@pytest.mark.parametrize("enc,tol", [("c128", 1e-12), ("c64", 5e-6)])
def test_batch_tile_mode_support_growth(enc, tol):
    # tile mode skips, in every pass after the first, the tiles with an
    # index bit set outside the qubits of the passes so far (zero before
    # and after the pass): states against the oracle, alone against in the
    # batch bit for bit, and exact zeros outside a one-pass circuit's qubits
    rng = np.random.default_rng(1805)
    inst = []
    for n in (13, 14, 16):
        inst += [(n, c) for c in support_growth_circuits(n, rng)]
    b = jq.Batch(inst, enc, fusion=4)
    b.run()
    for i, (n, circ) in enumerate(inst):
        got = b.amplitudes(i)
        ref = oracle_state(n, circ)
        assert O.rel_l2(got, ref) <= tol, (i, n, O.rel_l2(got, ref))
        alone = jq.Batch([inst[i]], enc, fusion=4)
        alone.run()
        assert np.array_equal(alone.amplitudes(0), got), i
        alone.close()
        if i % 4 == 1:
            outside = np.arange(1 << n) >= (1 << 10)
            assert not np.any(got[outside]), i
        if not circ:
            assert got[0] == 1 and not np.any(got[1:]), i
    b.close()


def test_batch_rejects_bad_input():
    with pytest.raises(jq.JqError):
        jq.Batch([(21, [])], "c128")
    with pytest.raises(jq.JqError):
        jq.Batch([(3, [("H", (3,), ())])], "c128")
    with pytest.raises(jq.JqError):
        jq.Batch([(3, [])], "compact")

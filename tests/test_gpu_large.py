"""GPU checks at the workload sizes: the 30-qubit layered circuit in the
benchmark's launch configuration, the first sizes whose plans use the
planner's large-state steps by default (1 GiB states: N=26 complex128, N=27
complex64, every amplitude against the oracle), and 256 GiB states (N=34
complex128, N=37 two-byte code).  At 30 qubits and above the oracle cannot
hold the state in its test budget, so the checks use outputs it can compute
one by one (product-state amplitudes through its own gate table), the
per-gate kernels (no planner; each checked against the oracle on every
target) and properties that hold at any size (a circuit followed by its
inverse returns |0...0>, norms, closed-form GHZ and uniform states)."""
import math
import threading

import numpy as np
import pytest

from oracle import core as O
from oracle import gates as OG
from paper_1805_04708_amd import jq
from paper_1805_04708_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    jq.lib()


def free_gib():
    import torch
    return torch.cuda.mem_get_info()[0] / 2 ** 30


def inverse(circ):
    """Inverse circuit: reversed order, each explicit matrix conjugate-transposed."""
    out = []
    for g in reversed(circ):
        name, q, p = g[0], g[1], g[2]
        if name == "MAT1":
            m = OG.matrix("MAT1", p).conj().T
            flat = np.empty(8)
            flat[0::2], flat[1::2] = m.real.ravel(), m.imag.ravel()
            out.append(("MAT1", q, tuple(flat)))
        elif name == "CZ":
            out.append(g)
        else:
            raise ValueError(name)
    return out


def chunked_compare(a, b, n, chunk=1 << 24):
    """(||a - b||, ||b||) over two states read back in chunks: a and b are
    states, or a state and a full host array."""
    d2 = r2 = 0.0
    for first in range(0, 1 << n, chunk):
        x = a.amplitudes(first, chunk) if hasattr(a, "amplitudes") else a[first:first + chunk]
        y = b.amplitudes(first, chunk) if hasattr(b, "amplitudes") else b[first:first + chunk]
        d2 += float(np.sum(np.abs(x - y) ** 2))
        r2 += float(np.sum(np.abs(y) ** 2))
    return math.sqrt(d2), math.sqrt(r2)


@pytest.mark.timeout(900)
def test_layered_circuit_at_the_first_searched_sizes_matches_the_oracle():
    # the smallest states on which the planner's large-state steps are on by
    # default (1 GiB: N=26 complex128, N=27 complex64), four layers of the
    # layered workload, every amplitude against the oracle; the oracle runs
    # in threads while the GPU works (its C loops release the interpreter)
    cases = [(26, "c128", 1e-12), (27, "c64", None)]
    circs = {n: W.layered_u2_cz(n, 4, seed=900 + n) for n, _, _ in cases}
    ref = {}

    def oracle(n):
        ref[n] = O.run(O.zero_state(n), n, circs[n])

    threads = {n: threading.Thread(target=oracle, args=(n,)) for n, _, _ in cases}
    for t in threads.values():
        t.start()
    try:
        for n, enc, tol in cases:
            key = lambda st: [(x["reg_q"], x["lane_q"], x["n_gates"]) for x in st]
            assert key(jq.plan_steps(n, enc, circs[n])) == key(jq.plan_steps(n, enc, circs[n],
                                                                               search=jq.JQ_SEARCH_ON))
            with jq.State(n, enc) as s:
                s.apply_circuit(circs[n])
                got = s.amplitudes()
            threads[n].join()
            err = O.rel_l2(got, ref[n])
            limit = tol if tol else 2e-6 * max(1.0, math.sqrt(len(circs[n]) / 100.0))
            print(f"N={n} {enc} {len(circs[n])} gates: rel L2 vs oracle {err:.3e}", flush=True)
            assert err <= limit, (n, enc, err)
            del got
            ref.pop(n)
    finally:
        for t in threads.values():
            t.join()


@pytest.mark.timeout(600)
def test_n30_headline_circuit_fused_equals_per_gate_and_c64_error():
    # the 40-layer headline circuit (1800 gates) at its own size: the fused
    # passes of the searched plan against one kernel per gate (no planner;
    # every per-gate kernel is checked against the oracle on every target),
    # and complex64's error against complex128
    n = 30
    if free_gib() < 41:
        pytest.skip("needs 40 GiB of free HBM")
    circ = W.layered_u2_cz(n, 40, seed=2018)
    with jq.State(n, "c128") as fused:
        fused.apply_circuit(circ)
        with jq.State(n, "c128") as single:
            single.apply_circuit(circ, fusion=1)
            d, r = chunked_compare(fused, single, n)
        print(f"N=30 fused vs per gate: rel L2 {d / r:.3e}", flush=True)
        assert d / r <= 1e-12, d / r
        with jq.State(n, "c64") as low:
            low.apply_circuit(circ)
            d64, _ = chunked_compare(low, fused, n)
        print(f"N=30 complex64 vs complex128: rel L2 {d64 / r:.3e}", flush=True)
        assert d64 / r <= 2e-6 * math.sqrt(len(circ) / 100.0), d64 / r
        assert abs(fused.norm() - 1.0) < 1e-12


def test_n30_c64_rz_cnot_chain_closed_form():
    # 20 layers of RZ and the CNOT chain from the uniform state in
    # complex64 (one-qubit diagonals on register qubits run as FP32 tables):
    # each amplitude is 2^-15 times the product of the RZ entries met along
    # its source index's path, to FP32 rounding
    n = 30
    circ = W.rz_cnot_chain(n, 20, seed=30)
    with jq.State(n, "c64") as s:
        s.init(jq.JQ_INIT_UNIFORM)
        s.apply_circuit(circ)
        src = np.random.default_rng(301).integers(0, 1 << n, 48)
        worst = 0.0
        for j in [int(x) for x in src] + [0, (1 << n) - 1, (1 << 29) | 4321]:
            i, amp = j, complex(2.0 ** (-n / 2))
            for name, q, p in circ:
                if name == "RZ":
                    amp *= OG.matrix("RZ", p)[(i >> q[0]) & 1, (i >> q[0]) & 1]
                elif (i >> q[0]) & 1:
                    i ^= 1 << q[1]
            got = s.amplitudes(i, 1)[0]
            worst = max(worst, abs(got - amp) / abs(amp))
        assert worst < 1e-5, worst
        assert abs(s.norm() - 1.0) < 1e-5


def test_n30_layer_amplitudes_one_by_one():
    # one layer from |0...0>: a product state times the CZ signs, so every
    # amplitude is prod_q U_q[b_q, 0] * (-1)^(sum over CZ pairs b_a b_b)
    n = 30
    circ = W.layered_u2_cz(n, 1, seed=2018)
    us = {g[1][0]: OG.matrix("MAT1", g[2]) for g in circ if g[0] == "MAT1"}
    pairs = [g[1] for g in circ if g[0] == "CZ"]
    rng = np.random.default_rng(1)
    samples = [0, (1 << n) - 1] + [int(x) for x in rng.integers(0, 1 << n, 200)]
    with jq.State(n, "c128") as s:
        s.apply_circuit(circ)
        for i in samples:
            bits = [(i >> q) & 1 for q in range(n)]
            ref = 1.0 + 0j
            for q in range(n):
                ref *= us[q][bits[q], 0]
            for a, b in pairs:
                if bits[a] and bits[b]:
                    ref = -ref
            got = s.amplitudes(i, 1)[0]
            assert abs(got - ref) <= 1e-12 * max(abs(ref), 2.0 ** (-n / 2)), (i, got, ref)
        assert abs(s.norm() - 1.0) < 1e-12


@pytest.mark.parametrize("enc,tol", [("c128", 1e-11), ("c64", 2e-4)])
def test_n30_circuit_then_inverse_returns_to_zero_state(enc, tol):
    n, layers = 30, 6
    circ = W.layered_u2_cz(n, layers, seed=7)
    with jq.State(n, enc) as s:
        s.apply_circuit(circ)
        mid = s.norm()
        s.apply_circuit(inverse(circ))
        a0 = s.amplitudes(0, 1)[0]
        assert abs(mid - 1.0) < tol
        assert abs(a0 - 1.0) < tol, a0
        p = s.probabilities([0, n - 1])
        assert abs(p[0] - 1.0) < tol


def test_n34_c128_uniform_and_ghz():
    n = 34
    if free_gib() < 257:
        pytest.skip("needs 256 GiB of free HBM")
    with jq.State(n, "c128") as s:
        s.apply_circuit(W.hadamard_all(n))
        amp = 2.0 ** (-n / 2)
        for i in [0, 1, (1 << n) - 1, 123456789]:
            assert abs(s.amplitudes(i, 1)[0] - amp) < 1e-15
        assert abs(s.norm() - 1.0) < 1e-12
        assert np.allclose(s.probabilities([n - 1]), [0.5, 0.5], atol=1e-12)
        s.init(jq.JQ_INIT_ZERO)
        s.apply_circuit(W.ghz(n))
        h = 1 / math.sqrt(2)
        assert abs(s.amplitudes(0, 1)[0] - h) < 1e-15
        assert abs(s.amplitudes((1 << n) - 1, 1)[0] - h) < 1e-15
        assert s.amplitudes(1 << 20, 1)[0] == 0
        assert np.allclose(s.probabilities([0, 17, n - 1]), [0.5, 0, 0, 0, 0, 0, 0, 0.5], atol=1e-12)


def test_n34_c128_twenty_rz_cnot_layers():
    # the 34-qubit complex128 workload: 20 layers of RZ and the CNOT chain
    # from the uniform state; every amplitude is 2^(-17) times the product
    # of the RZ entries met along its source index's path through the
    # circuit (each CNOT moves the index)
    n = 34
    if free_gib() < 257:
        pytest.skip("needs 256 GiB of free HBM")
    circ = W.rz_cnot_chain(n, 20, seed=34)
    with jq.State(n, "c128") as s:
        s.init(jq.JQ_INIT_UNIFORM)
        s.apply_circuit(circ)
        assert abs(s.norm() - 1.0) < 1e-12
        src = np.random.default_rng(341).integers(0, 1 << n, 32)
        for j in [int(x) for x in src] + [0, (1 << n) - 1, (1 << 33) | 777]:
            i, amp = j, complex(2.0 ** (-n / 2))
            for name, q, p in circ:
                if name == "RZ":
                    amp *= OG.matrix("RZ", p)[(i >> q[0]) & 1, (i >> q[0]) & 1]
                elif (i >> q[0]) & 1:
                    i ^= 1 << q[1]
            got = s.amplitudes(i, 1)[0]
            assert abs(got - amp) < 1e-12 * abs(amp), (j, i, got, amp)


def test_n37_two_byte_code_ghz_and_phases():
    n = 37
    if free_gib() < 257:
        pytest.skip("needs 256 GiB of free HBM")
    with jq.State(n, "compact") as s:
        s.apply_circuit(W.ghz(n))
        h = 1 / math.sqrt(2)
        a = s.amplitudes(0, 1)[0], s.amplitudes((1 << n) - 1, 1)[0]
        assert abs(a[0] - h) < 1e-15 and abs(a[1] - h) < 1e-15
        b0, b1, rng = s.codes((1 << n) - 4, 4)
        assert list(b0) == [-128, -128, -128, -127] and rng[0] == rng[1]
        assert abs(s.norm() - 1.0) < 1e-14
        # uniform state, 20 layers of RZ and the CNOT chain (the 37-qubit
        # two-byte workload): moduli never change
        s.init(jq.JQ_INIT_UNIFORM)
        circ = W.rz_cnot_chain(n, 20, seed=5)
        s.apply_circuit(circ)
        b0, b1, rng = s.codes(0, 1 << 12)
        assert np.all(b0 == -127) and abs(rng[0] - 2.0 ** (-n / 2)) < 1e-30
        assert abs(s.norm() - 1.0) < 1e-13
        # phase codes one by one, all over the index range (tiles whose base
        # has bit 31 and above set): follow a source index through the
        # circuit; each RZ adds its entry's phase in code units, 128 arg / pi
        # rounded, mod 256 (a phase of 0 to start), each CNOT moves the index
        src = np.random.default_rng(371).integers(0, 1 << n, 48)
        for j in [int(x) for x in src] + [(1 << n) - 1, 1 << 31, (1 << 36) | 12345]:
            i, code = j, 0
            for name, q, p in circ:
                if name == "RZ":
                    e = OG.matrix("RZ", p)[(i >> q[0]) & 1, (i >> q[0]) & 1]
                    code = ((code + int(np.rint(128 * np.angle(e) / math.pi)) + 128) & 255) - 128
                elif (i >> q[0]) & 1:
                    i ^= 1 << q[1]
            c0, c1, _ = s.codes(i, 1)
            assert int(c0[0]) == -127 and int(c1[0]) == code, (j, i)
        # sampling at 2^37 amplitudes (the block sums loop over their blocks):
        # every probability is the same rounded value of 2^-37, so the event
        # is floor(u 2^37) up to the rounding of the cumulative sums
        u = np.random.default_rng(37).random(4096)
        got = s.sample(u).astype(np.int64)
        assert np.max(np.abs(got - np.floor(u * 2.0 ** n).astype(np.int64))) <= 1


def test_n34_per_gate_kernels_on_the_full_grid():
    # unfused gates at 2^34 amplitudes: the per-gate kernels loop over chunks
    # of a capped grid (a launch holds at most 2^32 threads)
    n = 34
    if free_gib() < 257:
        pytest.skip("needs 256 GiB of free HBM")
    with jq.State(n, "c128") as s:
        s.init(jq.JQ_INIT_UNIFORM)
        theta, phi, psi = 0.8, 0.3, 1.1
        m2 = np.linalg.qr(np.random.default_rng(34).normal(size=(4, 4))
                          + 1j * np.random.default_rng(35).normal(size=(4, 4)))[0]
        flat = np.empty(32)
        flat[0::2], flat[1::2] = m2.real.ravel(), m2.imag.ravel()
        # qubits 0-2 take the lane-exchange kernels (dense, X and the
        # two-qubit gate on (1, 3)), whose capped grids loop over the 2^26
        # chunks of 256 amplitudes (2^25 of 256 pairs)
        s.apply_circuit([("RZ", (5,), (theta,)), ("CNOT", (3, 33), ()), ("H", (7,), ()),
                         ("RZ", (1,), (phi,)), ("X", (1,), ()), ("RZ", (2,), (psi,)), ("H", (2,), ()),
                         ("H", (0,), ()), ("MAT2", (1, 3), tuple(flat))], fusion=1)
        amp = 2.0 ** (-n / 2)
        r2 = math.sqrt(2)
        f1 = [np.exp(0.5j * phi), np.exp(-0.5j * phi)]  # qubit 1 after RZ and X
        for i in [0, 1 << 5, 2, 4, 6, 0b100110, (1 << n) - 1, (1 << n) - 1 - 0b10000001, 987654321, 987654320]:
            b = [(i >> q) & 1 for q in range(8)]
            # the state stays a product over qubits: CNOT(3, 33) leaves a
            # state uniform in both of its qubits unchanged
            want = amp
            want *= np.exp(0.5j * theta) if b[5] else np.exp(-0.5j * theta)
            want *= 0.0 if b[7] else r2  # H on a uniform qubit
            want *= 0.0 if b[0] else r2
            want *= -1j * r2 * math.sin(psi / 2) if b[2] else r2 * math.cos(psi / 2)
            # the two-qubit gate on (1, 3) (qubit 1 the row's most significant
            # bit) mixes qubit 1's phases, qubit 3 still uniform
            want *= sum(m2[2 * b[1] + ((i >> 3) & 1), c] * f1[c >> 1] for c in range(4))
            assert abs(s.amplitudes(i, 1)[0] - want) < 1e-15, i
        assert abs(s.norm() - 1.0) < 1e-12


@pytest.mark.parametrize("enc,tol", [("c128", 1e-15), ("c64", 2e-7)])
def test_n30_two_qubit_gates_on_low_qubits_closed_form(enc, tol):
    # two-qubit dense gates on disjoint pairs of a uniform 30-qubit state,
    # whose lower qubit lies inside a 128-byte line (the lane-exchange kernel
    # for complex128 pairs (0, 1) and (5, 2), complex64 also (4, 3)): the
    # state stays a product over the pairs, each amplitude the uniform
    # amplitude times one row sum of each matrix
    n = 30
    if free_gib() < 17:
        pytest.skip("needs 16 GiB of free HBM")
    rng = np.random.default_rng(30)
    pairs = [(0, 1), (5, 2), (4, 3), (20, 9)]
    mats = []
    for _ in pairs:
        q, _r = np.linalg.qr(rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4)))
        mats.append(q)
    circ = []
    for (a, b), m in zip(pairs, mats):
        flat = np.empty(32)
        flat[0::2], flat[1::2] = m.real.ravel(), m.imag.ravel()
        circ.append(("MAT2", (a, b), tuple(flat)))
    amp = 2.0 ** (-n / 2)
    with jq.State(n, enc) as s:
        s.init(jq.JQ_INIT_UNIFORM)
        s.apply_circuit(circ, fusion=1)
        idx = [0, 1, 2, 3, 0b111111, (1 << n) - 1, 987654321] + [int(x) for x in rng.integers(0, 1 << n, 40)]
        for i in idx:
            want, scale = amp, amp
            for (a, b), m in zip(pairs, mats):
                # the first-listed qubit is the most significant bit of the row
                row = m[2 * ((i >> a) & 1) + ((i >> b) & 1)]
                want *= row.sum()
                scale *= np.abs(row).sum()
            # each gate's rounding is relative to its terms, not its sum
            assert abs(s.amplitudes(i, 1)[0] - want) <= 8 * len(pairs) * tol * scale, (i, enc)
        assert abs(s.norm() - 1.0) < (1e-12 if enc == "c128" else 1e-5)

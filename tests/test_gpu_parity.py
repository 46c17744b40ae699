"""GPU parity: the HIP path against the CPU oracle, through the C ABI.

Tolerances
* complex128: relative L2 <= 1e-12 (the target stated for the method);
* complex64: relative L2 <= 2e-6 per 100 gates (FP32 rounding, ~sqrt(G) * 2^-24
  growth with margin);
* reductions: absolute 1e-12 (c128) in FP64.
"""
import math

import numpy as np
import pytest

from oracle import core as O
from oracle import gates as OG
from paper_1805_04708_amd import jq
from paper_1805_04708_amd import workloads as W

pytestmark = pytest.mark.gpu


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")
    jq.lib()


TOL = {"c128": 1e-12, "c64": 2e-6}


def run_gpu(n, enc, circuit, fusion=0, init=None, search=jq.JQ_SEARCH_AUTO):
    with jq.State(n, enc) as s:
        if isinstance(init, np.ndarray):
            s.write_amplitudes(init)
        elif isinstance(init, int):
            s.init(jq.JQ_INIT_BASIS, init)
        elif init == "uniform":
            s.init(jq.JQ_INIT_UNIFORM)
        if circuit:
            s.apply_circuit(circuit, fusion=fusion, search=search)
        return s.amplitudes()


# The planner's large-state steps (tile-slot search, register/lane split,
# lane order) are on by default only for states of 1 GiB or more; the fused
# tests below also run them forced on, so the plans the 30-qubit workloads
# get are checked against the oracle at sizes it finishes in seconds.
SEARCH = [jq.JQ_SEARCH_AUTO, jq.JQ_SEARCH_ON]


def run_oracle(n, circuit, init=None):
    if isinstance(init, np.ndarray):
        psi = init.astype(np.complex128).copy()
    elif isinstance(init, int):
        psi = O.basis_state(n, init)
    elif init == "uniform":
        psi = O.uniform_state(n)
    else:
        psi = O.zero_state(n)
    return O.run(psi, n, circuit)


def rand_state(rng, n):
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return psi / np.linalg.norm(psi)


def tol(enc, gates=1):
    return TOL[enc] * (1 if enc == "c128" else max(1.0, math.sqrt(gates / 100.0)))


# --------------------------------------------------------------- init --

@pytest.mark.parametrize("enc", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 5, 12])
def test_init_modes(enc, n):
    assert np.array_equal(run_gpu(n, enc, []), O.zero_state(n))
    u = run_gpu(n, enc, [], init="uniform")
    ref = 2.0 ** (-n / 2)
    assert np.max(np.abs(u - ref)) <= (1e-7 if enc == "c64" else 0.0) * ref
    b = run_gpu(n, enc, [], init=(1 << n) - 1)
    assert np.array_equal(b, O.basis_state(n, (1 << n) - 1))


# ---------------------------------------------------- per-gate kernels --

def single_gate_cases(n, rng):
    """Every target, with controls below, above and between, for each class."""
    cases = []
    for t in range(n):
        u = W.haar_u2(rng)
        cases.append(("MAT1", (t,), u))
        cases.append(("RZ", (t,), (float(rng.uniform(0, 6.28)),)))
        cases.append(("T", (t,), ()))
        cases.append(("X", (t,), ()))
        others = [q for q in range(n) if q != t]
        if others:
            c = int(rng.choice(others))
            cases.append(("CNOT", (c, t), ()))
            cases.append(("CP", (c, t), (float(rng.uniform(0, 6.28)),)))
            cases.append(("MAT1", (t,), W.haar_u2(rng), (c,)))
            cases.append(("SWAP", (t, c), ()))
            m2 = np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))[0]
            flat = np.empty(32)
            flat[0::2], flat[1::2] = m2.real.ravel(), m2.imag.ravel()
            cases.append(("MAT2", (c, t), tuple(flat)))
            cases.append(("RZ", (t,), (0.4,), (c,)))
        if len(others) >= 2:
            c1, c2 = (int(x) for x in rng.choice(others, 2, replace=False))
            cases.append(("TOFFOLI", (c1, c2, t), ()))
            cases.append(("MAT1", (t,), W.haar_u2(rng), (c1, c2)))
    return cases


@pytest.mark.parametrize("enc", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 2, 3, 6, 7, 8, 11, 14])
def test_every_gate_class_every_target(enc, n):
    # N = 8 is the smallest state whose uncontrolled gates on targets 0-2 run
    # the lane-exchange kernel (one chunk of 256 amplitudes); below it they
    # run the pair kernel
    rng = np.random.default_rng(1000 + n)
    psi0 = rand_state(rng, n)
    for g in single_gate_cases(n, rng):
        got = run_gpu(n, enc, [g], fusion=1, init=psi0)
        ref = run_oracle(n, [g], init=psi0)
        assert O.rel_l2(got, ref) <= tol(enc), (enc, n, g[:2], O.rel_l2(got, ref))


@pytest.mark.parametrize("enc", ["c128", "c64"])
def test_reduced_kind_circuit_at_the_default_width(enc):
    # uncontrolled one-qubit dense gates and controlled Zs (with up to two
    # more controls) plan at the default width (2^5 register slots for
    # complex128, 2^6 for complex64) and run the reduced op loop, negations
    # with register and thread controls included
    n = 14
    rng = np.random.default_rng(31)
    circ = []
    for _ in range(6):
        circ += [("MAT1", (q,), W.haar_u2(rng)) for q in range(n)]
        for _ in range(5):
            a, b, c, d = (int(x) for x in rng.permutation(n)[:4])
            k = int(rng.integers(0, 3))
            circ.append(("CZ", (a, b), (), (c, d)[:k]) if k else ("CZ", (a, b), ()))
    k_want = 6 if enc == "c64" else 5
    assert {st["k_reg"] for st in jq.plan_steps(n, enc, circ) if st["fused"]} == {k_want}
    psi0 = rand_state(rng, n)
    got = run_gpu(n, enc, circ, init=psi0)
    ref = run_oracle(n, circ, init=psi0)
    assert O.rel_l2(got, ref) <= tol(enc, len(circ)), O.rel_l2(got, ref)


@pytest.mark.parametrize("enc", ["c128", "c64"])
@pytest.mark.parametrize("n", [8, 9, 12])
def test_two_qubit_dense_gates_on_low_qubits(enc, n):
    # every ordered pair with a qubit below 4: from N = 9 up the uncontrolled
    # ones whose lower qubit lies inside a 128-byte line (below 3 for
    # complex128, 4 for complex64) run the lane-exchange kernel (whole chunks
    # of 256 pairs), the others and all at N = 8 the four-amplitude kernel;
    # controlled ones always run the latter
    rng = np.random.default_rng(700 + n)
    psi0 = rand_state(rng, n)
    circ = []
    for a in range(n):
        for b in range(n):
            if a != b and min(a, b) < 4:
                circ.append(("MAT2", (a, b), random_u4(rng)))
    got = run_gpu(n, enc, circ, fusion=1, init=psi0)
    ref = run_oracle(n, circ, init=psi0)
    assert O.rel_l2(got, ref) <= tol(enc, len(circ)), O.rel_l2(got, ref)
    ctrl = [("MAT2", (0, 1), random_u4(rng), (5,)), ("MAT2", (2, 0), random_u4(rng), (4, 7))]
    got = run_gpu(n, enc, ctrl, fusion=1, init=psi0)
    ref = run_oracle(n, ctrl, init=psi0)
    assert O.rel_l2(got, ref) <= tol(enc, len(ctrl)), O.rel_l2(got, ref)


@pytest.mark.parametrize("enc", ["c128", "c64"])
def test_apply_gate_entry_point(enc):
    n = 9
    rng = np.random.default_rng(5)
    psi0 = rand_state(rng, n)
    u = OG.matrix("MAT1", W.haar_u2(rng))
    with jq.State(n, enc) as s:
        s.write_amplitudes(psi0)
        s.apply_gate(jq.JQ_DENSE, [4], [7], u)
        s.apply_gate(jq.JQ_DIAGONAL, [2, 6], [], np.array([1, 1j, -1, np.exp(0.3j)]))
        s.apply_gate(jq.JQ_PERM_X, [0], [3, 5])
        got = s.amplitudes()
    ref = O.apply(psi0.copy(), n, [4], [7], u)
    ref = O.apply(ref, n, [2, 6], [], np.diag([1, 1j, -1, np.exp(0.3j)]))
    ref = O.apply(ref, n, [0], [3, 5], OG.matrix("X"))
    assert O.rel_l2(got, ref) <= tol(enc)


def test_invalid_gates_leave_state_untouched():
    n = 5
    with jq.State(n, "c128") as s:
        s.init(jq.JQ_INIT_UNIFORM)
        before = s.amplitudes()
        for bad in ([("H", (5,), ())], [("CNOT", (1, 1), ())], [("H", (0,), ()), ("X", (9,), ())]):
            with pytest.raises(jq.JqError) as e:
                s.apply_circuit(bad)
            assert e.value.code == jq.JQ_EINVAL
        with pytest.raises(jq.JqError):
            s.apply_gate(jq.JQ_DIAGONAL, [0], [], None)
        nan = np.array([[np.nan, 0], [0, 1]])
        with pytest.raises(jq.JqError):
            s.apply_gate(jq.JQ_DENSE, [0], [], nan)
        assert np.array_equal(s.amplitudes(), before)


# --------------------------------------------------------- circuits --

def random_u4(rng):
    q, _ = np.linalg.qr(rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4)))
    flat = []
    for x in q.ravel():
        flat += [float(x.real), float(x.imag)]
    return tuple(flat)


@pytest.mark.parametrize("search", SEARCH)
@pytest.mark.parametrize("enc", ["c128", "c64"])
@pytest.mark.parametrize("fusion", [0, 2, 3, 4, 5])
def test_swap_in_fused_passes(enc, fusion, search):
    # SWAPs (some controlled) run inside passes as three controlled X ops,
    # with diagonal gates on their qubits before and after (which must not
    # move past them) and a general two-qubit gate that stays unfused
    n = 13
    rng = np.random.default_rng(100 + fusion)
    circ = [("H", (q,), ()) for q in range(n)]
    for _ in range(60):
        a, b, c = (int(x) for x in rng.permutation(n)[:3])
        circ += [("CP", (a, c), (float(rng.uniform(-3, 3)),)), ("RZ", (b,), (float(rng.uniform(0, 6)),)),
                 ("SWAP", (a, b), ()) if rng.random() < 0.7 else ("SWAP", (a, b), (), (c,)),
                 ("T", (a,), ()), ("CZ", (b, c), ()), ("MAT1", (a,), W.haar_u2(rng))]
        if rng.random() < 0.1:
            circ.append(("MAT2", (a, c), random_u4(rng)))
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    got = run_gpu(n, enc, circ, fusion=fusion, init=psi0, search=search)
    ref = run_oracle(n, circ, init=psi0)
    assert O.rel_l2(got, ref) <= tol(enc, len(circ)), O.rel_l2(got, ref)


@pytest.mark.parametrize("enc", ["c128", "c64"])
def test_per_gate_kernel_variants_19_qubits(enc):
    # one kernel per gate on a random 19-qubit state: dense and X targets
    # below and above qubit 17 (one or four pairs per thread), controls
    # inside a 128-byte line (plain accesses) and above it (streaming),
    # diagonals with low and high bits, a Toffoli and a controlled dense gate
    n = 19
    rng = np.random.default_rng(19)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    circ = []
    for t in (0, 2, 3, 9, 16, 17, 18):
        circ.append(("MAT1", (t,), W.haar_u2(rng)))
        circ.append(("X", (t,), ()))
    circ += [("CNOT", (0, 18), ()), ("CNOT", (1, 17), ()), ("CNOT", (5, 18), ()), ("CNOT", (18, 3), ()),
             ("MAT1", (17,), W.haar_u2(rng), (2,)), ("MAT1", (18,), W.haar_u2(rng), (12,)),
             ("MAT1", (4,), W.haar_u2(rng), (0, 1)), ("TOFFOLI", (1, 2, 18), ()), ("TOFFOLI", (10, 11, 17), ()),
             ("CZ", (0, 1), ()), ("CZ", (2, 3), ()), ("CZ", (5, 6), ()), ("CZ", (17, 18), ()),
             ("CP", (0, 18), (0.7,)), ("RZ", (1,), (1.1,)), ("RZ", (18,), (2.3,)), ("T", (0,), ()),
             ("S", (17,), ())]
    got = run_gpu(n, enc, circ, fusion=1, init=psi0)
    ref = run_oracle(n, circ, init=psi0)
    assert O.rel_l2(got, ref) <= tol(enc, len(circ)), O.rel_l2(got, ref)


@pytest.mark.parametrize("enc", ["c128", "c64"])
def test_per_gate_access_orders_20_qubits(enc):
    # one kernel per gate, controls on the index bits that change the
    # kernels' access order: byte-address bits 10 and 20 (qubits 6 and 16
    # for complex128, 7 and 17 for complex64: the chunks are dealt out in 64
    # interleaved streams) and bits inside a 128-byte line (qubit 0 fixed:
    # the whole state read and written; other low qubits: one thread per
    # index), with selectors and phases on diagonals
    n = 20
    rng = np.random.default_rng(20)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    circ = []
    for a, b in ((5, 6), (6, 7), (7, 8), (15, 16), (16, 17), (17, 18), (0, 1), (1, 2), (2, 3), (3, 4), (0, 19), (8, 9)):
        circ += [("CZ", (a, b), ()), ("CP", (b, a), (float(rng.uniform(0, 6.28)),))]
    circ += [("CNOT", (6, 10), ()), ("CNOT", (16, 3), ()), ("CNOT", (7, 1), ()), ("CNOT", (17, 19), ()),
             ("MAT1", (4,), W.haar_u2(rng), (16,)), ("MAT1", (12,), W.haar_u2(rng), (7,)),
             ("MAT1", (18,), W.haar_u2(rng), (6, 16)), ("TOFFOLI", (6, 16, 2), ()),
             ("RZ", (5,), (0.3,), (0,)), ("RZ", (9,), (1.3,), (1, 3)), ("RZ", (0,), (2.1,), (6,)),
             ("U", (2, 11), (3,), (0,)), ("T", (17,), (), (16,)), ("S", (3,), (), (2,))]
    got = run_gpu(n, enc, circ, fusion=1, init=psi0)
    ref = run_oracle(n, circ, init=psi0)
    assert O.rel_l2(got, ref) <= tol(enc, len(circ)), O.rel_l2(got, ref)


@pytest.mark.parametrize("enc", ["c128", "c64"])
@pytest.mark.parametrize("fusion", [1, 0])
def test_random_circuit_16_qubits(enc, fusion):
    # the 16-qubit, 200-gate random circuit workload
    n = 16
    circ = W.random_circuit(n, 200, seed=7)
    got = run_gpu(n, enc, circ, fusion=fusion)
    ref = run_oracle(n, circ)
    assert O.rel_l2(got, ref) <= tol(enc, 200), O.rel_l2(got, ref)


@pytest.mark.parametrize("search", SEARCH)
@pytest.mark.parametrize("enc", ["c128", "c64"])
@pytest.mark.parametrize("n,fusion", [(10, 0), (13, 0), (17, 0), (17, 3), (18, 2), (19, 5), (20, 6)])
def test_layered_circuit_fused(enc, n, fusion, search):
    if enc == "c128" and fusion > 5:
        pytest.skip()
    circ = W.layered_u2_cz(n, 3 if search == jq.JQ_SEARCH_AUTO else 8, seed=n)
    got = run_gpu(n, enc, circ, fusion=fusion, search=search)
    ref = run_oracle(n, circ)
    assert O.rel_l2(got, ref) <= tol(enc, len(circ)), O.rel_l2(got, ref)


@pytest.mark.parametrize("search", SEARCH)
@pytest.mark.parametrize("enc", ["c128", "c64"])
def test_fused_mixed_gates_with_controls(enc, search):
    n = 15
    rng = np.random.default_rng(9)
    circ = []
    for _ in range(300):
        q = [int(x) for x in rng.permutation(n)]
        r = rng.random()
        if r < 0.3:
            circ.append(("MAT1", (q[0],), W.haar_u2(rng)))
        elif r < 0.4:
            circ.append(("MAT1", (q[0],), W.haar_u2(rng), (q[1],)))
        elif r < 0.55:
            circ.append(("CNOT", (q[0], q[1]), ()))
        elif r < 0.65:
            circ.append(("TOFFOLI", (q[0], q[1], q[2]), ()))
        elif r < 0.8:
            circ.append(("CP", (q[0], q[1]), (float(rng.uniform(0, 6)),)))
        elif r < 0.9:
            circ.append(("RZ", (q[0],), (float(rng.uniform(0, 6)),)))
        else:
            circ.append(("Y", (q[0],), ()))
    psi0 = rand_state(rng, n)
    ref = run_oracle(n, circ, init=psi0)
    for fusion in (0, 2, 3, 4):
        got = run_gpu(n, enc, circ, fusion=fusion, init=psi0, search=search)
        assert O.rel_l2(got, ref) <= tol(enc, 300), (fusion, O.rel_l2(got, ref))


@pytest.mark.parametrize("search", SEARCH)
@pytest.mark.parametrize("enc", ["c128", "c64"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fused_diagonal_folding(enc, seed, search):
    # dense gates surrounded by runs of diagonal gates on their qubits: the
    # planner folds up to two selector qubits into each dense gate
    n = 14
    rng = np.random.default_rng(300 + seed)
    circ = []
    for _ in range(120):
        t = int(rng.integers(n))
        for _ in range(int(rng.integers(0, 4))):
            o = int(rng.choice([q for q in range(n) if q != t]))
            r = rng.random()
            if r < 0.4:
                circ.append(("CZ", (o, t), ()))
            elif r < 0.7:
                circ.append(("CP", (t, o), (float(rng.uniform(0, 6)),)))
            elif r < 0.85:
                circ.append(("RZ", (t,), (float(rng.uniform(0, 6)),)))
            else:
                circ.append(("U", (o, t), (int(rng.integers(-5, 6)),)))
        circ.append(("MAT1", (t,), W.haar_u2(rng)))
    psi0 = rand_state(rng, n)
    ref = run_oracle(n, circ, init=psi0)
    for fusion in (0, 2, 3):
        got = run_gpu(n, enc, circ, fusion=fusion, init=psi0, search=search)
        assert O.rel_l2(got, ref) <= tol(enc, len(circ)), (fusion, O.rel_l2(got, ref))


@pytest.mark.parametrize("n", [4, 9, 12])
def test_closed_forms_on_gpu(n):
    u = run_gpu(n, "c128", W.hadamard_all(n))
    assert np.max(np.abs(u - 2.0 ** (-n / 2))) < 1e-15
    g = run_gpu(n, "c128", W.ghz(n))
    ref = np.zeros(1 << n, dtype=complex)
    ref[0] = ref[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(g - ref)) < 1e-15
    x = 5 % (1 << n)
    q = run_gpu(n, "c128", W.qft(n), init=x)
    k = np.arange(1 << n)
    assert np.max(np.abs(q - 2.0 ** (-n / 2) * np.exp(2j * np.pi * x * k / 2 ** n))) < 1e-13


# -------------------------------------------------------- reductions --

@pytest.mark.parametrize("enc", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 3, 8, 15])
def test_norm_probabilities_expectations(enc, n):
    rng = np.random.default_rng(n)
    circ = W.random_circuit(n, 40, seed=n)
    ref = run_oracle(n, circ)
    t = 1e-12 if enc == "c128" else 2e-6
    with jq.State(n, enc) as s:
        s.apply_circuit(circ)
        got = s.amplitudes()
        assert abs(s.norm() - O.norm2(got, n)) < 1e-12
        assert abs(s.norm() - 1.0) < t
        sets = [[], [0], [n - 1], list(range(n))[::-1]]
        if n >= 3:
            sets += [[1, 0], [n - 1, 0, 1]]
        if n >= 8:
            sets += [[7, 2, 5, 0, 6, 1, 4, 3][: min(n, 8)], [0, 1, 2, 3, 4, 5, 6, 7]]
        for qs in sets:
            p = s.probabilities(qs)
            assert np.max(np.abs(p - O.probabilities(ref, n, qs))) < t, qs
            # repeated calls give identical bits (fixed summation order)
            assert np.array_equal(p, s.probabilities(qs))
        ex = s.expectations()
        er = O.expect_q(ref, n)
        for a, b in zip(ex, er):
            assert np.max(np.abs(a - b)) < t
        s.apply_gate(jq.JQ_DIAGONAL, [0], [], np.array([2.0, 2.0]))
        assert abs(s.norm() - 4.0) < 4 * t
        s.renormalize()
        assert abs(s.norm() - 1.0) < t


def test_probabilities_argument_errors():
    with jq.State(4, "c128") as s:
        for bad in ([4], [0, 0], [-1]):
            with pytest.raises(jq.JqError):
                s.probabilities(bad)


# ------------------------------------------- the two-byte code (Sec. 4.1) --

def compact_compare(n, circ, init=None):
    """GPU two-byte code vs the oracle's, gate by gate quantisation."""
    if init == "uniform":
        st = O.CompactState.encode(O.uniform_state(n), n)
    else:
        st = O.CompactState.encode(O.zero_state(n), n)
    st.run(circ)
    with jq.State(n, "compact") as s:
        if init == "uniform":
            s.init(jq.JQ_INIT_UNIFORM)
        s.apply_circuit(circ)
        b0, b1, rng = s.codes()
        amps = s.amplitudes()
    return st, b0, b1, rng, amps


def code_diffs(b0, b1, o0, o1):
    d0 = np.abs(b0.astype(int) - o0.astype(int))
    d1 = np.abs(((b1.astype(int) - o1.astype(int)) + 128) % 256 - 128)
    return d0, d1


def random_codes(rng, n, zero_frac=0.1):
    b0 = rng.integers(-127, 127, 1 << n).astype(np.int8)
    b1 = rng.integers(-128, 128, 1 << n).astype(np.int8)
    b0[rng.random(1 << n) < zero_frac] = -128
    b1[b0 == -128] = 0
    return b0, b1


def one_gate_cases(n, rng):
    t, c, c2 = (int(x) for x in rng.permutation(n)[:3])
    return [("MAT1", (t,), W.haar_u2(rng)), ("H", (t,), ()), ("+X", (t,), ()),
            ("MAT1", (t,), W.haar_u2(rng), (c,)), ("RZ", (t,), (float(rng.uniform(0, 6.28)),)),
            ("T", (t,), ()), ("CP", (c, t), (float(rng.uniform(0, 6.28)),)), ("CZ", (c, t), ()),
            ("X", (t,), ()), ("CNOT", (c, t), ()), ("TOFFOLI", (c, c2, t), ()),
            ("SWAP", (c, t), ()), ("MAT1", (t,), (2.0, 0, 0, 0, 0, 0, 0.5, 0))]


@pytest.mark.parametrize("n", [3, 9, 14])
def test_compact_single_gate_step_matches_oracle(n):
    # one quantisation step from identical codes: decode, apply, new range,
    # encode.  Codes may differ only where the value sits on a rounding tie
    # and the two atan2/sqrt implementations round its last bit differently.
    rng = np.random.default_rng(70 + n)
    for g in one_gate_cases(n, rng):
        b0, b1 = random_codes(rng, n)
        r0, r1 = 0.01, 0.3
        st = O.CompactState(n, b0.copy(), b1.copy(), r0, r1).run([g])
        with jq.State(n, "compact") as s:
            s.write_codes(b0, b1, (r0, r1))
            s.apply_circuit([g])
            g0, g1, rng_gpu = s.codes()
        d0, d1 = code_diffs(g0, g1, st.b0, st.b1)
        assert np.array_equal(rng_gpu, st.rng), (g[0], rng_gpu, st.rng)
        assert d0.max() <= 1 and d1.max() <= 1, (g[0], d0.max(), d1.max())
        mismatched = int(np.sum((d0 != 0) | (d1 != 0)))
        assert mismatched <= max(2, 1e-3 * d0.size), (g[0], mismatched)


@pytest.mark.parametrize("n", [3, 8, 12])
def test_compact_random_circuit(n):
    # whole circuits: a tie decided differently early on changes later codes,
    # so the check is on accuracy: the GPU's encoded state is as close to the
    # exact state as the oracle's (fidelity loss within 2x), and almost all
    # codes agree.
    circ = W.random_circuit(n, 60, seed=30 + n)
    st = O.CompactState.encode(O.zero_state(n), n).run(circ)
    with jq.State(n, "compact") as s:
        s.apply_circuit(circ)
        b0, b1, rng = s.codes()
        amps = s.amplitudes()
    d0, d1 = code_diffs(b0, b1, st.b0, st.b1)
    assert int(np.sum((d0 != 0) | (d1 != 0))) <= max(2, 0.01 * d0.size)
    exact = run_oracle(n, circ)
    f_gpu, f_or = O.fidelity(amps, exact), O.fidelity(st.decode(), exact)
    assert 1 - f_gpu <= 2 * (1 - f_or) + 1e-12, (f_gpu, f_or)


@pytest.mark.parametrize("n", [6, 13])
def test_compact_haar_circuit_codes_identical(n):
    # no exact ties: Haar U(2) gates and random-angle RZ
    circ = W.layered_u2_cz(n, 3, seed=n)
    st = O.CompactState.encode(O.zero_state(n), n).run(circ)
    with jq.State(n, "compact") as s:
        s.apply_circuit(circ)
        b0, b1, rng = s.codes()
    d0, d1 = code_diffs(b0, b1, st.b0, st.b1)
    assert np.mean((d0 == 0) & (d1 == 0)) >= 1 - 1e-4
    assert np.allclose(rng, st.rng, rtol=1e-12, atol=0)


@pytest.mark.parametrize("n", [5, 11])
def test_compact_uniform_ghz_exact(n):
    with jq.State(n, "compact") as s:
        s.apply_circuit(W.hadamard_all(n))
        assert np.max(np.abs(s.amplitudes() - 2.0 ** (-n / 2))) < 1e-15
        s.init(jq.JQ_INIT_ZERO)
        s.apply_circuit(W.ghz(n))
        ref = np.zeros(1 << n, dtype=complex)
        ref[0] = ref[-1] = 1 / math.sqrt(2)
        assert np.max(np.abs(s.amplitudes() - ref)) < 1e-15
        assert abs(s.norm() - 1) < 1e-15


def test_compact_rz_cnot_chain_matches_oracle_codes():
    n = 12
    circ = W.rz_cnot_chain(n, 4, seed=3)
    st, b0, b1, rng, amps = compact_compare(n, circ, init="uniform")
    assert np.array_equal(b0, st.b0)
    d1 = np.abs(((b1.astype(int) - st.b1.astype(int)) + 128) % 256 - 128)
    assert np.mean(d1 == 0) >= 1 - 1e-4 and d1.max() <= 1


@pytest.mark.parametrize("enc", ["c128", "c64"])
def test_fused_op_ring_wraps_and_grows(enc):
    # one state, many calls: the fused ops of each call go to the device
    # through a ring (about a thousand ops) that wraps around across calls
    # and grows when one upload needs more (passes of up to 256 SWAPs, three
    # ops each); every call must still match the oracle
    n = 14
    rng = np.random.default_rng(21)
    psi = rand_state(rng, n)
    ref = psi.copy()
    total = 0
    with jq.State(n, enc) as s:
        s.write_amplitudes(psi)
        for k in range(10):
            circ = W.layered_u2_cz(n, 20, seed=100 + k)
            s.apply_circuit(circ)
            ref = O.run(ref, n, circ)
            total += len(circ)
            got = s.amplitudes()
            assert O.rel_l2(got, ref) <= tol(enc, total), (k, O.rel_l2(got, ref))
        swaps = []
        for _ in range(1500):  # qubits 0..9 fit one tile: 256 SWAPs a pass
            a, b = rng.choice(10, size=2, replace=False)
            swaps.append(("SWAP", (int(a), int(b)), ()))
        s.apply_circuit(swaps, max_ops=256)
        ref = O.run(ref, n, swaps)
        got = s.amplitudes()
        assert O.rel_l2(got, ref) <= tol(enc, total), O.rel_l2(got, ref)


@pytest.mark.parametrize("search", SEARCH)
@pytest.mark.parametrize("enc", ["c128", "c64"])
@pytest.mark.parametrize("n", [12, 16, 21])
def test_one_qubit_diagonals_run_grouped(enc, n, search):
    # layers of one-qubit diagonals (RZ, T, S, Z, U1) on every qubit between
    # Hadamards and a CNOT chain: in a pass, those on lane qubits and on
    # qubits outside the tile run as products, one factor per thread
    rng = np.random.default_rng(n)
    circ = []
    for _ in range(6):
        circ += [("H", (q,), ()) for q in range(0, n, 3)]
        for q in range(n):
            k = int(rng.integers(5))
            if k == 0:
                circ.append(("RZ", (q,), (float(rng.uniform(0.0, 2.0 * math.pi)),)))
            elif k == 1:
                circ.append(("U1", (q,), (float(rng.uniform(0.0, 2.0 * math.pi)),)))
            else:
                circ.append((["T", "S", "Z"][k - 2], (q,), ()))
        circ += [("CNOT", (q, q + 1), ()) for q in range(n - 1)]
    psi = rand_state(rng, n)
    got = run_gpu(n, enc, circ, init=psi, search=search)
    ref = run_oracle(n, circ, init=psi)
    assert O.rel_l2(got, ref) <= tol(enc, len(circ)), O.rel_l2(got, ref)


@pytest.mark.parametrize("enc", ["c128", "c64"])
@pytest.mark.parametrize("n", [14, 18])
def test_searched_plans_differ_and_match_the_oracle(enc, n):
    # the searched plan of a deep layered circuit is not the first-come plan
    # (else the forced runs above would test nothing new), and both give the
    # oracle's state
    circ = W.layered_u2_cz(n, 12, seed=40 + n) + W.rz_cnot_chain(n, 6, seed=n)
    on = jq.plan_steps(n, enc, circ, search=jq.JQ_SEARCH_ON)
    off = jq.plan_steps(n, enc, circ, search=jq.JQ_SEARCH_OFF)
    assert [(s["reg_q"], s["lane_q"]) for s in on] != [(s["reg_q"], s["lane_q"]) for s in off]
    psi = rand_state(np.random.default_rng(n), n)
    ref = run_oracle(n, circ, init=psi)
    for search in (jq.JQ_SEARCH_ON, jq.JQ_SEARCH_OFF):
        got = run_gpu(n, enc, circ, init=psi, search=search)
        assert O.rel_l2(got, ref) <= tol(enc, len(circ)), (search, O.rel_l2(got, ref))


GPU_SNIPPET = """
import sys
sys.path.insert(0, {root!r})
import numpy as np
import torch
from oracle import core as O
from paper_1805_04708_amd import jq, workloads as W
torch.cuda.set_device(0)
n = 14
circ = W.layered_u2_cz(n, 3, seed=5) + W.random_circuit(n, 80, seed=6)
ref = O.run(O.zero_state(n), n, circ)
for enc, tol in (("c128", 1e-12), ("c64", 4e-6)):
    with jq.State(n, enc) as s:
        s.apply_circuit(circ)
        err = O.rel_l2(s.amplitudes(), ref)
        assert err <= tol, (enc, err)
print("switches ok")
"""


@pytest.mark.parametrize("force", ["per_gate", "fused"])
def test_debug_switches_keep_oracle_parity(force):
    # a child process with every kernel waited for and checked
    # (JQ_LAUNCH_BLOCKING), roctx ranges on, and the kernel class forced
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, JQ_LAUNCH_BLOCKING="1", JQ_ROCTX="1", JQ_FORCE_KERNEL=force)
    print(f"child with JQ_FORCE_KERNEL={force}", flush=True)
    r = subprocess.run([sys.executable, "-c", GPU_SNIPPET.format(root=root)], env=env, capture_output=True,
                       text=True, timeout=240)
    assert r.returncode == 0 and "switches ok" in r.stdout, r.stderr[-3000:]


LOOP_SNIPPET = """
import hashlib, sys
sys.path.insert(0, {root!r})
import torch
from paper_1805_04708_amd import jq, workloads as W
torch.cuda.set_device(0)
cases = {cases!r}
out = []
for enc, n, k in cases:
    with jq.State(n, enc) as s:
        s.apply_circuit(W.layered_u2_cz(n, 6, seed=n + k), fusion=k)
        out.append(hashlib.sha256(s.amplitudes().tobytes()).hexdigest())
print("hashes " + " ".join(out))
"""


def test_reduced_op_loop_matches_the_general_loop_bit_for_bit():
    # layered U(2) + CZ circuits lower to dense and multiplexed 2x2s and
    # negations only, so every pass runs the op loop compiled for those
    # kinds; JQ_FUSED_OPS=all (read once per process: a child) runs the same
    # plans with the loop compiled for every kind.  Both share the ops' code,
    # so the amplitudes agree bit for bit.
    import hashlib
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cases = [("c128", 16, 4), ("c128", 16, 5), ("c64", 16, 5), ("c64", 17, 6)]
    here = []
    for enc, n, k in cases:
        with jq.State(n, enc) as s:
            s.apply_circuit(W.layered_u2_cz(n, 6, seed=n + k), fusion=k)
            here.append(hashlib.sha256(s.amplitudes().tobytes()).hexdigest())
    env = dict(os.environ, JQ_FUSED_OPS="all")
    print("child with JQ_FUSED_OPS=all", flush=True)
    r = subprocess.run([sys.executable, "-c", LOOP_SNIPPET.format(root=root, cases=cases)], env=env,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-3000:]
    line = [x for x in r.stdout.splitlines() if x.startswith("hashes ")][-1]
    assert line.split()[1:] == here

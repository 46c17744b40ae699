"""ctypes binding of the oracle's C code (``oracle/jq_oracle.c``).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""
import ctypes
import os

import numpy as np

from . import gates as G
from .build import LIB, build

_lib = None

GATE_DT = np.dtype([("k", np.int32), ("nc", np.int32), ("targets", np.int32, 3),
                    ("controls", np.int32, 8), ("m", np.float64, 128)], align=True)

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_bp = ctypes.POINTER(ctypes.c_int8)


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("JQ_ORACLE_LIB")  # another build (the sanitizer build, say)
        if not path:
            path = LIB
            if not os.path.exists(LIB):
                build(force=False)
        L = ctypes.CDLL(path)
        L.oq_apply.argtypes = [_dp, ctypes.c_int, _ip, ctypes.c_int, _ip, ctypes.c_int, _dp]
        L.oq_run.argtypes = [_dp, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]
        L.oq_norm2.argtypes = [_dp, ctypes.c_int]
        L.oq_norm2.restype = ctypes.c_double
        L.oq_probabilities.argtypes = [_dp, ctypes.c_int, _ip, ctypes.c_int, _dp]
        L.oq_expect_q.argtypes = [_dp, ctypes.c_int, _dp, _dp, _dp]
        L.oq_project.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oq_project.restype = ctypes.c_double
        L.oq_measure.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp]
        L.oq_sample.argtypes = [_dp, ctypes.c_int, _dp, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]
        L.oq_compact_decode.argtypes = [_bp, _bp, ctypes.c_uint64, ctypes.c_double, ctypes.c_double, _dp]
        L.oq_compact_encode.argtypes = [_dp, ctypes.c_uint64, ctypes.c_double, ctypes.c_double, _bp, _bp]
        L.oq_compact_range.argtypes = [_dp, ctypes.c_uint64, _dp, _dp]
        L.oq_compact_run.argtypes = [_bp, _bp, ctypes.c_int, _dp, ctypes.c_void_p, ctypes.c_int, _dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _b(a):
    return a.ctypes.data_as(_bp)


def zero_state(n):
    """|0...0> (Sec. 2: all qubits in state |0>)."""
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def uniform_state(n):
    """All amplitudes 2^(-N/2): the state after H on every qubit (Sec. 5.1)."""
    return np.full(1 << n, 2.0 ** (-n / 2.0), dtype=np.complex128)


def basis_state(n, x):
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[x] = 1.0
    return psi


def gate_records(circuit):
    """Lower named gates with the oracle's own table into C records."""
    recs = np.zeros(len(circuit), dtype=GATE_DT)
    for i, g in enumerate(circuit):
        targets, controls, m = G.lower(g)
        k = len(targets)
        K = 1 << k
        recs[i]["k"] = k
        recs[i]["nc"] = len(controls)
        recs[i]["targets"][:k] = targets
        recs[i]["controls"][:len(controls)] = controls
        flat = np.empty(2 * K * K)
        flat[0::2] = m.real.ravel()
        flat[1::2] = m.imag.ravel()
        recs[i]["m"][:2 * K * K] = flat
    return recs


def apply(psi, n, targets, controls, m):
    """Apply one explicit matrix in place (Sec. 2, Eq. NUM2 generalised)."""
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous and psi.size == 1 << n
    t = np.ascontiguousarray(targets, dtype=np.int32)
    c = np.ascontiguousarray(controls if len(controls) else [0], dtype=np.int32)
    K = 1 << len(targets)
    mm = np.empty(2 * K * K)
    m = np.asarray(m, dtype=np.complex128)
    mm[0::2] = m.real.ravel()
    mm[1::2] = m.imag.ravel()
    rc = lib().oq_apply(_d(psi.view(np.float64)), n, _i(t), len(targets), _i(c), len(controls), _d(mm))
    if rc:
        raise ValueError("invalid gate for the oracle")
    return psi


def run(psi, n, circuit):
    """Apply a whole circuit of named gates in place."""
    recs = gate_records(circuit)
    if len(recs):
        rc = lib().oq_run(_d(psi.view(np.float64)), n, recs.ctypes.data, len(recs))
        if rc:
            raise ValueError("invalid gate for the oracle")
    return psi


def norm2(psi, n):
    return lib().oq_norm2(_d(psi.view(np.float64)), n)


def probabilities(psi, n, qubits):
    q = np.ascontiguousarray(qubits if len(qubits) else [0], dtype=np.int32)
    out = np.zeros(1 << len(qubits))
    if lib().oq_probabilities(_d(psi.view(np.float64)), n, _i(q), len(qubits), _d(out)):
        raise ValueError("invalid qubits")
    return out


def expect_q(psi, n):
    """(<Qx(i)>, <Qy(i)>, <Qz(i)>) for every qubit (App. A, BEGIN MEASUREMENT)."""
    qx, qy, qz = np.zeros(n), np.zeros(n), np.zeros(n)
    lib().oq_expect_q(_d(psi.view(np.float64)), n, _d(qx), _d(qy), _d(qz))
    return qx, qy, qz


def project(psi, n, q, v):
    """Project qubit q onto |v> and renormalise in place (App. A, CLEAR /
    SET); returns the probability p of |v> (0: the state is unchanged)."""
    return lib().oq_project(_d(psi.view(np.float64)), n, q, v)


def measure(psi, n, q, u):
    """Projective measurement of qubit q (App. A, M) with the draw u in
    [0, 1): outcome 1 iff u >= p0 / (p0 + p1).  Returns (outcome, p1)."""
    p1 = ctypes.c_double(0.0)
    out = lib().oq_measure(_d(psi.view(np.float64)), n, q, u, ctypes.byref(p1))
    if out < 0:
        raise ValueError("zero state")
    return out, p1.value


def sample(psi, n, u):
    """Basis states drawn from |a|^2 (App. A, GENERATE EVENTS) for the draws
    u in [0, 1): event k is the least i whose cumulative probability (in
    index order) exceeds u_k times the total."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(max(1, len(u)), dtype=np.uint64)
    if lib().oq_sample(_d(psi.view(np.float64)), n, _d(u), len(u),
                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))):
        raise ValueError("zero state")
    return out[:len(u)]


def cdf(psi):
    """Cumulative probabilities in index order (the sums oq_sample uses)."""
    return np.cumsum(np.abs(psi) ** 2)


def run_program(psi, n, program, draws=()):
    """Run gates and the instructions M, CLEAR and SET (App. A) in order.
    draws supplies u for each M; returns the list of M outcomes.  CLEAR and
    SET on an outcome of probability zero raise ValueError."""
    draws = iter(draws)
    outcomes = []
    for ins in program:
        name, q = ins[0], ins[1]
        if name == "M":
            outcomes.append(measure(psi, n, q[0], next(draws))[0])
        elif name in ("CLEAR", "SET"):
            if project(psi, n, q[0], 0 if name == "CLEAR" else 1) == 0.0:
                raise ValueError(f"{name} {q[0]}: projection onto a zero-amplitude state")
        else:
            run(psi, n, [ins])
    return outcomes


def rel_l2(psi, ref):
    return float(np.linalg.norm(psi - ref) / np.linalg.norm(ref))


def fidelity(psi, ref):
    return float(abs(np.vdot(ref, psi)) ** 2 / (np.vdot(ref, ref).real * np.vdot(psi, psi).real))


# -- the two-byte encoding (Sec. 4.1) --------------------------------------

class CompactState:
    """Codes b0, b1 (int8 planes) and the range (r0, r1) of Sec. 4.1."""

    def __init__(self, n, b0, b1, r0, r1):
        self.n, self.b0, self.b1 = n, b0, b1
        self.rng = np.array([r0, r1], dtype=np.float64)

    @classmethod
    def encode(cls, psi, n, r0=None, r1=None):
        """Encode psi; the range is taken from psi unless given."""
        dim = 1 << n
        b0 = np.zeros(dim, dtype=np.int8)
        b1 = np.zeros(dim, dtype=np.int8)
        if r0 is None:
            lo, hi = ctypes.c_double(0.0), ctypes.c_double(0.0)
            lib().oq_compact_range(_d(psi.view(np.float64)), dim, ctypes.byref(lo), ctypes.byref(hi))
            r0, r1 = lo.value, hi.value
        lib().oq_compact_encode(_d(psi.view(np.float64)), dim, r0, r1, _b(b0), _b(b1))
        return cls(n, b0, b1, r0, r1)

    def decode(self):
        psi = np.zeros(1 << self.n, dtype=np.complex128)
        lib().oq_compact_decode(_b(self.b0), _b(self.b1), 1 << self.n, self.rng[0], self.rng[1],
                                _d(psi.view(np.float64)))
        return psi

    def project(self, q, v):
        """Projection with renormalisation as a quantisation step (App. A,
        CLEAR / SET; Sec. 4.1): decode, p = sum of |z|^2 over bit q = v, then
        the diagonal gate sqrt(1/p)|v><v| on qubit q with a new range.
        Returns p; on p == 0 the codes are unchanged."""
        psi = self.decode()
        b = 1 << q
        idx = np.arange(1 << self.n)
        keep = ((idx & b) != 0) == (v != 0)
        p = float(np.sum(np.abs(psi[keep]) ** 2))
        if p == 0.0:
            return 0.0
        f = 1.0 / np.sqrt(p)
        d = (f, 0, 0, 0, 0, 0, 0, 0) if v == 0 else (0, 0, 0, 0, 0, 0, f, 0)
        self.run([("MAT1", (q,), d)])
        return p

    def run(self, circuit, blocks=None):
        """Apply a circuit.  blocks=None quantises after every gate (the
        paper's procedure); otherwise blocks is a list of gate counts and the
        state is decoded/encoded once per block."""
        recs = gate_records(circuit)
        scratch = np.zeros(2 << self.n, dtype=np.float64)
        sizes = [1] * len(recs) if blocks is None else list(blocks)
        assert sum(sizes) == len(recs)
        pos = 0
        for cnt in sizes:
            rc = lib().oq_compact_run(_b(self.b0), _b(self.b1), self.n, _d(self.rng),
                                      recs[pos:pos + cnt].ctypes.data, cnt, _d(scratch))
            if rc:
                raise ValueError("invalid gate for the oracle")
            pos += cnt
        return self

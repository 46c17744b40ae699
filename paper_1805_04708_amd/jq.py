"""ctypes binding of ``libjq.so`` (the C ABI in ``include/jq.h``).

Argument marshalling only: every step of gate application, reduction and
encoding runs in the library's HIP kernels.  The library must be built
(``python -m paper_1805_04708_amd.build``); importing this module without it
raises, and there is no fallback.

PyTorch supplies device memory (``use_torch_allocator``) and streams
(``State.set_stream(torch.cuda.current_stream())``); nothing else of it is
used.
"""
import ctypes
import os

import numpy as np

from .build import LIB

JQ_OK, JQ_EINVAL, JQ_ENOMEM, JQ_EDEVICE, JQ_EUNSUPPORTED, JQ_EZERO, JQ_EBUSY = 0, -1, -2, -3, -4, -5, -6
JQ_C128, JQ_C64, JQ_COMPACT = 0, 1, 2
JQ_INIT_ZERO, JQ_INIT_UNIFORM, JQ_INIT_BASIS = 0, 1, 2
JQ_DENSE, JQ_DIAGONAL, JQ_PERM_X = 0, 1, 2
JQ_COMPACT_PER_GATE, JQ_COMPACT_PER_BLOCK = 0, 1
JQ_SEARCH_AUTO, JQ_SEARCH_ON, JQ_SEARCH_OFF = 0, 1, 2
JQ_TUNE_DEFAULT, JQ_TUNE_MEASURED, JQ_TUNE_CACHED, JQ_TUNE_SET = 0, 1, 2, 3
JQ_TUNE_FORCE, JQ_TUNE_NO_CACHE = 1, 2
JQ_MAX_CONTROLS = 4
ENCODINGS = {"c128": JQ_C128, "c64": JQ_C64, "compact": JQ_COMPACT}


class JqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class Gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nq", ctypes.c_int32), ("nc", ctypes.c_int32),
                ("qubits", ctypes.c_int32 * 2), ("controls", ctypes.c_int32 * JQ_MAX_CONTROLS),
                ("pad_", ctypes.c_int32), ("m", ctypes.c_double * 32)]


class Tuning(ctypes.Structure):
    _fields_ = [("k_reg", ctypes.c_int32), ("wide_target", ctypes.c_int32), ("pass_ops", ctypes.c_double),
                ("n_qubits", ctypes.c_int32), ("source", ctypes.c_int32), ("tuned_ms", ctypes.c_double),
                ("default_ms", ctypes.c_double), ("search", ctypes.c_int32), ("reserved_", ctypes.c_int32),
                ("wide_mask", ctypes.c_uint64)]


class ExecOpts(ctypes.Structure):
    _fields_ = [("fusion", ctypes.c_int32), ("compact_mode", ctypes.c_int32), ("max_ops", ctypes.c_int32),
                ("search", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]


class PlanStep(ctypes.Structure):
    _fields_ = [("fused", ctypes.c_int32), ("k_reg", ctypes.c_int32), ("reg_q", ctypes.c_int32 * 8),
                ("lane_q", ctypes.c_int32 * 6), ("n_gates", ctypes.c_int32), ("n_ops", ctypes.c_int32),
                ("table_tag", ctypes.c_int32), ("n_tables", ctypes.c_int32)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class Circuit(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("pad_", ctypes.c_int32), ("n_gates", ctypes.c_uint64),
                ("gates", ctypes.POINTER(Gate))]


class Result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int32), ("n_qubits", ctypes.c_int32),
                ("norm", ctypes.c_double), ("latency_ms", ctypes.c_double), ("queue_ms", ctypes.c_double),
                ("state", ctypes.c_void_p)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("throughput_per_s", ctypes.c_double), ("peak_resident_bytes", ctypes.c_uint64)]


_VP = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int)
_BP = ctypes.POINTER(ctypes.c_int8)
_U64 = ctypes.c_uint64

# name -> (restype, argtypes); every function declared in include/jq.h
SIGNATURES = {
    "jq_state_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(_VP)]),
    "jq_state_destroy": (ctypes.c_int, [_VP]),
    "jq_state_init": (ctypes.c_int, [_VP, ctypes.c_int, _U64]),
    "jq_state_info": (ctypes.c_int, [_VP, _IP, _IP, ctypes.POINTER(_U64)]),
    "jq_shorbox": (ctypes.c_int, [_VP, ctypes.c_int, _U64, _U64]),
    "jq_state_device_ptr": (ctypes.c_int, [_VP, ctypes.POINTER(_VP)]),
    "jq_set_stream": (ctypes.c_int, [_VP, _VP]),
    "jq_synchronize": (ctypes.c_int, [_VP]),
    "jq_set_allocator": (ctypes.c_int, [_VP, _VP, _VP]),
    "jq_gate_named": (ctypes.c_int, [ctypes.c_char_p, _IP, ctypes.c_int, _DP, ctypes.c_int, ctypes.POINTER(Gate)]),
    "jq_gates_named": (ctypes.c_int, [ctypes.c_size_t, ctypes.POINTER(ctypes.c_char_p), _IP, _IP, _IP, _DP, _IP, _IP,
                                      ctypes.POINTER(Gate)]),
    "jq_apply_gate": (ctypes.c_int, [_VP, ctypes.c_int, _IP, ctypes.c_int, _IP, ctypes.c_int, _DP]),
    "jq_apply_circuit": (ctypes.c_int, [_VP, ctypes.POINTER(Gate), ctypes.c_size_t, ctypes.POINTER(ExecOpts)]),
    "jq_apply_circuit_noalloc": (ctypes.c_int, [_VP, ctypes.POINTER(Gate), ctypes.c_size_t,
                                                ctypes.POINTER(ExecOpts)]),
    "jq_apply_circuit_noisy": (ctypes.c_int, [_VP, ctypes.POINTER(Gate), ctypes.c_size_t, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_double, _DP, ctypes.POINTER(ExecOpts)]),
    "jq_plan_schedule": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(Gate), ctypes.c_size_t,
                                        ctypes.POINTER(ExecOpts), ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_size_t)]),
    "jq_plan_steps": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(Gate), ctypes.c_size_t,
                                     ctypes.POINTER(ExecOpts), ctypes.POINTER(PlanStep), ctypes.c_size_t,
                                     ctypes.POINTER(ctypes.c_size_t)]),
    "jq_tuning_get": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(Tuning)]),
    "jq_tuning_set": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(Tuning)]),
    "jq_autotune": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Gate), ctypes.c_size_t,
                                   ctypes.POINTER(Tuning)]),
    "jq_norm": (ctypes.c_int, [_VP, _DP]),
    "jq_probabilities": (ctypes.c_int, [_VP, _IP, ctypes.c_int, _DP]),
    "jq_expectations": (ctypes.c_int, [_VP, _DP, _DP, _DP]),
    "jq_renormalize": (ctypes.c_int, [_VP]),
    "jq_aux_amplitudes": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(Gate), ctypes.c_size_t,
                                         ctypes.POINTER(_U64), ctypes.c_size_t, _DP]),
    "jq_sample": (ctypes.c_int, [_VP, _DP, ctypes.c_size_t, ctypes.POINTER(_U64)]),
    "jq_project": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _DP]),
    "jq_measure": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_double, _IP, _DP]),
    "jq_read_amplitudes": (ctypes.c_int, [_VP, _U64, _U64, _DP]),
    "jq_write_amplitudes": (ctypes.c_int, [_VP, _U64, _U64, _DP]),
    "jq_read_codes": (ctypes.c_int, [_VP, _U64, _U64, _BP, _BP, _DP]),
    "jq_write_codes": (ctypes.c_int, [_VP, _BP, _BP, _DP]),
    "jq_profile_enable": (ctypes.c_int, [_VP, ctypes.c_int]),
    "jq_profile_read": (ctypes.c_int, [_VP, ctypes.POINTER(KernelStat), ctypes.c_int, _IP]),
    "jq_batch_create": (ctypes.c_int, [ctypes.POINTER(Circuit), ctypes.c_size_t, ctypes.c_int,
                                       ctypes.POINTER(ExecOpts), _VP, ctypes.POINTER(_VP)]),
    "jq_batch_run": (ctypes.c_int, [_VP, _DP]),
    "jq_batch_read": (ctypes.c_int, [_VP, ctypes.c_size_t, _U64, _U64, _DP]),
    "jq_batch_destroy": (ctypes.c_int, [_VP]),
    "jq_server_create": (ctypes.c_int, [_U64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_VP)]),
    "jq_server_submit": (ctypes.c_int, [_VP, ctypes.POINTER(Circuit), ctypes.c_int, ctypes.POINTER(_U64)]),
    "jq_server_wait": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.POINTER(Result)]),
    "jq_server_release": (ctypes.c_int, [_VP, _U64]),
    "jq_server_stats_get": (ctypes.c_int, [_VP, ctypes.POINTER(ServerStats)]),
    "jq_server_destroy": (ctypes.c_int, [_VP]),
    "jq_last_error": (ctypes.c_char_p, []),
    "jq_version": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libjq.so (raises if it has not been built: there is no fallback).
    The environment variable JQ_LIB names another build of the library to
    load instead (the host-sanitizer build, say)."""
    global _lib
    if _lib is None:
        path = os.environ.get("JQ_LIB") or LIB
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with `python -m paper_1805_04708_amd.build`")
        L = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != JQ_OK:
        raise JqError(rc, lib().jq_last_error().decode())
    return rc


def _dp(a):
    return a.ctypes.data_as(_DP)


def _ip(a):
    return a.ctypes.data_as(_IP)


# ------------------------------------------------------------- gates --

def gate(name, qubits, params=(), controls=()):
    """A named instruction (App. A names, plus RZ, CZ, CP, SWAP, MAT1, MAT2)
    lowered by the library; extra controls are appended."""
    q = np.ascontiguousarray(list(qubits) or [0], dtype=np.int32)
    p = np.ascontiguousarray(list(params) or [0.0], dtype=np.float64)
    g = Gate()
    check(lib().jq_gate_named(name.encode(), _ip(q), len(qubits), _dp(p), len(params), ctypes.byref(g)))
    if controls:
        if g.nc + len(controls) > JQ_MAX_CONTROLS:
            raise JqError(JQ_EINVAL, "too many controls")
        for c in controls:
            g.controls[g.nc] = int(c)
            g.nc += 1
    return g


def gates(circuit):
    """Lower a list of (name, qubits, params[, controls]) tuples into a Gate
    array (one jq_gates_named call)."""
    n = len(circuit)
    arr = (Gate * max(1, n))()
    if n == 0:
        return arr, 0
    names = (ctypes.c_char_p * n)(*[g[0].encode() for g in circuit])
    nq = np.fromiter((len(g[1]) for g in circuit), dtype=np.int32, count=n)
    qs = np.fromiter((q for g in circuit for q in g[1]), dtype=np.int32)
    npar = np.fromiter((len(g[2]) for g in circuit), dtype=np.int32, count=n)
    ps = np.fromiter((p for g in circuit for p in g[2]), dtype=np.float64)
    nc = np.fromiter((len(g[3]) if len(g) > 3 else 0 for g in circuit), dtype=np.int32, count=n)
    cs = np.fromiter((c for g in circuit if len(g) > 3 for c in g[3]), dtype=np.int32)
    check(lib().jq_gates_named(n, names, _ip(nq), _ip(qs) if qs.size else None, _ip(npar),
                               _dp(ps) if ps.size else None, _ip(nc), _ip(cs) if cs.size else None, arr))
    return arr, n


def exec_opts(fusion=0, compact_mode=JQ_COMPACT_PER_GATE, max_ops=0, search=JQ_SEARCH_AUTO):
    o = ExecOpts()
    o.fusion, o.compact_mode, o.max_ops, o.search = fusion, compact_mode, max_ops, search
    return o


def plan_steps(n, enc, circuit, fusion=0, compact_mode=JQ_COMPACT_PER_GATE, max_ops=0, search=JQ_SEARCH_AUTO):
    """Host-only list of the steps jq_apply_circuit runs (jq_plan_steps), as dicts."""
    arr, cnt = circuit if isinstance(circuit, tuple) else gates(circuit)
    opts = exec_opts(fusion, compact_mode, max_ops, search)
    n_steps = ctypes.c_size_t()
    check(lib().jq_plan_steps(n, ENCODINGS.get(enc, enc), arr, cnt, ctypes.byref(opts), None, 0,
                              ctypes.byref(n_steps)))
    out = (PlanStep * max(1, n_steps.value))()
    check(lib().jq_plan_steps(n, ENCODINGS.get(enc, enc), arr, cnt, ctypes.byref(opts), out, n_steps.value,
                              ctypes.byref(n_steps)))
    return [{"fused": bool(st.fused), "k_reg": st.k_reg, "reg_q": list(st.reg_q[:st.k_reg]),
             "lane_q": list(st.lane_q), "n_gates": st.n_gates, "n_ops": st.n_ops, "table_tag": st.table_tag,
             "n_tables": st.n_tables} for st in out[:n_steps.value]]


_TUNE_SOURCES = {JQ_TUNE_DEFAULT: "default", JQ_TUNE_MEASURED: "measured", JQ_TUNE_CACHED: "cached",
                 JQ_TUNE_SET: "set"}


def _tuning_dict(t):
    return {"k_reg": t.k_reg, "wide_target": t.wide_target, "wide_mask": t.wide_mask, "pass_ops": t.pass_ops,
            "search": t.search, "n_qubits": t.n_qubits,
            "source": _TUNE_SOURCES.get(t.source, t.source), "tuned_ms": t.tuned_ms, "default_ms": t.default_ms}


def tuning_get(n, enc):
    """The tuning jq_apply_circuit uses for an n-qubit state (jq_tuning_get), as a dict."""
    t = Tuning()
    check(lib().jq_tuning_get(n, ENCODINGS.get(enc, enc), ctypes.byref(t)))
    return _tuning_dict(t)


def tuning_set(n, enc, k_reg=None, wide_target=None, pass_ops=None, search=None, clear=False, wide_mask=None):
    """Override (jq_tuning_set) fields of the current tuning; clear=True removes an override.
    wide_target sets the per-gate width as a threshold, wide_mask target by target."""
    if clear:
        check(lib().jq_tuning_set(n, ENCODINGS.get(enc, enc), None))
        return
    t = Tuning()
    check(lib().jq_tuning_get(n, ENCODINGS.get(enc, enc), ctypes.byref(t)))
    if k_reg is not None:
        t.k_reg = k_reg
    if wide_target is not None:
        t.wide_target = wide_target
        t.wide_mask = 0  # from the threshold
    if wide_mask is not None:
        t.wide_mask = wide_mask
    if pass_ops is not None:
        t.pass_ops = pass_ops
    if search is not None:
        t.search = search
    check(lib().jq_tuning_set(n, ENCODINGS.get(enc, enc), ctypes.byref(t)))


def autotune(n, enc, circuit=None, force=False, no_cache=False):
    """Measure the tuning on the current device (jq_autotune), as a dict;
    circuit (named gates or a gates() tuple) is the tuning workload."""
    t = Tuning()
    flags = (JQ_TUNE_FORCE if force else 0) | (JQ_TUNE_NO_CACHE if no_cache else 0)
    arr, cnt = (None, 0) if circuit is None else (circuit if isinstance(circuit, tuple) else gates(circuit))
    check(lib().jq_autotune(n, ENCODINGS.get(enc, enc), flags, arr, cnt, ctypes.byref(t)))
    return _tuning_dict(t)


def plan_schedule(n, enc, circuit, fusion=0, compact_mode=JQ_COMPACT_PER_GATE, max_ops=0, search=JQ_SEARCH_AUTO):
    """Host-only schedule of jq_apply_circuit: (order, block_len, block_fused),
    order being input gate indices in the order applied, split into
    consecutive blocks of block_len gates (fused tile pass or single gate)."""
    arr, cnt = circuit if isinstance(circuit, tuple) else gates(circuit)
    opts = exec_opts(fusion, compact_mode, max_ops, search)
    m = max(1, cnt)
    order = np.zeros(m, dtype=np.int32)
    blen = np.zeros(m, dtype=np.int32)
    bfused = np.zeros(m, dtype=np.int32)
    nb = ctypes.c_size_t()
    i32 = ctypes.POINTER(ctypes.c_int32)
    check(lib().jq_plan_schedule(n, ENCODINGS.get(enc, enc), arr, cnt, ctypes.byref(opts), order.ctypes.data_as(i32),
                                 blen.ctypes.data_as(i32), bfused.ctypes.data_as(i32), ctypes.byref(nb)))
    k = int(blen[:nb.value].sum())
    return order[:k].copy(), blen[:nb.value].copy(), bfused[:nb.value].astype(bool)


def aux_amplitudes(n, circuit, basis):
    """<b|circuit|0...0> for each b in basis by the auxiliary-variable method
    (Sec. 4.2): no state vector, time exponential only in the number of
    entangling gates."""
    arr, cnt = circuit if isinstance(circuit, tuple) else gates(circuit)
    b = np.ascontiguousarray(basis, dtype=np.uint64)
    out = np.zeros(max(1, b.size), dtype=np.complex128)
    check(lib().jq_aux_amplitudes(n, arr, cnt, b.ctypes.data_as(ctypes.POINTER(_U64)), b.size,
                                  _dp(out.view(np.float64))))
    return out[:b.size]


# -------------------------------------------------------------- state --

class State:
    """An N-qubit state on the current HIP device (owns its device memory,
    unless it was borrowed from a server result)."""

    def __init__(self, n, encoding="c128", handle=None):
        self.n = int(n)
        self.encoding = ENCODINGS[encoding] if isinstance(encoding, str) else int(encoding)
        self.owned = handle is None
        if handle is not None:
            self.h = _VP(handle)
            return
        h = _VP()
        check(lib().jq_state_create(self.n, self.encoding, ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            h, self.h = self.h, None
            if self.owned:
                check(lib().jq_state_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def nbytes(self):
        b = _U64()
        check(lib().jq_state_info(self.h, None, None, ctypes.byref(b)))
        return b.value

    def init(self, mode=JQ_INIT_ZERO, basis=0):
        check(lib().jq_state_init(self.h, mode, basis))
        return self

    def set_stream(self, stream):
        """stream: a torch.cuda.Stream, an int handle, or None (library stream)."""
        handle = getattr(stream, "cuda_stream", stream)
        check(lib().jq_set_stream(self.h, _VP(handle or 0) if handle else None))
        return self

    def synchronize(self):
        check(lib().jq_synchronize(self.h))

    def apply_gate(self, kind, qubits, controls=(), matrix=None):
        q = np.ascontiguousarray(qubits, dtype=np.int32)
        c = np.ascontiguousarray(list(controls) or [0], dtype=np.int32)
        m = None
        if matrix is not None:
            mc = np.ascontiguousarray(matrix, dtype=np.complex128).ravel()
            m = np.empty(2 * mc.size)
            m[0::2], m[1::2] = mc.real, mc.imag
        check(lib().jq_apply_gate(self.h, kind, _ip(q), len(q), _ip(c), len(controls),
                                  _dp(m) if m is not None else None))
        return self

    def apply_circuit(self, circuit, fusion=0, compact_mode=JQ_COMPACT_PER_GATE, max_ops=0, search=JQ_SEARCH_AUTO):
        """circuit: list of named gates, or (Gate array, count) from gates()."""
        arr, cnt = circuit if isinstance(circuit, tuple) else gates(circuit)
        opts = exec_opts(fusion, compact_mode, max_ops, search)
        check(lib().jq_apply_circuit(self.h, arr, cnt, ctypes.byref(opts)))
        return self

    def apply_circuit_noalloc(self, circuit, fusion=0, compact_mode=JQ_COMPACT_PER_GATE, max_ops=0,
                              search=JQ_SEARCH_AUTO):
        """apply_circuit through jq_apply_circuit_noalloc (fixed device workspace, no allocation)."""
        arr, cnt = circuit if isinstance(circuit, tuple) else gates(circuit)
        opts = exec_opts(fusion, compact_mode, max_ops, search)
        check(lib().jq_apply_circuit_noalloc(self.h, arr, cnt, ctypes.byref(opts)))
        return self

    def apply_circuit_noisy(self, circuit, px, py, pz, u, fusion=0, compact_mode=JQ_COMPACT_PER_GATE, max_ops=0):
        """apply_circuit with the depolarizing channel (App. A); u holds one
        draw in [0, 1) per gate and qubit, u[g * N + q]."""
        arr, cnt = circuit if isinstance(circuit, tuple) else gates(circuit)
        u = np.ascontiguousarray(u, dtype=np.float64)
        if u.size != cnt * self.n:
            raise JqError(JQ_EINVAL, "one draw per gate and qubit")
        opts = exec_opts(fusion, compact_mode, max_ops)
        check(lib().jq_apply_circuit_noisy(self.h, arr, cnt, px, py, pz, _dp(u if u.size else np.zeros(1)),
                                           ctypes.byref(opts)))
        return self

    def norm(self):
        out = ctypes.c_double()
        check(lib().jq_norm(self.h, ctypes.byref(out)))
        return out.value

    def probabilities(self, qubits):
        q = np.ascontiguousarray(list(qubits) or [0], dtype=np.int32)
        out = np.zeros(1 << len(qubits))
        check(lib().jq_probabilities(self.h, _ip(q), len(qubits), _dp(out)))
        return out

    def expectations(self):
        qx, qy, qz = np.zeros(self.n), np.zeros(self.n), np.zeros(self.n)
        check(lib().jq_expectations(self.h, _dp(qx), _dp(qy), _dp(qz)))
        return qx, qy, qz

    def renormalize(self):
        check(lib().jq_renormalize(self.h))
        return self

    def shorbox(self, n_x, G, y):
        """SHORBOX (App. A): 2^(-n_x/2) sum_x |x>|y^x mod G>, x on the low n_x qubits."""
        check(lib().jq_shorbox(self.h, n_x, G, y))
        return self

    def sample(self, u):
        """Basis states drawn from |a|^2 (App. A, GENERATE EVENTS) for the
        caller's draws u in [0, 1); returns a uint64 array."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        out = np.zeros(max(1, len(u)), dtype=np.uint64)
        check(lib().jq_sample(self.h, _dp(u), len(u), out.ctypes.data_as(ctypes.POINTER(_U64))))
        return out[:len(u)]

    def project(self, qubit, value):
        """Project qubit onto |value> and renormalise (App. A, CLEAR / SET);
        returns the probability of |value>.  JqError (JQ_EZERO) if it is 0."""
        p = ctypes.c_double()
        check(lib().jq_project(self.h, qubit, value, ctypes.byref(p)))
        return p.value

    def measure(self, qubit, u):
        """Projective measurement (App. A, M) with the caller's draw u in
        [0, 1): returns (outcome, p1)."""
        out, p1 = ctypes.c_int(), ctypes.c_double()
        check(lib().jq_measure(self.h, qubit, u, ctypes.byref(out), ctypes.byref(p1)))
        return out.value, p1.value

    def run_program(self, program, draws=()):
        """Gates and the instructions M, CLEAR, SET in order; consecutive
        gates go to jq_apply_circuit together.  Returns the M outcomes."""
        draws = iter(draws)
        outcomes, run = [], []
        for ins in list(program) + [None]:
            if ins is not None and ins[0] not in ("M", "CLEAR", "SET"):
                run.append(ins)
                continue
            if run:
                self.apply_circuit(run)
                run = []
            if ins is None:
                break
            if ins[0] == "M":
                outcomes.append(self.measure(ins[1][0], next(draws))[0])
            else:
                self.project(ins[1][0], 0 if ins[0] == "CLEAR" else 1)
        return outcomes

    def amplitudes(self, first=0, count=None):
        count = (1 << self.n) - first if count is None else count
        out = np.zeros(count, dtype=np.complex128)
        check(lib().jq_read_amplitudes(self.h, first, count, _dp(out.view(np.float64))))
        return out

    def write_amplitudes(self, psi, first=0):
        a = np.ascontiguousarray(psi, dtype=np.complex128)
        check(lib().jq_write_amplitudes(self.h, first, a.size, _dp(a.view(np.float64))))
        return self

    def codes(self, first=0, count=None):
        count = (1 << self.n) - first if count is None else count
        b0 = np.zeros(count, dtype=np.int8)
        b1 = np.zeros(count, dtype=np.int8)
        rng = np.zeros(2)
        check(lib().jq_read_codes(self.h, first, count, b0.ctypes.data_as(_BP), b1.ctypes.data_as(_BP), _dp(rng)))
        return b0, b1, rng

    def write_codes(self, b0, b1, rng):
        b0 = np.ascontiguousarray(b0, dtype=np.int8)
        b1 = np.ascontiguousarray(b1, dtype=np.int8)
        r = np.ascontiguousarray(rng, dtype=np.float64)
        check(lib().jq_write_codes(self.h, b0.ctypes.data_as(_BP), b1.ctypes.data_as(_BP), _dp(r)))
        return self

    def profile(self, on=True):
        check(lib().jq_profile_enable(self.h, 1 if on else 0))

    def profile_read(self):
        arr = (KernelStat * 16)()
        cnt = ctypes.c_int()
        check(lib().jq_profile_read(self.h, arr, 16, ctypes.byref(cnt)))
        return {arr[i].name.decode(): {"launches": arr[i].launches, "ms": arr[i].total_ms, "bytes": arr[i].bytes}
                for i in range(min(cnt.value, 16))}


# -------------------------------------------------------------- batch --

def circuit_struct(n, circuit):
    """(jq_circuit, keep-alive) for a list of named gates."""
    arr, cnt = gates(circuit)
    c = Circuit()
    c.n_qubits, c.n_gates = n, cnt
    c.gates = ctypes.cast(arr, ctypes.POINTER(Gate))
    return c, arr


class Batch:
    """Many small circuits run in one persistent launch (jq_batch_*)."""

    def __init__(self, instances, encoding="c128", fusion=0, stream=None):
        enc = ENCODINGS[encoding] if isinstance(encoding, str) else int(encoding)
        self.ns = [int(n) for n, _ in instances]
        structs = (Circuit * len(instances))()
        self._keep = []
        for i, (n, circ) in enumerate(instances):
            c, arr = circuit_struct(n, circ)
            structs[i] = c
            self._keep.append(arr)
        opts = exec_opts(fusion)
        h = _VP()
        handle = getattr(stream, "cuda_stream", stream)
        check(lib().jq_batch_create(structs, len(instances), enc, ctypes.byref(opts),
                                    _VP(handle) if handle else None, ctypes.byref(h)))
        self.h = h
        self._keep = None

    def run(self, timed=False):
        ms = ctypes.c_double()
        check(lib().jq_batch_run(self.h, ctypes.byref(ms) if timed else None))
        return ms.value if timed else None

    def amplitudes(self, index):
        dim = 1 << self.ns[index]
        out = np.zeros(dim, dtype=np.complex128)
        check(lib().jq_batch_read(self.h, index, 0, dim, _dp(out.view(np.float64))))
        return out

    def close(self):
        if self.h:
            h, self.h = self.h, None
            check(lib().jq_batch_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ server --

class Server:
    """Request loop (jq_server_*): circuits of mixed N admitted by state bytes
    against an HBM budget, run concurrently on several streams."""

    def __init__(self, hbm_budget, n_streams=4, queue_cap=4096, encoding="c64"):
        self.encoding = ENCODINGS[encoding] if isinstance(encoding, str) else int(encoding)
        h = _VP()
        check(lib().jq_server_create(int(hbm_budget), n_streams, queue_cap, self.encoding, ctypes.byref(h)))
        self.h = h

    def submit(self, n, circuit, blocking=True):
        """circuit: named gates, or a (Gate array, count) pair from gates()."""
        arr, cnt = circuit if isinstance(circuit, tuple) else gates(circuit)
        c = Circuit()
        c.n_qubits, c.n_gates = int(n), cnt
        c.gates = ctypes.cast(arr, ctypes.POINTER(Gate))
        t = _U64()
        check(lib().jq_server_submit(self.h, ctypes.byref(c), 1 if blocking else 0, ctypes.byref(t)))
        return t.value

    def wait(self, timeout_ms=-1):
        """The next finished request as a dict, or None after timeout_ms."""
        r = Result()
        rc = lib().jq_server_wait(self.h, int(timeout_ms), ctypes.byref(r))
        if rc == JQ_EBUSY:
            return None
        check(rc)
        return {"ticket": r.ticket, "status": r.status, "n": r.n_qubits, "norm": r.norm,
                "latency_ms": r.latency_ms, "queue_ms": r.queue_ms, "state": r.state}

    def state(self, result):
        """Borrowed view of a finished request's state (valid until release)."""
        return State(result["n"], self.encoding, handle=result["state"])

    def release(self, ticket):
        check(lib().jq_server_release(self.h, int(ticket)))

    def stats(self):
        st = ServerStats()
        check(lib().jq_server_stats_get(self.h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self.h:
            h, self.h = self.h, None
            check(lib().jq_server_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------- torch memory --

_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_torch_hooks = None


def use_torch_allocator():
    """Route state allocations through torch's caching allocator."""
    global _torch_hooks
    import torch

    live = {}

    def _alloc(size, ctx):
        t = torch.empty(int(size), dtype=torch.uint8, device="cuda")
        live[t.data_ptr()] = t
        return t.data_ptr()

    def _free(ptr, ctx):
        live.pop(ptr, None)

    a, f = _ALLOC_T(_alloc), _FREE_T(_free)
    _torch_hooks = (a, f, live)
    check(lib().jq_set_allocator(ctypes.cast(a, _VP), ctypes.cast(f, _VP), None))


def use_hip_allocator():
    global _torch_hooks
    check(lib().jq_set_allocator(None, None, None))
    _torch_hooks = None

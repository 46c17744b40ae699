"""ctypes binding of the paper's OpenMP method (``oracle/paper_cpu.c``, Sec. 3.1).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): the multi-core CPU
baseline of the benchmark.  Gate records come from the oracle's own gate
table (``oracle.core.gate_records``).
"""
import ctypes
import os

import numpy as np

from . import core
from .build import PC_LIB, build

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("JQ_PAPERCPU_LIB")  # another build (the sanitizer build, say)
        if not path:
            path = PC_LIB
            if not os.path.exists(PC_LIB):
                build(force=False)
        L = ctypes.CDLL(path)
        L.pc_run.argtypes = [_dp, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
        L.pc_run_many.argtypes = [ctypes.POINTER(_dp), ctypes.POINTER(ctypes.c_int), ctypes.c_void_p,
                                  ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                  ctypes.c_int]
        L.pc_max_threads.argtypes = []
        _lib = L
    return _lib


def max_threads():
    return lib().pc_max_threads()


def run(psi, n, circuit, threads=0):
    """Apply a circuit of named gates in place with the Sec. 3.1 loop split
    on `threads` OpenMP threads (0: the OpenMP default)."""
    recs = core.gate_records(circuit)
    if len(recs):
        if lib().pc_run(psi.view(np.float64).ctypes.data_as(_dp), n, recs.ctypes.data, len(recs), threads):
            raise ValueError("invalid gate")
    return psi


def pack_many(circuits):
    """Gate records of many circuits, packed for run_many (lowering is done
    here, outside any timed call)."""
    recs = [core.gate_records(c) for c in circuits]
    counts = np.array([len(r) for r in recs], dtype=np.int32)
    first = np.zeros(len(recs), dtype=np.int64)
    first[1:] = np.cumsum(counts[:-1])
    allrecs = np.concatenate(recs) if len(recs) else np.zeros(0, dtype=core.GATE_DT)
    return allrecs, first, counts


def run_many(states, ns, circuits, threads=0):
    """Independent circuits (one thread each at a time), states updated in
    place; circuits is a list of gate lists or the result of pack_many."""
    allrecs, first, counts = circuits if isinstance(circuits, tuple) else pack_many(circuits)
    ptrs = (_dp * len(states))(*[s.view(np.float64).ctypes.data_as(_dp) for s in states])
    nn = np.ascontiguousarray(ns, dtype=np.int32)
    bad = lib().pc_run_many(ptrs, nn.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), allrecs.ctypes.data,
                            first.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(states), threads)
    if bad:
        raise ValueError(f"{bad} circuits had an invalid gate")
    return states

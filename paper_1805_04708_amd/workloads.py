"""Seeded synthetic circuits.

This module only draws random numbers and lays out gate lists; it does none
of the simulator's arithmetic.  A gate is a tuple
``(name, qubits, params[, controls])`` using the instruction names of the
paper's App. A (H, X, Z, S, T, CNOT, U(k), TOFFOLI, ...) plus RZ, CZ, CP and
explicit matrices (``MAT1``: 8 floats, row-major interleaved re/im).  Both
the GPU library and the CPU checker lower the names with their own tables.

Workloads (the paper's synthetic circuit families, Sec. 5, scaled to one GPU):

* ``random_circuit``  N qubits, G gates: half single-qubit gates drawn from
  {H, X, Z, S, T, Haar U(2)}, half CNOT / controlled-phase on a random ordered
  qubit pair (phase 2 pi / 2^k, k uniform in 1..10, i.e. the paper's U(k));
* ``layered_u2_cz``   each layer: Haar U(2) on every qubit, then CZ on a
  random perfect matching;
* ``rz_cnot_chain``   each layer: RZ(theta ~ U[0, 2 pi)) on every qubit, then
  the CNOT chain (0,1), (1,2), ..., (N-2,N-1) of Sec. 5.2;
* ``hadamard_all`` / ``ghz``  the two validation circuits of Sec. 5.1/5.2;
* ``qft``             the quantum Fourier transform from H and U(k), the
  construction the paper recalls in Sec. 4.2, followed by qubit reversal;
* ``serving_trace``   Poisson arrivals of layered random circuits with N drawn
  with weight 2^(-N/2).

Haar-random U(2) matrices use the QR decomposition of a complex Ginibre
matrix with the phases of R's diagonal divided out (Mezzadri, Notices AMS
54 (2007) 592).
"""
import math

import numpy as np

SINGLE_KINDS = ("H", "X", "Z", "S", "T", "U2H")


def haar_u2(rng):
    """A Haar-random 2x2 unitary as the 8-float MAT1 parameter list."""
    z = (rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    q = q * (d / np.abs(d))
    out = np.empty(8)
    out[0::2] = q.real.ravel()
    out[1::2] = q.imag.ravel()
    return tuple(float(x) for x in out)


def random_circuit(n, n_gates, seed):
    """Random circuit of the 16-qubit / 100..200-gate workloads."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_gates):
        if rng.random() < 0.5 or n < 2:
            kind = SINGLE_KINDS[int(rng.integers(len(SINGLE_KINDS)))]
            q = int(rng.integers(n))
            if kind == "U2H":
                out.append(("MAT1", (q,), haar_u2(rng)))
            else:
                out.append((kind, (q,), ()))
        else:
            a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
            if rng.random() < 0.5:
                out.append(("CNOT", (a, b), ()))
            else:
                k = int(rng.integers(1, 11))
                out.append(("CP", (a, b), (2.0 * math.pi / 2 ** k,)))
    return out


def layered_u2_cz(n, layers, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(layers):
        for q in range(n):
            out.append(("MAT1", (q,), haar_u2(rng)))
        perm = rng.permutation(n)
        for i in range(0, n - 1, 2):
            out.append(("CZ", (int(perm[i]), int(perm[i + 1])), ()))
    return out


def rz_cnot_chain(n, layers, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(layers):
        for q in range(n):
            out.append(("RZ", (q,), (float(rng.uniform(0.0, 2.0 * math.pi)),)))
        for q in range(n - 1):
            out.append(("CNOT", (q, q + 1), ()))
    return out


def hadamard_all(n):
    return [("H", (q,), ()) for q in range(n)]


def ghz(n):
    return [("H", (0,), ())] + [("CNOT", (q, q + 1), ()) for q in range(n - 1)]


def qft(n):
    """QFT: for j = N-1 down to 0, H on j then U(k = j-m+1) controlled by
    each lower qubit m; then reverse the qubit order with SWAPs."""
    out = []
    for j in range(n - 1, -1, -1):
        out.append(("H", (j,), ()))
        for m in range(j - 1, -1, -1):
            out.append(("U", (m, j), (j - m + 1,)))
    for q in range(n // 2):
        out.append(("SWAP", (q, n - 1 - q), ()))
    return out


def batch_instances(count, base_seed, n_lo=8, n_hi=16, n_gates=100):
    """Independent small circuits: N uniform in [n_lo, n_hi], seed base+i."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(base_seed + i)
        n = int(rng.integers(n_lo, n_hi + 1))
        out.append((n, random_circuit(n, n_gates, base_seed + i)))
    return out


def layered_random(n, depth, rng):
    """Layers of random single-qubit gates on every qubit plus CZ on a random
    matching, until `depth` gates are placed."""
    out = []
    while len(out) < depth:
        for q in range(n):
            kind = SINGLE_KINDS[int(rng.integers(len(SINGLE_KINDS)))]
            out.append(("MAT1", (q,), haar_u2(rng)) if kind == "U2H" else (kind, (q,), ()))
        perm = rng.permutation(n)
        for i in range(0, n - 1, 2):
            out.append(("CZ", (int(perm[i]), int(perm[i + 1])), ()))
    return out[:depth]


def serving_trace(count, rate_hz, seed, n_lo=10, n_hi=28, d_lo=20, d_hi=200):
    """Poisson arrivals at rate_hz; returns [(t_arrival_s, n, circuit)]."""
    rng = np.random.default_rng(seed)
    ns = np.arange(n_lo, n_hi + 1)
    w = 2.0 ** (-ns / 2.0)
    w /= w.sum()
    t = 0.0
    out = []
    for _ in range(count):
        t += float(rng.exponential(1.0 / rate_hz))
        n = int(rng.choice(ns, p=w))
        d = int(rng.integers(d_lo, d_hi + 1))
        out.append((t, n, layered_random(n, d, rng)))
    return out

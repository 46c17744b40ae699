"""Oracle for the Shor workload (Sec. 5.3; App. A, SHORBOX).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU leg, never by the product library.

SHORBOX prepares 2^(-n_x/2) sum_x |x>|y^x mod G>: the x-register holds the
n_x low qubits (x's least significant bit on qubit 0) and the f-register the
qubits above (the garbled upper summation limit is read as 2^n_x - 1).  The
quantum Fourier transform on the x-register then maps each f-branch
independently, so the x-register's single-qubit expectation values are sums
over the residues f of terms computed from a length-2^n_x discrete Fourier
transform (numpy's FFT) of that branch.
"""
import numpy as np


def orbit(n_x, G, y):
    """f(x) = y^x mod G for x = 0 .. 2^n_x - 1 (repeated multiplication)."""
    out = np.empty(1 << n_x, dtype=np.int64)
    cur = 1
    for x in range(1 << n_x):
        out[x] = cur
        cur = cur * y % G
    return out


def shorbox_state(n, n_x, G, y):
    """The SHORBOX state on n qubits as a complex128 vector."""
    if not (1 <= n_x < n) or G > (1 << (n - n_x)):
        raise ValueError("registers do not fit")
    psi = np.zeros(1 << n, dtype=np.complex128)
    x = np.arange(1 << n_x, dtype=np.int64)
    psi[x + (orbit(n_x, G, y) << n_x)] = 2.0 ** (-n_x / 2)
    return psi


def qft_expectations(n_x, G, y):
    """<Qx(i)>, <Qy(i)>, <Qz(i)> (App. A, BEGIN MEASUREMENT) of the x-register
    qubits after SHORBOX and the quantum Fourier transform on the x-register
    (output amplitude k = 2^(-n_x/2) sum_x e^(2 pi i x k / 2^n_x) in_x).
    Branches with different f are orthogonal, so the expectations add over
    f; within a branch sigma^x_q pairs k with k xor 2^q."""
    M = 1 << n_x
    f = orbit(n_x, G, y)
    k = np.arange(M, dtype=np.int64)
    sx, sy, sz = np.zeros(n_x), np.zeros(n_x), np.zeros(n_x)
    for r in np.unique(f):
        v = np.where(f == r, 2.0 ** (-n_x / 2), 0.0).astype(np.complex128)
        out = np.fft.ifft(v) * np.sqrt(M)
        p = np.abs(out) ** 2
        for q in range(n_x):
            bit = (k >> q) & 1
            partner = out[k ^ (1 << q)]
            sx[q] += np.vdot(out, partner).real
            # sigma^y maps |0> to i|1> and |1> to -i|0>
            sy[q] += np.vdot(out, np.where(bit == 1, 1j, -1j) * partner).real
            sz[q] += np.sum(np.where(bit == 1, -p, p))
    return (1 - sx) / 2, (1 - sy) / 2, (1 - sz) / 2

"""The oracle's gate table: named instructions -> explicit matrices.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Every matrix is written out from the instruction set of App. A.  For
multi-qubit instructions the matrix is in the basis |q0, q1, ...> with the
first-listed qubit as the most significant bit, as App. A states for CNOT,
U(k) and TOFFOLI ("in the computational basis |control,target>").  No
instruction is special-cased: CNOT is its 4x4 matrix on (control, target),
TOFFOLI its 8x8 matrix.

Gates the workloads use that App. A does not define:

* ``RZ q theta``  = diag(exp(-i theta/2), exp(+i theta/2)) (the usual
  z-rotation; App. A has only U1, which differs from it by a global phase);
* ``CZ a b``      = U(k=1) of App. A, i.e. diag(1, 1, 1, -1);
* ``CP a b phi``  = diag(1, 1, 1, exp(i phi)), which is U(k) for phi = 2 pi/2^k;
* ``SWAP a b``    = the 4x4 exchange of |01> and |10>;
* ``MAT1 q m..``  and ``MAT2 a b m..``: an explicit 2x2 / 4x4 matrix given
  as 8 / 32 floats, row-major interleaved (re, im).

A gate is a tuple ``(name, qubits, params[, controls])``; extra controls
restrict the gate to the subspace where all of them are 1.
"""
import cmath
import math

import numpy as np

SQ2 = 1.0 / math.sqrt(2.0)


def _m(rows):
    return np.array(rows, dtype=np.complex128)


def _phase(a):
    return cmath.exp(1j * a)


def matrix(name, params=()):
    """Matrix of a named gate (App. A), as a 2^k x 2^k complex ndarray."""
    p = [float(x) for x in params]
    n = name.upper()
    if n == "I":
        return _m([[1, 0], [0, 1]])
    if n == "H":
        return SQ2 * _m([[1, 1], [1, -1]])
    if n == "X":
        return _m([[0, 1], [1, 0]])
    if n == "Y":
        return _m([[0, -1j], [1j, 0]])
    if n == "Z":
        return _m([[1, 0], [0, -1]])
    if n == "S":
        return _m([[1, 0], [0, 1j]])
    if n == "S+":
        return _m([[1, 0], [0, -1j]])
    if n == "T":
        return _m([[1, 0], [0, (1 + 1j) * SQ2]])
    if n == "T+":
        return _m([[1, 0], [0, (1 - 1j) * SQ2]])
    if n == "U1":
        (lam,) = p
        return _m([[1, 0], [0, _phase(lam)]])
    if n == "U2":
        phi, lam = p
        return SQ2 * _m([[1, -_phase(lam)], [_phase(phi), _phase(phi + lam)]])
    if n == "U3":
        th, phi, lam = p
        c, s = math.cos(th / 2), math.sin(th / 2)
        return _m([[c, -_phase(lam) * s], [_phase(phi) * s, _phase(phi + lam) * c]])
    if n == "+X":
        return SQ2 * _m([[1, 1j], [1j, 1]])
    if n == "-X":
        return SQ2 * _m([[1, -1j], [-1j, 1]])
    if n == "+Y":
        return SQ2 * _m([[1, 1], [-1, 1]])
    if n == "-Y":
        return SQ2 * _m([[1, -1], [1, 1]])
    if n == "R":
        # R(k) and, for a negative argument, its inverse (App. A: "R n -k").
        (k,) = p
        k = int(k)
        sign = -1.0 if k < 0 else 1.0
        return _m([[1, 0], [0, _phase(sign * 2 * math.pi / 2 ** abs(k))]])
    if n == "RZ":
        (th,) = p
        return _m([[_phase(-th / 2), 0], [0, _phase(th / 2)]])
    if n == "CNOT":
        return _m([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]])
    if n == "U":
        (k,) = p
        k = int(k)
        sign = -1.0 if k < 0 else 1.0
        return np.diag([1, 1, 1, _phase(sign * 2 * math.pi / 2 ** abs(k))]).astype(np.complex128)
    if n == "CZ":
        return np.diag([1, 1, 1, -1]).astype(np.complex128)
    if n == "CP":
        (phi,) = p
        return np.diag([1, 1, 1, _phase(phi)]).astype(np.complex128)
    if n == "SWAP":
        return _m([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]])
    if n == "TOFFOLI":
        m = np.eye(8, dtype=np.complex128)
        m[6, 6] = m[7, 7] = 0
        m[6, 7] = m[7, 6] = 1
        return m
    if n in ("MAT1", "MAT2"):
        k = 1 if n == "MAT1" else 2
        K = 1 << k
        a = np.array(p, dtype=np.float64)
        if a.size != 2 * K * K:
            raise ValueError(f"{n} needs {2 * K * K} floats")
        return (a[0::2] + 1j * a[1::2]).reshape(K, K)
    raise ValueError(f"unknown gate {name!r}")


def lower(gate):
    """(name, qubits, params[, controls]) -> (targets, controls, matrix)."""
    name, qubits, params = gate[0], tuple(gate[1]), tuple(gate[2])
    controls = tuple(gate[3]) if len(gate) > 3 else ()
    m = matrix(name, params)
    if m.shape[0] != 1 << len(qubits):
        raise ValueError(f"{name} acts on {m.shape[0].bit_length() - 1} qubits, got {qubits}")
    return qubits, controls, m

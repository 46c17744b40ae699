"""Oracle for the auxiliary-variable method (Sec. 4.2, Eqs. appa2-appa7).

TEST INFRASTRUCTURE ONLY: imported by tests/ and the benchmark's CPU leg,
never by the product library.  Plain Python and numpy, FP64, small P only.

Steps, in the order of Sec. 4.2:
1. single-qubit gates act on one qubit's two-component state (Eq. appa1);
   the circuit starts from the product state |0...0> (Eq. appa0);
2. every controlled phase shift U(a) (Eq. appa4) - CNOT being
   H_t U(pi) H_t on its target - is written with a two-valued variable s as
   (1/2) sum_s exp(i (sigma^z_0 + sigma^z_1)(x s - a/4)), cos 2x = exp(ia/2)
   (Eqs. appa5, appa6): on each of its two qubits a diagonal single-qubit
   factor diag(exp(i(xs - a/4)), exp(-i(xs - a/4)));
3. for each assignment of the P variables every qubit evolves alone, and
   the state is 2^-P times the sum over assignments of the product states
   (Eq. appa7); an amplitude <b|psi> multiplies the qubits' components b_j.
"""
import cmath
import itertools

import numpy as np

from . import gates as G

CONTROLLED_PHASE = {"CZ": lambda p: cmath.pi, "U": lambda p: 2 * cmath.pi / 2 ** int(p[0]),
                    "CP": lambda p: float(p[0])}


def program(circuit, n):
    """Per-qubit item lists: ("M", 2x2 matrix) or ("S", p, sign of sigma^z
    eigenvalue convention); returns (items, xs, as_) with one x and one a per
    variable."""
    items = [[] for _ in range(n)]
    xs, as_ = [], []

    def phase(a, q0, q1):
        p = len(xs)
        x = cmath.acos(cmath.exp(0.5j * a)) / 2
        xs.append(x)
        as_.append(a)
        items[q0].append(("S", p))
        items[q1].append(("S", p))

    for g in circuit:
        name, q, par = g[0], tuple(g[1]), tuple(g[2])
        if len(g) > 3 and g[3]:
            raise ValueError("extra controls are not supported")
        if name in CONTROLLED_PHASE:
            phase(CONTROLLED_PHASE[name](par), q[0], q[1])
        elif name == "CNOT":
            h = G.matrix("H", ())
            items[q[1]].append(("M", h))
            phase(cmath.pi, q[0], q[1])
            items[q[1]].append(("M", h))
        elif name == "I":
            continue
        else:
            m = G.matrix(name, par)
            if m.shape != (2, 2):
                raise ValueError(f"{name} is not a single-qubit gate")
            items[q[0]].append(("M", m))
    return items, xs, as_


def amplitudes(circuit, n, basis):
    """<b|psi> for each b in basis, psi = circuit |0...0>, by Eq. appa7."""
    items, xs, as_ = program(circuit, n)
    P = len(xs)
    basis = [int(b) for b in basis]
    out = np.zeros(len(basis), dtype=np.complex128)
    for s in itertools.product((1, -1), repeat=P):
        comps = []
        for j in range(n):
            v = np.array([1.0 + 0j, 0.0 + 0j])
            for it in items[j]:
                if it[0] == "M":
                    v = it[1] @ v
                else:
                    p = it[1]
                    e = cmath.exp(1j * (xs[p] * s[p] - as_[p] / 4))
                    # sigma^z is +1 on |0>, -1 on |1>
                    v = np.array([v[0] * e, v[1] / e])
            comps.append(v)
        for k, b in enumerate(basis):
            t = 1.0 + 0j
            for j in range(n):
                t *= comps[j][(b >> j) & 1]
            out[k] += t
    return out / 2 ** P

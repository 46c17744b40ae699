"""Dense brute force: build the full 2^N x 2^N gate matrix and multiply.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  For N <= 8.

Sec. 2 writes a single-qubit gate on qubit j as the Kronecker product
1_0 x ... x U_j x ... x 1_{N-1} acting on the whole vector.  Here that product
is taken literally with ``numpy.kron``: a 2^k x 2^k matrix is expanded into
sums of one-qubit operators |a><b| (one factor per target), and controls
contribute the projector |1><1| on the controlled part and 1 - P on the rest.
Qubit 0 is the least significant bit of the basis index (Sec. 2), so in the
Kronecker chain the factor for qubit N-1 comes first.  This code never
looks at index bits, so it checks the oracle's bit loops independently.
"""
import itertools

import numpy as np

E = {(a, b): np.array([[1.0 if (r, c) == (a, b) else 0.0 for c in (0, 1)] for r in (0, 1)],
                      dtype=np.complex128) for a in (0, 1) for b in (0, 1)}
I2 = np.eye(2, dtype=np.complex128)
P1 = E[(1, 1)]


def _chain(n, factors):
    """Kronecker product over qubits N-1 .. 0 of factors[q] (default 1)."""
    out = np.ones((1, 1), dtype=np.complex128)
    for q in range(n - 1, -1, -1):
        out = np.kron(out, factors.get(q, I2))
    return out


def full_matrix(n, targets, controls, m):
    """The 2^N x 2^N matrix of gate m on targets (first = MSB), controlled."""
    k = len(targets)
    K = 1 << k
    G = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    ctrl = {c: P1 for c in controls}
    for r, c in itertools.product(range(K), range(K)):
        if m[r, c] == 0:
            continue
        f = dict(ctrl)
        for s, t in enumerate(targets):
            bit_r = (r >> (k - 1 - s)) & 1
            bit_c = (c >> (k - 1 - s)) & 1
            f[t] = E[(bit_r, bit_c)]
        G += m[r, c] * _chain(n, f)
    if controls:
        # 1 - P_controls on the whole space, identity on the targets there.
        G += np.eye(1 << n, dtype=np.complex128) - _chain(n, ctrl)
    return G


def apply(psi, n, targets, controls, m):
    return full_matrix(n, targets, controls, m) @ psi

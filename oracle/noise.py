"""Oracle for the depolarizing channel (App. A, DEPOLARIZING CHANNEL).

TEST INFRASTRUCTURE ONLY: imported by tests/ and the benchmark's CPU leg,
never by the product library.

After each gate of the circuit (identity gates included), every qubit q gets
an X gate with probability p_x, a Y gate with probability p_y or a Z gate
with probability p_z.  One draw u in [0, 1) per gate and qubit, supplied by
the caller (u[g * N + q]), decides: X if u < p_x, Y if p_x <= u < p_x + p_y,
Z if p_x + p_y <= u < p_x + p_y + p_z, nothing otherwise.
"""
import numpy as np


def expand(circuit, n, px, py, pz, u):
    """The circuit with the channel's Pauli gates written out."""
    u = np.asarray(u, dtype=np.float64)
    if len(u) != len(circuit) * n:
        raise ValueError("one draw per gate and qubit")
    out = []
    for g, gate in enumerate(circuit):
        out.append(gate)
        for q in range(n):
            x = u[g * n + q]
            if x < px:
                out.append(("X", (q,), ()))
            elif x < px + py:
                out.append(("Y", (q,), ()))
            elif x < px + py + pz:
                out.append(("Z", (q,), ()))
    return out

"""Pins of the auxiliary-variable oracle (Sec. 4.2): the discrete
Hubbard-Stratonovich identity of Eq. appa6 checked numerically, the product
state of Eq. appa2, and agreement with the state-vector oracle on small
circuits of single-qubit gates, CNOT and controlled phase shifts."""
import cmath
import math

import numpy as np
import pytest

from oracle import aux as A
from oracle import core as O
from paper_1805_04708_amd import workloads as W


@pytest.mark.parametrize("a", [math.pi, math.pi / 2, 2 * math.pi / 32, 0.37, -1.2])
def test_hubbard_stratonovich_identity(a):
    # (1/2) sum_s exp(i (sigma_0 + sigma_1)(x s - a/4)) = diag(1, 1, 1, e^{ia})
    x = cmath.acos(cmath.exp(0.5j * a)) / 2
    assert abs(cmath.cos(2 * x) - cmath.exp(0.5j * a)) < 1e-14
    for (s0, s1), want in (((1, 1), 1), ((1, -1), 1), ((-1, 1), 1), ((-1, -1), cmath.exp(1j * a))):
        got = 0.5 * sum(cmath.exp(1j * (s0 + s1) * (x * s - a / 4)) for s in (1, -1))
        assert abs(got - want) < 1e-14


def test_product_state_without_entangling_gates():
    n = 5
    rng = np.random.default_rng(2)
    circ = [("MAT1", (q,), W.haar_u2(rng)) for q in range(n)] + [("T", (1,), ()), ("H", (3,), ())]
    ref = O.run(O.zero_state(n), n, circ)
    got = A.amplitudes(circ, n, range(1 << n))
    assert np.max(np.abs(got - ref)) < 1e-14


def mixed_circuit(n, n_single, n_pairs, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_single + n_pairs):
        if i % 3 != 2 or n_pairs == 0:
            q = int(rng.integers(n))
            out.append(("MAT1", (q,), W.haar_u2(rng)) if rng.random() < 0.5 else ("H", (q,), ()))
        else:
            n_pairs -= 1
            a, b = (int(x) for x in rng.permutation(n)[:2])
            kind = int(rng.integers(4))
            out.append([("CNOT", (a, b), ()), ("CZ", (a, b), ()), ("U", (a, b), (int(rng.integers(1, 6)),)),
                        ("CP", (a, b), (float(rng.uniform(-3, 3)),))][kind])
    return out


@pytest.mark.parametrize("n,pairs,seed", [(4, 3, 1), (6, 6, 2), (8, 8, 3)])
def test_matches_state_vector(n, pairs, seed):
    circ = mixed_circuit(n, 3 * n, pairs, seed)
    ref = O.run(O.zero_state(n), n, circ)
    got = A.amplitudes(circ, n, range(1 << n))
    assert np.max(np.abs(got - ref)) < 1e-12


def test_unsupported_gates():
    with pytest.raises(ValueError):
        A.program([("SWAP", (0, 1), ())], 2)
    with pytest.raises(ValueError):
        A.program([("TOFFOLI", (0, 1, 2), ())], 3)

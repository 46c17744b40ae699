"""The paper's OpenMP method (Sec. 3.1, ``oracle/paper_cpu.c``), the CPU
baseline of the benchmark, pinned to the single-threaded oracle.

Both implement Eq. NUM2 and its group generalisation with the same
arithmetic, so every state must be identical bit for bit, whatever the
thread count and whichever side of the paper's outer/inner test a target
falls on (low targets parallelise the outer loop, high ones the inner).
"""
import math

import numpy as np
import pytest

from oracle import core as O
from oracle import paper_cpu as PC
from paper_1805_04708_amd import workloads as W


def rand_state(rng, n):
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return psi / np.linalg.norm(psi)


def mixed_circuit(rng, n, count):
    """One- to three-qubit gates, controls, explicit matrices, every target."""
    out = []
    for _ in range(count):
        r = rng.random()
        q = [int(x) for x in rng.choice(n, size=min(n, 5), replace=False)]
        if r < 0.3:
            out.append(("MAT1", (q[0],), W.haar_u2(rng)))
        elif r < 0.45 and n >= 2:
            m = rng.standard_normal(32)
            out.append(("MAT2", (q[0], q[1]), tuple(float(x) for x in m)))
        elif r < 0.55 and n >= 3:
            out.append(("TOFFOLI", (q[0], q[1], q[2]), ()))
        elif r < 0.7 and n >= 2:
            out.append(("CNOT", (q[0], q[1]), ()))
        elif r < 0.8 and n >= 2:
            out.append(("CP", (q[0], q[1]), (float(rng.uniform(0, 2 * math.pi)),)))
        elif r < 0.9 and n >= 4:
            out.append(("H", (q[0],), (), (q[1], q[2])))
        else:
            out.append(("T", (q[0],), ()))
    return out


@pytest.mark.parametrize("n", [1, 2, 5, 9, 12])
@pytest.mark.parametrize("threads", [1, 3, 8])
def test_openmp_method_is_bit_identical_to_the_oracle(n, threads):
    rng = np.random.default_rng(100 * n + threads)
    circ = mixed_circuit(rng, n, 60)
    start = rand_state(rng, n)
    ref = O.run(start.copy(), n, circ)
    got = PC.run(start.copy(), n, circ, threads=threads)
    assert np.array_equal(ref.view(np.uint64), got.view(np.uint64))


def test_every_target_on_both_sides_of_the_loop_test():
    # N = 11: targets 0..4 pass nstates/(i+i) >= i (outer loop shared),
    # 5..10 do not (inner loop shared)
    n = 11
    nstates = 1 << (n - 1)
    sides = {(nstates // (2 << t)) >= (1 << t) for t in range(n)}
    assert sides == {True, False}
    rng = np.random.default_rng(3)
    start = rand_state(rng, n)
    for t in range(n):
        circ = [("MAT1", (t,), W.haar_u2(rng))]
        ref = O.run(start.copy(), n, circ)
        got = PC.run(start.copy(), n, circ, threads=4)
        assert np.array_equal(ref.view(np.uint64), got.view(np.uint64)), t


def test_many_circuits_match_one_at_a_time():
    rng = np.random.default_rng(11)
    ns = [int(x) for x in rng.integers(3, 10, size=24)]
    circs = [W.random_circuit(n, 40, 500 + i) for i, n in enumerate(ns)]
    states = [O.zero_state(n) for n in ns]
    PC.run_many(states, ns, circs, threads=4)
    for n, c, s in zip(ns, circs, states):
        assert np.array_equal(s.view(np.uint64), O.run(O.zero_state(n), n, c).view(np.uint64))


def test_invalid_gate_is_reported():
    with pytest.raises(ValueError):
        PC.run(O.zero_state(3), 3, [("CNOT", (1, 1), ())])

"""Host-side checks of the benchmark's measurement helpers (no GPU): the
closed form it holds 256 GiB RZ + CNOT-chain states to, and the error
metrics it reports for reduced-precision states."""
import numpy as np

import bench
from oracle import core as O
from paper_1805_04708_amd import workloads as W


def test_rz_cnot_closed_form_matches_the_oracle():
    n = 9
    circ = W.rz_cnot_chain(n, 4, seed=3)
    psi = O.run(O.uniform_state(n), n, circ)
    seen = set()
    for j in range(1 << n):
        i, amp = bench.rz_cnot_closed_form(n, circ, j)
        seen.add(i)
        assert abs(psi[i] - amp) <= 1e-15
    assert len(seen) == 1 << n  # the CNOT chain permutes the basis


class _FakeState:
    def __init__(self, a):
        self.a = a

    def amplitudes(self, first, count):
        return self.a[first:first + count]


def test_compare_states_metrics():
    rng = np.random.default_rng(2)
    n = 10
    ref = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    got = ref * np.exp(0.3j) * 1.5  # global phase and scale: fidelity 1
    r = bench.compare_states(_FakeState(got), _FakeState(ref), n, chunk=100)
    assert abs(r["fidelity"] - 1.0) < 1e-12
    assert abs(r["rel_l2"] - np.linalg.norm(got - ref) / np.linalg.norm(ref)) < 1e-12
    noisy = ref + 1e-3 * (rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n))
    r = bench.compare_states(_FakeState(noisy), _FakeState(ref), n, chunk=1 << n)
    assert abs(r["fidelity"] - O.fidelity(noisy, ref)) < 1e-12
    assert abs(r["rel_l2"] - O.rel_l2(noisy, ref)) < 1e-12

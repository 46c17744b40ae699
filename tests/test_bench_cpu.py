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


def test_metrics_log_records(tmp_path):
    import json
    out = {"metric": "m", "value": 1.5, "unit": "gates/s", "config": {"workload": "w", "seed": 3},
           "kernels": {"fused": {"launches_per_step": 54.0}}, "roofline": {"frac": 0.5, "traffic": 7.0},
           "higher_is_better": True, "c64_same_circuit": {"rel_l2_vs_c128": 1e-6},
           "cpu_baseline": {"value": 0.3, "cores": 1}}
    path = tmp_path / "m.jsonl"
    bench.write_metrics_log(str(path), out)
    bench.write_metrics_log(str(path), out)
    recs = [json.loads(line) for line in path.read_text().splitlines()]
    assert len(recs) == 6 and len({r["run"] for r in recs}) == 2
    head = recs[0]
    assert head["workload"] == "headline" and head["value"] == 1.5 and head["fused_passes_per_step"] == 54.0
    assert head["config"]["seed"] == 3 and head["frac_of_hbm_peak"] == 0.5
    assert {r["workload"] for r in recs[1:3]} == {"c64_same_circuit", "cpu_baseline"}

"""The library's debug switches (environment variables read once per
process, so each case runs in a child process): JQ_FORCE_KERNEL forces one
kernel per gate or a fused pass for every run of fusable gates; an unknown
value changes nothing."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SNIPPET = """
import json, sys
sys.path.insert(0, {root!r})
from paper_1805_04708_amd import jq, workloads as W
circ = W.random_circuit(12, 60, 1)
steps = jq.plan_steps(12, "c128", circ)
single = jq.plan_steps(12, "c128", [("H", (5,), ())])
print(json.dumps({{"fused": sum(s["fused"] for s in steps), "steps": len(steps),
                   "single_fused": single[0]["fused"]}}))
"""


def plan_with(env_value):
    env = dict(os.environ)
    env.pop("JQ_FORCE_KERNEL", None)
    if env_value is not None:
        env["JQ_FORCE_KERNEL"] = env_value
    r = subprocess.run([sys.executable, "-c", SNIPPET.format(root=ROOT)], env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_force_kernel_class():
    base = plan_with(None)
    assert base["fused"] >= 1 and not base["single_fused"]
    per_gate = plan_with("per_gate")
    assert per_gate["fused"] == 0 and per_gate["steps"] == 60
    fused = plan_with("fused")
    assert fused["single_fused"] and fused["fused"] >= base["fused"]
    assert plan_with("something else") == base

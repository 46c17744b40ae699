"""GPU tests of jq_autotune: measured values lie in range, are written to
and read back from the cache file, and the plans they give (and extreme
settings of every tuned value) still match the oracle."""
import json

import numpy as np
import pytest

from oracle import core as O
from paper_1805_04708_amd import jq
from paper_1805_04708_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    jq.lib()


@pytest.fixture(autouse=True)
def _cache(tmp_path, monkeypatch):
    path = tmp_path / "tuning.json"
    monkeypatch.setenv("JQ_TUNE_CACHE", str(path))
    yield path
    for n in (14, 16, 17):
        for enc in ("c128", "c64"):
            jq.tuning_set(n, enc, clear=True)


TOL = {"c128": 1e-12, "c64": 2e-6}


@pytest.mark.parametrize("enc", ["c128", "c64"])
def test_autotune_measures_caches_and_matches_the_oracle(enc, _cache):
    n = 16
    print(f"autotune n={n} enc={enc}", flush=True)
    t = jq.autotune(n, enc, force=True)
    assert t["source"] == "measured" and t["n_qubits"] == n
    assert 3 <= t["k_reg"] <= (6 if enc == "c64" else 5)
    assert 0 < t["pass_ops"] <= 10000 and 0 <= t["wide_target"] <= 64
    assert 0 < t["tuned_ms"] <= t["default_ms"] * 1.0000001
    assert jq.tuning_get(n, enc)["k_reg"] == t["k_reg"]
    # written to the cache file under this device's key, and read back
    data = json.loads(_cache.read_text())
    (e,) = [x for x in data["entries"] if x["n"] == n and x["encoding"] == enc]
    assert e["device"] != "host" and e["k_reg"] == t["k_reg"] and e["wide_target"] == t["wide_target"]
    # the per-target widths: chosen from target 8 up, the file holding the
    # targets below 53
    assert e["wide_mask"] == t["wide_mask"] & (2**53 - 1)
    assert t["wide_target"] == (64 if t["wide_mask"] == 0 else (t["wide_mask"] & -t["wide_mask"]).bit_length() - 1)
    jq.tuning_set(n, enc, clear=True)
    c = jq.autotune(n, enc)
    assert c["source"] == "cached" and c["k_reg"] == t["k_reg"]
    # tuning on the caller's workload, then that workload's plan against
    # the oracle
    circ = W.layered_u2_cz(n, 6, seed=16) + W.random_circuit(n, 150, seed=17)
    w = jq.autotune(n, enc, circ, force=True, no_cache=True)
    assert w["source"] == "measured" and jq.tuning_get(n, enc)["k_reg"] == w["k_reg"]
    t = w
    ref = O.run(O.zero_state(n), n, circ)
    with jq.State(n, enc) as s:
        s.apply_circuit(circ)
        assert O.rel_l2(s.amplitudes(), ref) <= TOL[enc] * 2
        steps = jq.plan_steps(n, enc, circ)
        # the random part holds CNOTs and controlled phases: the planner keeps
        # such circuits at the widest width of 4 waves per SIMD for the kernel
        # compiled for every op kind
        cap = 5 if enc == "c64" else 4
        assert {st["k_reg"] for st in steps if st["fused"]} <= {min(t["k_reg"], cap)}


@pytest.mark.parametrize("enc", ["c128", "c64"])
def test_every_tuned_value_keeps_oracle_parity(enc):
    n = 17
    circ = W.layered_u2_cz(n, 4, seed=3) + W.random_circuit(n, 120, seed=4)
    ref = O.run(O.zero_state(n), n, circ)
    for k in range(2, (6 if enc == "c64" else 5) + 1):
        for ops in (1.0, 19.0, 500.0):
            jq.tuning_set(n, enc, k_reg=k, pass_ops=ops)
            with jq.State(n, enc) as s:
                s.apply_circuit(circ)
                assert O.rel_l2(s.amplitudes(), ref) <= TOL[enc] * 2, (k, ops)
    # per-gate kernels: one pair per thread everywhere, four everywhere,
    # from target 9 up, and a mask that alternates target by target
    for wide in (0, 64, 9):
        jq.tuning_set(n, enc, wide_target=wide)
        with jq.State(n, enc) as s:
            s.apply_circuit(circ, fusion=1)
            assert O.rel_l2(s.amplitudes(), ref) <= TOL[enc] * 2, wide
    jq.tuning_set(n, enc, wide_mask=int("01" * 16, 2))
    with jq.State(n, enc) as s:
        s.apply_circuit(circ, fusion=1)
        assert O.rel_l2(s.amplitudes(), ref) <= TOL[enc] * 2

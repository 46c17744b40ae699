"""Host-side checks of the single-state tuning table (no GPU): built-in
defaults, the JSON cache file (exact size, the streaming-size fallback,
malformed files), in-process overrides and their validation, and the
planner picking the tuned register width.  Without a GPU the device is
"host", so cache entries for it apply here."""
import json

import pytest

from paper_1805_04708_amd import jq
from paper_1805_04708_amd import workloads as W
from paper_1805_04708_amd.build import ensure_built


@pytest.fixture(autouse=True)
def _cache(tmp_path, monkeypatch):
    ensure_built()
    path = tmp_path / "tuning.json"
    monkeypatch.setenv("JQ_TUNE_CACHE", str(path))
    yield path
    for n in (18, 20, 26, 28, 30):
        for enc in ("c128", "c64"):
            jq.tuning_set(n, enc, clear=True)


def entry(n, enc="c128", k=3, ops=7.5, wide=12, device="host"):
    return {"device": device, "encoding": enc, "n": n, "k_reg": k, "pass_ops": ops, "wide_target": wide,
            "tuned_ms": 1.0, "default_ms": 2.0}


def write(path, entries, version=1):
    path.write_text(json.dumps({"version": version, "entries": entries}))


def test_defaults_without_a_cache_file():
    # complex128: one pair per thread on every target; complex64: four from 17 up
    for enc, k, ops, wide, mask in (("c128", 5, 19.0, 64, 0), ("c64", 6, 6.0, 17, (2**64 - 1) ^ (2**17 - 1))):
        t = jq.tuning_get(30, enc)
        assert (t["k_reg"], t["pass_ops"], t["wide_target"], t["wide_mask"], t["source"]) == \
            (k, ops, wide, mask, "default")


def test_cache_exact_size_and_streaming_fallback(_cache):
    write(_cache, [entry(26, k=3), entry(28, k=5, ops=30.0), entry(20, k=2), entry(28, "c64", k=6, wide=64),
                   entry(28, device="gfx950:another device", k=2)])
    t = jq.tuning_get(28, "c128")
    assert (t["k_reg"], t["pass_ops"], t["wide_target"], t["source"], t["n_qubits"]) == (5, 30.0, 12, "cached", 28)
    # N >= 25 without an entry: the largest tuned size from 25 up to N
    assert jq.tuning_get(34, "c128")["k_reg"] == 5
    assert jq.tuning_get(27, "c128")["k_reg"] == 3
    assert jq.tuning_get(25, "c128")["source"] == "default"
    # below 25 only an exact entry applies
    assert jq.tuning_get(20, "c128")["k_reg"] == 2
    assert jq.tuning_get(21, "c128")["source"] == "default"
    assert jq.tuning_get(28, "c64")["wide_target"] == 64
    # the two-byte code is not tuned
    assert jq.tuning_get(28, "compact")["source"] == "default"


@pytest.mark.parametrize("text", [
    "", "{", "not json", '{"version": 2, "entries": []}', '{"entries": [{"device": "host"}]}',
    '{"version": 1, "entries": [{"device": "host", "encoding": "c128", "n": 28, "k_reg": 9, '
    '"pass_ops": 5, "wide_target": 3}]}',
    '{"version": 1, "entries": [{"device": "host", "encoding": "c128", "n": 28, "k_reg": 3, '
    '"pass_ops": 5, "wide_target": 3}]} trailing',
])
def test_malformed_cache_files_count_as_empty(_cache, text):
    _cache.write_text(text)
    assert jq.tuning_get(28, "c128")["source"] == "default"


def test_overrides_win_and_are_validated(_cache):
    write(_cache, [entry(28, k=5)])
    jq.tuning_set(28, "c128", k_reg=3, pass_ops=40.0, wide_target=20)
    t = jq.tuning_get(28, "c128")
    assert (t["k_reg"], t["pass_ops"], t["wide_target"], t["source"]) == (3, 40.0, 20, "set")
    for bad in ({"k_reg": 6}, {"k_reg": 1}, {"pass_ops": 0.0}, {"pass_ops": 1e5}, {"wide_target": 65}):
        with pytest.raises(jq.JqError) as e:
            jq.tuning_set(28, "c128", **bad)
        assert e.value.code == jq.JQ_EINVAL
    assert jq.tuning_get(28, "c128")["k_reg"] == 3  # unchanged by the rejected calls
    with pytest.raises(jq.JqError):
        jq.tuning_set(28, "compact", k_reg=4)
    jq.tuning_set(28, "c64", k_reg=6)  # complex64 allows 6
    jq.tuning_set(28, "c128", clear=True)
    assert jq.tuning_get(28, "c128")["source"] == "cached"


def test_tuned_search_switch(_cache):
    # the large-state steps are off below 1 GiB by the size rule; a tuned
    # value (from the cache file or set) turns them on, an explicit option wins
    # (the cache file is read once per path: written before the first lookup)
    n = 18
    circ = W.layered_u2_cz(n, 6, seed=18)
    write(_cache, [dict(entry(n, k=4, ops=19.0, wide=17), search=jq.JQ_SEARCH_ON)])
    plain = jq.plan_steps(n, "c128", circ, search=jq.JQ_SEARCH_OFF)
    searched = jq.plan_steps(n, "c128", circ, search=jq.JQ_SEARCH_ON)
    assert plain != searched
    assert jq.tuning_get(n, "c128")["search"] == jq.JQ_SEARCH_ON
    assert jq.plan_steps(n, "c128", circ) == searched
    assert jq.plan_steps(n, "c128", circ, search=jq.JQ_SEARCH_OFF) == plain
    jq.tuning_set(n, "c128", search=jq.JQ_SEARCH_OFF)
    assert jq.plan_steps(n, "c128", circ) == plain
    with pytest.raises(jq.JqError):
        jq.tuning_set(n, "c128", search=7)
    jq.tuning_set(n, "c128", clear=True)


def test_planner_uses_the_tuned_register_width():
    circ = W.layered_u2_cz(26, 2, seed=1)
    assert {s["k_reg"] for s in jq.plan_steps(26, "c128", circ) if s["fused"]} == {5}
    jq.tuning_set(26, "c128", k_reg=3)
    assert {s["k_reg"] for s in jq.plan_steps(26, "c128", circ) if s["fused"]} == {3}
    # an explicit fusion width in the options wins over the tuning
    assert {s["k_reg"] for s in jq.plan_steps(26, "c128", circ, fusion=5) if s["fused"]} == {5}


def test_wide_register_width_only_for_reduced_kind_circuits():
    # a width above the one where the fused kernel compiled for every op kind
    # keeps 4 waves per SIMD (complex128 4, complex64 5) is kept only when
    # every gate lowers to the reduced kinds (uncontrolled one-qubit dense
    # gates, controlled Zs); a width asked for in the options is kept as given
    n = 26
    lite = W.layered_u2_cz(n, 2, seed=1)
    with_cnot = lite + [("CNOT", (0, 9), ())]
    with_rz = lite + [("RZ", (3,), (0.4,))]
    with_ccz = lite + [("CZ", (1, 2), (), (3,))]  # a CZ with one more control
    for enc, cap in (("c128", 4), ("c64", 5)):
        def widths(c, **kw):
            return {s["k_reg"] for s in jq.plan_steps(n, enc, c, **kw) if s["fused"]}
        jq.tuning_set(n, enc, k_reg=cap + 1)
        assert widths(lite) == {cap + 1}
        assert widths(with_ccz) == {cap + 1}
        assert widths(with_cnot) == {cap}
        assert widths(with_rz) == {cap}
        assert widths(with_cnot, fusion=cap + 1) == {cap + 1}
        # at or below the limit the tuned width stands
        jq.tuning_set(n, enc, k_reg=3)
        assert widths(with_cnot) == {3}
        jq.tuning_set(n, enc, clear=True)


def test_autotune_needs_a_device():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is visible (the GPU tests cover jq_autotune)")
    except ImportError:
        pass
    with pytest.raises(jq.JqError) as e:
        jq.autotune(20, "c128", no_cache=True)
    assert e.value.code == jq.JQ_EDEVICE
    with pytest.raises(jq.JqError) as e:
        jq.autotune(9, "c128")
    assert e.value.code == jq.JQ_EINVAL
    with pytest.raises(jq.JqError) as e:  # an invalid workload gate
        jq.autotune(12, "c128", [("CNOT", (3, 3), ())])
    assert e.value.code == jq.JQ_EINVAL


def test_per_target_width_mask(_cache):
    # an entry without wide_mask takes the targets from wide_target up; one
    # with a mask keeps it (and reports its lowest target); the file written
    # by the tuner round-trips the mask
    low = 2**53 - 1
    write(_cache, [entry(26, wide=12), dict(entry(28, wide=12), wide_mask=(1 << 9) | (1 << 20) | (1 << 21))])
    t = jq.tuning_get(26, "c128")
    assert t["wide_mask"] & low == low ^ (2**12 - 1) and t["wide_target"] == 12
    t = jq.tuning_get(28, "c128")
    assert t["wide_mask"] == (1 << 9) | (1 << 20) | (1 << 21) and t["wide_target"] == 9
    # set: a threshold, then a mask, then none at all
    jq.tuning_set(28, "c128", wide_target=20)
    t = jq.tuning_get(28, "c128")
    assert t["wide_target"] == 20 and t["wide_mask"] == (2**64 - 1) ^ (2**20 - 1)
    jq.tuning_set(28, "c128", wide_mask=(1 << 5) | (1 << 27))
    t = jq.tuning_get(28, "c128")
    assert (t["wide_target"], t["wide_mask"], t["source"]) == (5, (1 << 5) | (1 << 27), "set")
    jq.tuning_set(28, "c128", wide_target=64)
    assert (jq.tuning_get(28, "c128")["wide_mask"], jq.tuning_get(28, "c128")["wide_target"]) == (0, 64)

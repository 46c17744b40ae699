"""GPU parity of the projection layer (App. A: M, CLEAR, SET) through the C
ABI: jq_project and jq_measure against the oracle's oq_project/oq_measure,
the App. B error-correction example against its printed outputs in every
encoding, and the failure and argument checks."""
import json
import math
import os

import numpy as np
import pytest

from oracle import core as O
from paper_1805_04708_amd import jq
from paper_1805_04708_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = {"c128": 1e-12, "c64": 2e-6}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    jq.lib()


def appb(golden_dir):
    fx = json.load(open(os.path.join(golden_dir, "appB_error_correction.json")))
    to = lambda lst: [(g[0], tuple(g[1]), ()) for g in lst]
    return fx, to(fx["prepare"]), {v: to(e) + to(fx["correct"]) for v, e in fx["errors"].items()}


@pytest.mark.parametrize("enc", ["c128", "c64", "compact"])
@pytest.mark.parametrize("variant,syndrome", [("i", [0, 0]), ("ii", [1, 1]), ("iii", [0, 1])])
def test_appendix_b_error_correction(golden_dir, enc, variant, syndrome):
    fx, prep, rest = appb(golden_dir)
    n, d = fx["n_qubits"], fx["digits"]
    with jq.State(n, enc) as s:
        s.apply_circuit(prep)
        for got, key in zip(s.expectations(), ("Qx", "Qy", "Qz")):
            assert np.all(np.round(got, d) == np.array(fx["first"][key])), (enc, key, got)
        assert s.run_program(rest[variant], draws=[0.5, 0.5]) == syndrome
        for got, key in zip(s.expectations(), ("Qx", "Qy", "Qz")):
            assert np.all(np.round(got, d) == np.array(fx["final"][variant][key])), (enc, variant, key, got)
        assert abs(s.norm() - 1.0) < (1e-12 if enc == "c128" else 1e-5)


@pytest.mark.parametrize("enc", ["c128", "c64"])
@pytest.mark.parametrize("n", [5, 13])
def test_project_and_measure_match_oracle(enc, n):
    circ = W.random_circuit(n, 80, seed=900 + n)
    rng = np.random.default_rng(n)
    steps = [("P", int(rng.integers(n)), int(rng.integers(2))) for _ in range(3)] + \
            [("M", int(rng.integers(n)), float(rng.random())) for _ in range(3)]
    ref = O.run(O.zero_state(n), n, circ)
    with jq.State(n, enc) as s:
        s.apply_circuit(circ)
        for kind, q, x in steps:
            if kind == "P":
                p_ref = O.project(ref, n, q, x)
                if p_ref == 0.0:
                    with pytest.raises(jq.JqError):
                        s.project(q, x)
                    continue
                assert abs(s.project(q, x) - p_ref) < 10 * TOL[enc]
            else:
                # keep the draw away from the threshold p0, where the two
                # sides' roundings of p0 could pick different outcomes
                pr = O.probabilities(ref, n, [q])
                p0 = pr[0] / pr.sum()
                u = x if abs(x - p0) > 1e-3 else (p0 / 2 if p0 > 0.5 else (1 + p0) / 2)
                out_ref, p1_ref = O.measure(ref, n, q, u)
                out, p1 = s.measure(q, u)
                assert abs(p1 - p1_ref) < 10 * TOL[enc]
                assert out == out_ref
            assert O.rel_l2(s.amplitudes(), ref) < TOL[enc] * 10, (kind, q, x)
        assert abs(s.norm() - 1.0) < 10 * TOL[enc]


def test_compact_projection_matches_oracle_step():
    # one projection as a quantisation step from identical codes.  The kept
    # amplitudes are code-centred values, so whole classes of them can land
    # exactly on a rounding tie of the new range (253 (c - c_min) / (c_max -
    # c_min) a half-integer); there either neighbouring code is correct and
    # the last bit of p decides.  Every other code must agree.
    n = 12
    circ = W.layered_u2_cz(n, 2, seed=4)
    st = O.CompactState.encode(O.run(O.zero_state(n), n, circ), n)
    before = st.decode()
    with jq.State(n, "compact") as s:
        s.write_codes(st.b0, st.b1, tuple(st.rng))
        p = s.project(5, 1)
        g0, g1, grng = s.codes()
    p_ref = st.project(5, 1)
    assert abs(p - p_ref) < 1e-12
    assert np.allclose(grng, st.rng, rtol=1e-12, atol=0)
    kept = ((np.arange(1 << n) >> 5) & 1) == 1
    assert np.all(g0[~kept] == -128) and np.all(g1[~kept] == 0)
    d0 = np.abs(g0.astype(int) - st.b0.astype(int))
    d1 = np.abs(((g1.astype(int) - st.b1.astype(int)) + 128) % 256 - 128)
    assert d0.max() <= 1 and d1.max() <= 1
    z = before * (1.0 / math.sqrt(p_ref))
    r0, r1 = st.rng
    q = 253.0 * (np.abs(z) - r0) / (r1 - r0)
    th = 128.0 * np.angle(z) / math.pi
    tie = lambda v: np.abs(v - np.floor(v) - 0.5) < 1e-9
    assert np.all(tie(q[d0 != 0])), q[d0 != 0]
    assert np.all(tie(th[d1 != 0])), th[d1 != 0]


@pytest.mark.parametrize("enc", ["c128", "c64", "compact"])
def test_projection_onto_zero_amplitude_fails_and_keeps_state(enc):
    n = 6
    with jq.State(n, enc) as s:
        s.apply_circuit([("H", (0,), ()), ("CNOT", (0, 1), ())])
        before = s.amplitudes()
        with pytest.raises(jq.JqError) as e:
            s.project(3, 1)
        assert e.value.code == jq.JQ_EZERO
        assert np.array_equal(s.amplitudes(), before)
        # certain outcome whatever the draw; the renormalisation by
        # 1/sqrt(p0), p0 = 1 up to rounding, moves amplitudes by an ulp at most
        assert s.measure(3, 0.999999) == (0, 0.0)
        assert np.max(np.abs(s.amplitudes() - before)) < (1e-15 if enc != "c64" else 1e-7)


def test_measure_threshold_and_argument_errors():
    n = 4
    c, sn = math.cos(0.6), math.sin(0.6)
    circ = [("MAT1", (2,), (c, 0, -sn, 0, sn, 0, c, 0))]
    p1 = sn * sn
    for u, want in ((0.0, 0), (1 - p1 - 1e-9, 0), (1 - p1 + 1e-9, 1), (0.999999, 1)):
        with jq.State(n, "c128") as s:
            s.apply_circuit(circ)
            out, p1_got = s.measure(2, u)
            assert out == want and abs(p1_got - p1) < 1e-15
            amp = s.amplitudes()
            assert abs(abs(amp[want << 2]) - 1.0) < 1e-15 and abs(s.norm() - 1.0) < 1e-15
    with jq.State(n, "c128") as s:
        for bad in (lambda: s.measure(2, 1.0), lambda: s.measure(2, -0.1), lambda: s.measure(4, 0.5),
                    lambda: s.project(-1, 0), lambda: s.project(0, 2)):
            with pytest.raises(jq.JqError) as e:
                bad()
            assert e.value.code == jq.JQ_EINVAL

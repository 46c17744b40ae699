"""GPU tests of the request loop: results match the oracle, each result is
bitwise the same alone and in a concurrent mix, admission by state bytes,
backpressure and rejection."""
import threading
import time

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
    jq.lib()


def alone(n, circ, enc):
    with jq.State(n, enc) as s:
        s.apply_circuit(circ)
        return s.amplitudes()


@pytest.mark.parametrize("enc,tol", [("c64", 5e-6), ("c128", 1e-12)])
def test_mix_matches_oracle_and_alone(enc, tol):
    rng = np.random.default_rng(5)
    reqs = []
    for _ in range(40):
        n = int(rng.integers(3, 19))
        reqs.append((n, W.layered_random(n, int(rng.integers(20, 120)), rng)))
    sv = jq.Server(hbm_budget=8 << 30, n_streams=4, encoding=enc)
    tickets = {}
    for i, (n, c) in enumerate(reqs):
        tickets[sv.submit(n, c)] = i
    got = {}
    for _ in reqs:
        r = sv.wait(60000)
        assert r is not None and r["status"] == 0
        i = tickets[r["ticket"]]
        got[i] = sv.state(r).amplitudes()
        assert abs(r["norm"] - 1.0) < 10 * tol
        sv.release(r["ticket"])
    st = sv.stats()
    assert st["completed"] == len(reqs) and st["p99_ms"] >= st["p50_ms"] > 0
    sv.close()
    for i, (n, c) in enumerate(reqs):
        if n <= 14:
            assert O.rel_l2(got[i], O.run(O.zero_state(n), n, c)) <= tol * max(1, len(c) / 100) ** 0.5 * 4
        assert np.array_equal(got[i], alone(n, c, enc)), i


def test_compact_requests():
    # served two-byte requests (per-gate quantisation, the paper's
    # procedure) against the oracle's two-byte run of the same circuit:
    # both code planes (a tie decided differently early on may change later
    # codes by one step, so almost all codes agree and none differs by more
    # than one step, phase codes mod 256), the range, and the accuracy of
    # the decoded state against the exact FP64 state (fidelity loss within
    # twice the oracle's own); each result also equals the same request run
    # alone, bit for bit
    rng = np.random.default_rng(8)
    sv = jq.Server(hbm_budget=1 << 30, n_streams=2, encoding="compact")
    reqs = [(int(n), W.layered_random(int(n), 40, rng)) for n in rng.integers(4, 13, 12)]
    t = {sv.submit(n, c): i for i, (n, c) in enumerate(reqs)}
    for _ in reqs:
        r = sv.wait(60000)
        assert r["status"] == 0
        n, c = reqs[t[r["ticket"]]]
        st = O.CompactState.encode(O.zero_state(n), n).run(c)
        b0, b1, rg = sv.state(r).codes()
        amps = sv.state(r).amplitudes()
        d0 = np.abs(b0.astype(int) - st.b0.astype(int))
        d1 = np.abs(((b1.astype(int) - st.b1.astype(int) + 128) % 256) - 128)
        assert d0.max() <= 1 and d1.max() <= 1, (n, d0.max(), d1.max())
        assert int(np.sum((d0 != 0) | (d1 != 0))) <= max(2, 0.01 * d0.size)
        assert np.allclose(rg, st.rng, rtol=1e-9, atol=0), (rg, st.rng)
        exact = O.run(O.zero_state(n), n, c)
        f_gpu, f_or = O.fidelity(amps, exact), O.fidelity(st.decode(), exact)
        assert 1 - f_gpu <= 2 * (1 - f_or) + 1e-12, (n, f_gpu, f_or)
        with jq.State(n, "compact") as s:
            s.apply_circuit(c)
            a0, a1, ar = s.codes()
        assert np.array_equal(a0, b0) and np.array_equal(a1, b1) and np.array_equal(ar, rg)
        sv.release(r["ticket"])
    sv.close()


def test_admission_budget_backpressure_and_rejection():
    sv = jq.Server(hbm_budget=1 << 20, n_streams=2, queue_cap=2, encoding="c64")
    # 2^18 * 8 B = 2 MiB > 1 MiB budget: rejected at submit
    with pytest.raises(jq.JqError) as e:
        sv.submit(18, [("H", (0,), ())])
    assert e.value.code == jq.JQ_ENOMEM
    # fill the budget with an unreleased result, then the queue
    sv.submit(16, [("H", (0,), ())])           # 512 KiB
    r = sv.wait(10000)
    assert r["status"] == 0
    sv.submit(16, [("H", (1,), ())])           # fits: 1 MiB total
    sv.submit(17, [("H", (1,), ())])           # 1 MiB: waits for a release
    sv.submit(17, [("H", (2,), ())])
    with pytest.raises(jq.JqError) as e:
        sv.submit(17, [("H", (3,), ())], blocking=False)
    assert e.value.code == jq.JQ_EBUSY
    r2 = sv.wait(10000)
    assert r2["status"] == 0
    assert sv.wait(200) is None                # the 2^17 requests cannot be admitted yet
    sv.release(r["ticket"])
    sv.release(r2["ticket"])
    r3 = sv.wait(10000)
    assert r3 is not None and r3["n"] == 17
    sv.release(r3["ticket"])
    r4 = sv.wait(10000)
    assert r4 is not None and r4["n"] == 17
    sv.release(r4["ticket"])
    st = sv.stats()
    assert st["peak_resident_bytes"] <= 1 << 20
    sv.close()


def test_invalid_circuit_rejected_at_submit():
    sv = jq.Server(hbm_budget=1 << 30, encoding="c64")
    with pytest.raises(jq.JqError) as e:
        sv.submit(4, [("CNOT", (0, 4), ())])
    assert e.value.code == jq.JQ_EINVAL
    sv.close()


def test_concurrent_submitters():
    sv = jq.Server(hbm_budget=2 << 30, n_streams=4, encoding="c64")
    rng = np.random.default_rng(2)
    work = [(int(n), W.layered_random(int(n), 30, rng)) for n in rng.integers(4, 16, 60)]
    done = []

    def client(chunk):
        for n, c in chunk:
            sv.submit(n, c)

    th = [threading.Thread(target=client, args=(work[i::3],)) for i in range(3)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    while len(done) < len(work):
        r = sv.wait(30000)
        assert r is not None and r["status"] == 0
        done.append(r)
        sv.release(r["ticket"])
    assert sv.stats()["completed"] == len(work)
    sv.close()

"""GPU parity of basis-state sampling (App. A, GENERATE EVENTS) through the C
ABI: jq_sample against the oracle's oq_sample on the same draws.

The two sum the probabilities in different orders (the oracle in index
order, the GPU in fixed blocks), so a draw whose target lies within rounding
of a cumulative boundary may pick either neighbour: such draws are checked
to be valid (the event is one of the two indices at that boundary), every
other draw must give the oracle's index."""
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


def check_against_oracle(psi_ref, n, u, got, rel=1e-12):
    want = O.sample(psi_ref, n, u)
    p = psi_ref.real ** 2 + psi_ref.imag ** 2
    c = np.cumsum(p)
    total = c[-1]
    assert np.all(p[got.astype(np.int64)] > 0), "zero-probability state drawn"
    bad = np.nonzero(got != want)[0]
    for k in bad:
        t = u[k] * total
        near = np.abs(c - t) <= rel * total
        assert near.any(), (k, u[k], got[k], want[k])
        assert abs(int(got[k]) - int(want[k])) <= np.count_nonzero(near) + np.count_nonzero(p == 0), (k, got[k], want[k])
    return len(bad)


@pytest.mark.parametrize("enc", ["c128", "c64", "compact"])
@pytest.mark.parametrize("n", [4, 10, 20])
def test_uniform_state_is_floor_of_u(enc, n):
    u = np.concatenate([[0.0, 1 - 2.0 ** -40], np.random.default_rng(n).random(4000)])
    with jq.State(n, enc) as s:
        s.init(jq.JQ_INIT_UNIFORM)
        assert np.array_equal(s.sample(u), np.floor(u * 2 ** n).astype(np.uint64))


@pytest.mark.parametrize("enc", ["c128", "compact"])
def test_ghz_and_basis(enc):
    n = 20
    u = np.random.default_rng(5).random(3000)
    u = u[np.abs(u - 0.5) > 1e-9]
    with jq.State(n, enc) as s:
        s.apply_circuit(W.ghz(n))
        assert np.array_equal(s.sample(u), np.where(u < 0.5, 0, (1 << n) - 1).astype(np.uint64))
        s.init(jq.JQ_INIT_BASIS, 123457)
        assert np.all(s.sample(u) == 123457)


@pytest.mark.parametrize("enc", ["c128", "c64"])
@pytest.mark.parametrize("n", [11, 13, 17])
def test_random_state_matches_oracle(enc, n):
    # N=13: two blocks of 4096; N=17: 32 blocks.  Zeros from a CNOT-heavy
    # circuit on part of the register exercise zero-probability runs.
    circ = W.random_circuit(n - 2, 120, seed=40 + n)
    u = np.random.default_rng(n).random(20000)
    with jq.State(n, enc) as s:
        s.apply_circuit(circ)
        got = s.sample(u)
        amp = s.amplitudes()
    # the oracle samples the GPU's own amplitudes, so only the summation order differs
    ref = amp.astype(np.complex128)
    mism = check_against_oracle(ref, n, u, got, rel=1e-12 if enc == "c128" else 1e-6)
    assert mism <= 20


def test_compact_state_matches_oracle_on_its_decoded_amplitudes():
    n = 14
    circ = W.layered_u2_cz(n, 2, seed=9)
    u = np.random.default_rng(2).random(20000)
    with jq.State(n, "compact") as s:
        s.apply_circuit(circ)
        got = s.sample(u)
        amp = s.amplitudes()
    assert check_against_oracle(amp, n, u, got) <= 20


def test_many_draws_take_several_batches():
    n = 10
    u = np.random.default_rng(7).random((1 << 20) + 1000)
    with jq.State(n, "c128") as s:
        s.init(jq.JQ_INIT_UNIFORM)
        assert np.array_equal(s.sample(u), np.floor(u * 2 ** n).astype(np.uint64))


def test_full_size_uniform_and_state_unchanged():
    n = 30
    u = np.random.default_rng(30).random(8192)
    with jq.State(n, "c128") as s:
        s.init(jq.JQ_INIT_UNIFORM)
        assert np.array_equal(s.sample(u), np.floor(u * 2 ** n).astype(np.uint64))
        assert abs(s.amplitudes(12345, 1)[0] - 2.0 ** -15) == 0


def test_sample_errors():
    with jq.State(6, "c128") as s:
        for bad in ([1.0], [-0.5], [0.2, np.nan]):
            with pytest.raises(jq.JqError) as e:
                s.sample(bad)
            assert e.value.code == jq.JQ_EINVAL
        s.write_amplitudes(np.zeros(64, dtype=np.complex128))
        with pytest.raises(jq.JqError) as e:
            s.sample([0.3])
        assert e.value.code == jq.JQ_EZERO
        assert len(s.sample([])) == 0

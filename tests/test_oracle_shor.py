"""Pins of the Shor oracle (Sec. 5.3; App. A, SHORBOX) on the CPU.

Two independent computations: the SHORBOX state vector followed by the
gate-level quantum Fourier transform of the oracle's C core, and the
residue-by-residue FFT of oracle/shor.py; and the printed exact column of
Table Shortab1 at 30 qubits."""
import json
import os

import numpy as np
import pytest

from oracle import core as O
from oracle import shor as S
from paper_1805_04708_amd import workloads as W


@pytest.mark.parametrize("n,n_x,G,y", [(12, 8, 15, 7), (15, 10, 21, 2), (13, 9, 15, 2)])
def test_fft_expectations_match_gate_level_qft(n, n_x, G, y):
    psi = S.shorbox_state(n, n_x, G, y)
    assert abs(O.norm2(psi, n) - 1.0) < 1e-14
    O.run(psi, n, W.qft(n_x))
    qx, qy, qz = O.expect_q(psi, n)
    ex, ey, ez = S.qft_expectations(n_x, G, y)
    for a, b in ((qx, ex), (qy, ey), (qz, ez)):
        assert np.max(np.abs(a[:n_x] - b)) < 1e-12


def test_shorbox_state_is_the_definition():
    n, n_x, G, y = 11, 7, 15, 2
    psi = S.shorbox_state(n, n_x, G, y)
    amp = 2.0 ** (-n_x / 2)
    for x in range(1 << n_x):
        f = pow(y, x, G)
        assert psi[x + (f << n_x)] == amp
    assert np.count_nonzero(psi) == 1 << n_x
    # the f-register marginal is uniform over the orbit {1, 2, 4, 8}
    pf = O.probabilities(psi.copy(), n, list(range(n_x, n)))
    assert set(np.nonzero(pf)[0]) == {1, 2, 4, 8} and np.allclose(pf[[1, 2, 4, 8]], 0.25)


def test_table_shortab1_exact_column(golden_dir):
    fx = json.load(open(os.path.join(golden_dir, "table_shortab1.json")))
    qx, qy, qz = S.qft_expectations(fx["n_x"], fx["G"], fx["y"])
    d = fx["digits"]
    ex = fx["exact"]
    assert np.all(np.round(qz, d) == np.array(ex["Qz"]))
    assert np.all(np.round(qy, d) == np.array(ex["Qy"]))
    skip = set(fx["exact_qx_differs_from_state_vector"])
    keep = [i for i in range(fx["n_x"]) if i not in skip]
    assert np.all(np.round(qx[keep], d) == np.array(ex["Qx"])[keep])
    # the three entries read differently (see the fixture): state-vector values
    assert np.round(qx[5], d) == 0.506 and fx["two_byte_code"]["Qx"][5] == 0.506

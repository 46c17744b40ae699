"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here touches the GPU library.  Each test would fail on a plausible
mistake in the oracle: a transposed or conjugated matrix, a wrong bit order,
a dropped control, a wrong sign in the phase convention, a wrong scale in the
two-byte code.
"""
import cmath
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import core as O
from oracle import dense as D
from oracle import gates as G
from paper_1805_04708_amd import workloads as W

ALL_1Q = ["I", "H", "X", "Y", "Z", "S", "S+", "T", "T+", "+X", "-X", "+Y", "-Y"]


def rand_complex(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def rand_state(rng, n):
    psi = rand_complex(rng, 1 << n)
    return psi / np.linalg.norm(psi)


# ---------------------------------------------------------------------------
# gate application against the Kronecker-product definition (Sec. 2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(40))
def test_apply_matches_kronecker_bruteforce(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 7))
    k = int(rng.integers(1, min(3, n) + 1))
    qs = [int(x) for x in rng.permutation(n)]
    targets = qs[:k]
    nc = int(rng.integers(0, min(2, n - k) + 1))
    controls = qs[k:k + nc]
    m = rand_complex(rng, 1 << k, 1 << k)  # any matrix, unitary or not
    psi = rand_complex(rng, 1 << n)
    ref = D.apply(psi.copy(), n, targets, controls, m)
    got = O.apply(psi.copy(), n, targets, controls, m)
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_bit_order_qubit0_is_lsb():
    # Sec. 2: qubit 0 is the rightmost bit.  X on qubit 0 maps |0..00> to |0..01> = index 1.
    psi = O.zero_state(3)
    O.run(psi, 3, [("X", (0,), ())])
    assert psi[1] == 1 and np.count_nonzero(psi) == 1
    psi = O.zero_state(3)
    O.run(psi, 3, [("X", (2,), ())])
    assert psi[4] == 1


def test_cnot_basis_is_control_target():
    # App. A: CNOT c t flips t when c is 1.  |c=1,t=0>: with c=qubit 2, t=qubit 0, index 4 -> 5.
    for c, t in [(2, 0), (0, 2), (1, 0)]:
        for x in range(8):
            psi = O.basis_state(3, x)
            O.run(psi, 3, [("CNOT", (c, t), ())])
            y = x ^ (1 << t) if (x >> c) & 1 else x
            assert abs(psi[y] - 1) < 1e-15


def test_toffoli_truth_table():
    for x in range(16):
        psi = O.basis_state(4, x)
        O.run(psi, 4, [("TOFFOLI", (3, 1, 2), ())])
        y = x ^ 4 if ((x >> 3) & 1 and (x >> 1) & 1) else x
        assert abs(psi[y] - 1) < 1e-15


@pytest.mark.parametrize("seed", range(12))
def test_named_random_circuits_match_bruteforce(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 7))
    circ = []
    for _ in range(30):
        r = rng.random()
        q = [int(x) for x in rng.permutation(n)]
        if r < 0.45:
            circ.append((ALL_1Q[int(rng.integers(len(ALL_1Q)))], (q[0],), ()))
        elif r < 0.6:
            name = ["U1", "U2", "U3", "RZ", "R"][int(rng.integers(5))]
            params = {"U1": (rng.uniform(-4, 4),), "U2": tuple(rng.uniform(-4, 4, 2)),
                      "U3": tuple(rng.uniform(-4, 4, 3)), "RZ": (rng.uniform(-4, 4),),
                      "R": (int(rng.integers(-6, 7)),)}[name]
            circ.append((name, (q[0],), params))
        elif r < 0.8:
            name = ["CNOT", "CZ", "CP", "U", "SWAP"][int(rng.integers(5))]
            params = {"CP": (rng.uniform(-4, 4),), "U": (int(rng.integers(-5, 6)),)}.get(name, ())
            circ.append((name, (q[0], q[1]), params))
        elif r < 0.9 and n >= 3:
            circ.append(("TOFFOLI", (q[0], q[1], q[2]), ()))
        else:
            circ.append(("MAT1", (q[0],), W.haar_u2(rng), (q[1],)))
    psi = rand_state(rng, n)
    ref = psi.copy()
    for g in circ:
        t, c, m = G.lower(g)
        ref = D.apply(ref, n, t, c, m)
    got = O.run(psi.copy(), n, circ)
    assert np.max(np.abs(got - ref)) < 1e-12


# ---------------------------------------------------------------------------
# the gate table against identities fixed by App. A and by algebra
# ---------------------------------------------------------------------------

def M(name, *p):
    return G.matrix(name, p)


@pytest.mark.parametrize("name", ALL_1Q + ["CNOT", "CZ", "SWAP", "TOFFOLI"])
def test_named_gates_are_unitary(name):
    m = M(name)
    assert np.allclose(m.conj().T @ m, np.eye(m.shape[0]), atol=1e-15)


def test_gate_identities():
    I2 = np.eye(2)
    X, Y, Z, H = M("X"), M("Y"), M("Z"), M("H")
    assert np.allclose(M("S") @ M("S"), Z, atol=1e-15)
    assert np.allclose(M("T") @ M("T"), M("S"), atol=1e-15)
    assert np.allclose(M("S") @ M("S+"), I2, atol=1e-15)
    assert np.allclose(M("T") @ M("T+"), I2, atol=1e-15)
    assert np.allclose(H @ Z @ H, X, atol=1e-15)
    assert np.allclose(1j * X @ Z, Y, atol=1e-15)
    # +X, -X rotate by -pi/2, +pi/2 about x: (+X)(-X) = 1, (+X)^2 = iX
    assert np.allclose(M("+X") @ M("-X"), I2, atol=1e-15)
    assert np.allclose(M("+X") @ M("+X"), 1j * X, atol=1e-15)
    assert np.allclose(M("+Y") @ M("-Y"), I2, atol=1e-15)
    assert np.allclose(M("+Y") @ M("+Y"), 1j * Y, atol=1e-15)
    for k in range(0, 8):
        assert np.allclose(M("R", k), M("U1", 2 * math.pi / 2 ** k), atol=1e-15)
        assert np.allclose(M("R", -k), M("U1", -2 * math.pi / 2 ** k), atol=1e-15)
    for phi, lam in [(0.3, -1.2), (2.0, 0.7)]:
        assert np.allclose(M("U3", math.pi / 2, phi, lam), M("U2", phi, lam), atol=1e-15)
        assert np.allclose(M("U3", 0.0, 0.0, lam), M("U1", lam), atol=1e-15)
    assert np.allclose(M("RZ", 0.9), cmath.exp(-0.45j) * M("U1", 0.9), atol=1e-15)
    assert np.allclose(M("U", 1), M("CZ"), atol=1e-15)
    assert np.allclose(M("CP", 2 * math.pi / 8), M("U", 3), atol=1e-15)


def test_u_gate_is_the_exponential_of_the_zz_form():
    # Sec. 4.2, Eq. appa4: U01(a) = exp(i a (1 + sz0 sz1 - sz0 - sz1)/4)
    sz = np.diag([1.0, -1.0])
    one = np.eye(4)
    ham = one + np.kron(sz, sz) - np.kron(sz, np.eye(2)) - np.kron(np.eye(2), sz)
    for k in range(1, 6):
        a = 2 * math.pi / 2 ** k
        expo = np.diag(np.exp(1j * a * np.diag(ham) / 4))
        assert np.allclose(expo, M("U", k), atol=1e-15)


def test_cnot_is_h_cz_h_and_controlled_x():
    # Sec. 4.2: the CNOT follows from U(pi) sandwiched between Hadamards on the target.
    rng = np.random.default_rng(7)
    for c, t in [(0, 1), (1, 0), (2, 0), (0, 2)]:
        psi = rand_state(rng, 3)
        a = O.run(psi.copy(), 3, [("CNOT", (c, t), ())])
        b = O.run(psi.copy(), 3, [("H", (t,), ()), ("CZ", (c, t), ()), ("H", (t,), ())])
        d = O.apply(psi.copy(), 3, [t], [c], M("X"))
        assert np.allclose(a, b, atol=1e-14) and np.allclose(a, d, atol=1e-15)


# ---------------------------------------------------------------------------
# closed forms of Sec. 5 and Sec. 4.2, and the worked example of App. B
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 5, 10, 16])
def test_hadamard_all_gives_uniform(n, golden_dir):
    psi = O.run(O.zero_state(n), n, W.hadamard_all(n))
    assert np.max(np.abs(psi - 2.0 ** (-n / 2))) < 1e-15 * 2 ** (-n / 2) * 8
    if n <= 12:
        tab = json.load(open(os.path.join(golden_dir, "table_htab.json")))
        qx, qy, qz = O.expect_q(psi, n)
        for got, key in ((qx, "Qx"), (qy, "Qy"), (qz, "Qz")):
            assert np.all(np.round(got, tab["digits"]) == tab[key])


@pytest.mark.parametrize("n", [2, 3, 8, 14])
def test_ghz(n, golden_dir):
    psi = O.run(O.zero_state(n), n, W.ghz(n))
    ref = np.zeros(1 << n, dtype=complex)
    ref[0] = ref[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(psi - ref)) < 1e-15
    tab = json.load(open(os.path.join(golden_dir, "table_cnottab.json")))
    qx, qy, qz = O.expect_q(psi, n)
    for got, key in ((qx, "Qx"), (qy, "Qy"), (qz, "Qz")):
        assert np.all(np.round(got, tab["digits"]) == tab[key])


@pytest.mark.parametrize("n", [1, 3, 5, 8])
def test_qft_of_basis_state_closed_form(n):
    for x in [0, 1, (1 << n) - 1, (0b1011 % (1 << n))]:
        psi = O.run(O.basis_state(n, x), n, W.qft(n))
        k = np.arange(1 << n)
        ref = 2.0 ** (-n / 2) * np.exp(2j * np.pi * x * k / 2 ** n)
        assert np.max(np.abs(psi - ref)) < 1e-13


@pytest.mark.parametrize("n", [2, 4, 7])
def test_qft_matches_inverse_fft(n):
    rng = np.random.default_rng(n)
    psi = rand_state(rng, n)
    got = O.run(psi.copy(), n, W.qft(n))
    assert np.max(np.abs(got - np.fft.ifft(psi, norm="ortho"))) < 1e-13


def test_appendix_b_first_measurement_block(golden_dir):
    fx = json.load(open(os.path.join(golden_dir, "appB_block1.json")))
    n = fx["n_qubits"]
    circ = [(g[0], tuple(g[1]), tuple(g[2])) for g in fx["circuit"]]
    psi = O.run(O.zero_state(n), n, circ)
    qx, qy, qz = O.expect_q(psi, n)
    for got, key in ((qx, "Qx"), (qy, "Qy"), (qz, "Qz")):
        assert np.all(np.round(got, fx["digits"]) == np.array(fx[key])), (key, got)
    # closed form behind the printed 0.146: (1 - cos(pi/4))/2
    assert abs(qz[0] - (1 - math.cos(math.pi / 4)) / 2) < 1e-15


def test_expectations_match_dense_pauli():
    rng = np.random.default_rng(3)
    n = 4
    psi = rand_state(rng, n)
    qx, qy, qz = O.expect_q(psi, n)
    for q in range(n):
        for got, pauli in ((qx, "X"), (qy, "Y"), (qz, "Z")):
            s = D.full_matrix(n, [q], [], M(pauli))
            assert abs(got[q] - (1 - np.vdot(psi, s @ psi).real) / 2) < 1e-14


@pytest.mark.parametrize("n", [6, 12])
def test_norm_preserved_over_200_gates(n):
    psi = O.run(O.zero_state(n), n, W.random_circuit(n, 200, seed=n))
    assert abs(O.norm2(psi, n) - 1.0) < 1e-13


def test_probabilities_match_tensor_sums():
    rng = np.random.default_rng(11)
    n = 6
    psi = rand_state(rng, n)
    t = (np.abs(psi) ** 2).reshape((2,) * n)  # axis a holds qubit n-1-a
    for qubits in [[0], [5], [2, 4], [4, 2], [1, 3, 0], list(range(n)), []]:
        got = O.probabilities(psi, n, qubits)
        keep = [n - 1 - q for q in qubits]
        other = tuple(a for a in range(n) if a not in keep)
        ref = t.sum(axis=other) if other else t
        # move kept axes so that qubits[m] is bit m of the flat index
        order = [sorted(keep).index(a) for a in reversed(keep)]
        ref = np.transpose(ref, order).ravel() if keep else np.array([ref.sum()])
        assert np.allclose(got, ref, atol=1e-15)
    assert abs(O.probabilities(psi, n, []).sum() - 1) < 1e-14


# ---------------------------------------------------------------------------
# the two-byte encoding of Sec. 4.1
# ---------------------------------------------------------------------------

def test_compact_special_codes_and_formula():
    n = 2
    r0, r1 = 0.1, 0.6
    b0 = np.array([-128, 127, -127, 126], dtype=np.int8)
    b1 = np.array([37, -64, 0, 64], dtype=np.int8)
    z = O.CompactState(n, b0, b1, r0, r1).decode()
    assert z[0] == 0
    assert abs(z[1] - cmath.exp(-1j * math.pi / 2)) < 1e-15     # r = 1, theta = pi*(-64)/128
    assert abs(z[2] - r0) < 1e-15                               # c = -127 -> r0
    assert abs(z[3] - r1 * 1j) < 1e-15                           # c = 126 -> r1, theta = pi/2


def test_compact_decode_encode_is_idempotent():
    rng = np.random.default_rng(5)
    n = 10
    b0 = rng.integers(-128, 128, 1 << n).astype(np.int8)
    b1 = rng.integers(-128, 128, 1 << n).astype(np.int8)
    b1[b0 == -128] = 0
    st = O.CompactState(n, b0, b1, 0.013, 0.71)
    z = st.decode()
    again = O.CompactState.encode(z, n, 0.013, 0.71)
    assert np.array_equal(again.b0, b0) and np.array_equal(again.b1, b1)
    assert np.array_equal(again.decode(), z)


def test_compact_phase_wraps_and_rounds():
    n = 1
    for ang, code in [(math.pi, -128), (-math.pi, -128), (math.pi - 1e-9, -128),
                      (math.pi / 2, 64), (-math.pi / 2, -64), (3 * math.pi / 256 + 1e-9, 2),
                      (0.0, 0)]:
        z = np.array([0.5 * cmath.exp(1j * ang), 0.5], dtype=complex)
        st = O.CompactState.encode(z, n)
        assert st.b1[0] == code, (ang, st.b1[0])


def test_compact_range_and_modulus_code():
    z = np.array([0.0, 0.2, 0.7, 1.0, 0.4, 0.2 + 1e-9, 0, 0], dtype=complex)
    st = O.CompactState.encode(z, 3)
    assert st.rng[0] == 0.2 and st.rng[1] == 0.7
    assert list(st.b0[:5]) == [-128, -127, 126, 127, round(253 * 0.2 / 0.5) - 127]


@pytest.mark.parametrize("n", [3, 9])
def test_compact_uniform_and_ghz_are_exact(n):
    # Tables Htab and CNOTtab: the encoded flavour gives the same exact results.
    z0 = O.zero_state(n)
    st = O.CompactState.encode(z0, n).run(W.hadamard_all(n))
    assert np.max(np.abs(st.decode() - 2.0 ** (-n / 2))) < 1e-15
    st = O.CompactState.encode(z0, n).run(W.ghz(n))
    ref = np.zeros(1 << n, dtype=complex)
    ref[0] = ref[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(st.decode() - ref)) < 1e-15
    # one code pass for the whole run (block mode) gives the same
    st = O.CompactState.encode(z0, n).run(W.ghz(n), blocks=[n])
    assert np.max(np.abs(st.decode() - ref)) < 1e-15


def test_compact_phase_quantisation_matches_error_model():
    # From a uniform start RZ never changes a modulus, so only phases are
    # rounded, to multiples of pi/128.  RZ(theta) on qubit q adds -x and +x
    # (x = 64 theta/pi code units) to the integer phase codes of the bit-0 and
    # bit-1 halves, so all of one half share the rounding error e and the
    # other half gets -e, e ~ U[-w, w], w = pi/256.  Errors of the gates on
    # one qubit add up; the fidelity is the product over qubits of
    # cos^2(sum_g e_g), with mean (1 + sinc(2w)^L)/2 for L gates per qubit.
    n, layers = 10, 20
    w = math.pi / 256
    expected = n * math.log((1 + (math.sin(2 * w) / (2 * w)) ** layers) / 2)
    logs = []
    for seed in range(8):
        rng = np.random.default_rng(seed)
        circ = [("RZ", (q,), (float(rng.uniform(0, 2 * math.pi)),)) for _ in range(layers) for q in range(n)]
        exact = O.run(O.uniform_state(n), n, circ)
        st = O.CompactState.encode(O.uniform_state(n), n).run(circ)
        logs.append(math.log(O.fidelity(st.decode(), exact)))
    # per-run spread is about 0.0024, so the mean of 8 is good to about 0.0009;
    # a code step of pi/256 or pi/64 would move the mean by 4x.
    assert abs(np.mean(logs) - expected) < 0.003, (np.mean(logs), expected)


def test_compact_accuracy_is_about_three_digits():
    # Sec. 4.1 / Sec. 5.4: the encoded flavour reproduces expectation values
    # to about three digits on typical circuits.
    n = 8
    circ = W.random_circuit(n, 60, seed=4)
    exact = O.run(O.zero_state(n), n, circ)
    st = O.CompactState.encode(O.zero_state(n), n).run(circ)
    approx = st.decode()
    e = O.expect_q(exact, n)
    a = O.expect_q(approx, n)
    assert max(np.max(np.abs(x - y)) for x, y in zip(e, a)) < 0.05

"""The planner's schedule (jq_plan_schedule, host only): which gates run
together in one tile pass and in which order.  These checks need no GPU:
the order must be a permutation of the circuit that the oracle maps to the
same state (gates only move past gates they commute with), every fused
block must fit one tile, and the options select the documented modes."""
import math

import numpy as np
import pytest

from oracle import core as O
from paper_1805_04708_amd import jq
from paper_1805_04708_amd import workloads as W

# tile shape per encoding: fixed lane bits F, default register bits K
# (circuits with gates outside the reduced op kinds plan narrower:
# complex128 4, complex64 5)
LAYOUT = {"c128": (3, 5), "c64": (4, 6), "compact": (6, 4)}
PER_BLOCK = jq.JQ_COMPACT_PER_BLOCK


def schedule(n, enc, circ, **kw):
    order, blen, fused = jq.plan_schedule(n, enc, circ, **kw)
    return list(order), list(blen), list(fused)


def non_identity(circ):
    return [i for i, g in enumerate(circ) if g[0] != "I"]


def circuits(n):
    return [W.random_circuit(n, 200, seed=n), W.layered_u2_cz(n, 3, seed=n),
            W.rz_cnot_chain(n, 3, seed=n), W.qft(n)]


def targets_of(g):
    # qubits a gate changes the value of (diagonal gates change none)
    name, q = g[0], list(g[1])
    if name in ("Z", "S", "S+", "T", "T+", "U1", "R", "RZ", "U", "CZ", "CP", "I"):
        return []
    if name == "CNOT":
        return [q[1]]
    if name == "TOFFOLI":
        return [q[2]]
    return q


SEARCH_ON = {"search": jq.JQ_SEARCH_ON}


@pytest.mark.parametrize("n", [8, 12, 16])
@pytest.mark.parametrize("enc,kw", [("c128", {}), ("c64", {}), ("c128", {"fusion": 2}),
                                    ("c128", {"fusion": 5}), ("compact", {"compact_mode": PER_BLOCK}),
                                    ("c128", SEARCH_ON), ("c64", SEARCH_ON), ("compact", SEARCH_ON),
                                    ("compact", {"compact_mode": PER_BLOCK, **SEARCH_ON})])
def test_schedule_is_a_commuting_reordering(n, enc, kw):
    for circ in circuits(n):
        order, blen, fused = schedule(n, enc, circ, **kw)
        assert sorted(order) == non_identity(circ)
        assert sum(blen) == len(order) and all(b >= 1 for b in blen)
        assert all(f or b == 1 for b, f in zip(blen, fused))
        # the reordered circuit is the same unitary: same state from a
        # random start, to rounding
        rng = np.random.default_rng(n)
        psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
        psi /= np.linalg.norm(psi)
        a = O.run(psi.copy(), n, circ)
        b = O.run(psi.copy(), n, [circ[i] for i in order])
        assert O.rel_l2(b, a) < 1e-13


@pytest.mark.parametrize("enc,kw", [("c128", {}), ("c64", {}), ("c128", {"fusion": 3}),
                                    ("compact", {"compact_mode": PER_BLOCK}), ("c128", SEARCH_ON),
                                    ("c64", SEARCH_ON)])
def test_fused_blocks_fit_one_tile(enc, kw):
    n = 20
    F, K = LAYOUT[enc]
    if "fusion" in kw:
        K = kw["fusion"]
    for circ in circuits(n):
        order, blen, fused = schedule(n, enc, circ, **kw)
        pos = 0
        n_fused = 0
        for b, f in zip(blen, fused):
            blk = [circ[i] for i in order[pos:pos + b]]
            pos += b
            if not f:
                continue
            n_fused += 1
            free = {q for g in blk for q in targets_of(g)} - set(range(F))
            assert len(free) <= (6 - F) + K, (enc, sorted(free))
            # two-qubit dense gates other than SWAP (a permutation: three
            # controlled X ops in the pass) run unfused
            assert all(g[0] == "SWAP" or len(g[1]) - (1 if g[0] == "CNOT" else 2 if g[0] == "TOFFOLI" else 0) <= 1
                       or not targets_of(g) for g in blk), "two-qubit dense gates run unfused"
        assert n_fused > 0


def test_swap_fuses_and_general_two_qubit_gates_do_not():
    # the QFT's closing SWAPs join passes; a general 4x4 runs alone
    n = 14
    rng = np.random.default_rng(3)
    circ = W.qft(n)
    q, r = np.linalg.qr(rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4)))
    flat = []
    for x in q.ravel():
        flat += [float(x.real), float(x.imag)]
    circ = circ[:40] + [("MAT2", (2, 9), tuple(flat))] + circ[40:]
    for enc, kw in [("c128", {}), ("c64", {}), ("compact", {"compact_mode": PER_BLOCK}), ("compact", {})]:
        order, blen, fused = schedule(n, enc, circ, **kw)
        where_fused = {}
        pos = 0
        for b, f in zip(blen, fused):
            for i in order[pos:pos + b]:
                where_fused[i] = bool(f)
            pos += b
        swaps = [i for i, g in enumerate(circ) if g[0] == "SWAP"]
        assert swaps and all(where_fused[i] for i in swaps), (enc, kw)
        mat2 = [i for i, g in enumerate(circ) if g[0] == "MAT2"][0]
        assert not where_fused[mat2]
        # the reordered circuit is the same unitary
        psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
        psi /= np.linalg.norm(psi)
        assert O.rel_l2(O.run(psi.copy(), n, [circ[i] for i in order]), O.run(psi.copy(), n, circ)) < 1e-13


def test_unfused_modes_keep_the_input_order():
    n = 12
    circ = W.random_circuit(n, 100, seed=4) + [("I", (3,), ())]
    for enc, kw in [("c128", {"fusion": 1}), ("c64", {"fusion": 1}), ("compact", {"fusion": 1}),
                    ("compact", {"compact_mode": PER_BLOCK, "fusion": 1})]:
        order, blen, fused = schedule(n, enc, circ, **kw)
        assert order == non_identity(circ)
        assert blen == [1] * len(order) and not any(fused)


def test_small_states_fall_back_to_single_gates():
    # a tile needs 6 + K >= 8 index bits
    for n in (1, 4, 7):
        circ = W.random_circuit(n, 40, seed=n) if n > 1 else [("H", (0,), ()), ("T", (0,), ())]
        for enc, kw in [("c128", {}), ("compact", {"compact_mode": PER_BLOCK})]:
            order, blen, fused = schedule(n, enc, circ, **kw)
            assert not any(fused) and order == non_identity(circ)


def test_keeps_modulus_blocks_are_recognisable():
    # a layer of RZ and the CNOT chain: every block keeps all moduli, so a
    # per-block compact run keeps the range (checked on the GPU); here the
    # blocks must exist and cover the circuit
    n = 14
    circ = W.rz_cnot_chain(n, 2, seed=1)
    order, blen, fused = schedule(n, "compact", circ, compact_mode=PER_BLOCK)
    assert any(fused) and sum(blen) == len(circ)


def test_schedule_errors():
    circ = [("H", (0,), ())]
    with pytest.raises(jq.JqError):
        jq.plan_schedule(0, "c128", circ)
    with pytest.raises(jq.JqError):
        jq.plan_schedule(4, 7, circ)
    with pytest.raises(jq.JqError):
        jq.plan_schedule(4, "compact", circ, compact_mode=5)
    with pytest.raises(jq.JqError) as e:
        jq.plan_schedule(2, "c128", [("H", (0,), ()), ("H", (2,), ())])
    assert e.value.code == jq.JQ_EINVAL and "gate 1" in str(e.value)


# gates that are exact on the two-byte code (permutations and phase shifts by
# an integer number of code units: 128 arg / pi is an integer or at least not
# within 1e-6 of a half-integer)
CODE_NAMES = {"X", "CNOT", "TOFFOLI", "Z", "S", "T", "S+", "T+", "CZ", "RZ", "U1", "R", "U", "CP"}


def is_code_op(g):
    name, p = g[0], g[2]
    if name not in CODE_NAMES:
        return False
    if name in ("U", "R"):      # phase 2 pi / 2^k: 256 / 2^k code units
        return int(p[0]) <= 8
    if name == "CP":            # phase p[0]
        return not (abs((128 * p[0] / math.pi) % 1 - 0.5) < 1e-6)
    if name in ("RZ", "U1"):
        d = 128 * p[0] / 2 / math.pi if name == "RZ" else 128 * p[0] / math.pi
        return not (abs(d % 1 - 0.5) < 1e-6)
    return True


@pytest.mark.parametrize("n,seed", [(12, 1), (14, 2), (20, 3)])
def test_compact_per_gate_fuses_only_exact_code_runs(n, seed):
    # per-gate quantisation: fused blocks hold only ops exact on the codes,
    # and no gate moves past a gate that decodes (everything before such a
    # gate in the input stays before it)
    circ = W.random_circuit(n, 200, seed=seed) + W.rz_cnot_chain(n, 2, seed=seed)
    order, blen, fused = schedule(n, "compact", circ)
    assert sorted(order) == non_identity(circ) and any(fused)
    pos = 0
    for b, f in zip(blen, fused):
        if f:
            assert all(is_code_op(circ[i]) for i in order[pos:pos + b]), [circ[i][0] for i in order[pos:pos + b]]
        pos += b
    where = {g: k for k, g in enumerate(order)}
    for i, g in enumerate(circ):
        if g[0] == "I" or is_code_op(g):
            continue
        before = {j for j in range(i) if circ[j][0] != "I"}
        assert set(order[:where[i]]) == before, (i, g[0])
    # tile: qubits 0, 1 in register slots, lane bits qubits 2..7, at most
    # five more register qubits
    pos = 0
    for b, f in zip(blen, fused):
        blk = [circ[i] for i in order[pos:pos + b]]
        pos += b
        if f:
            assert len({q for g in blk for q in targets_of(g)} - set(range(8))) <= 5


def test_compact_rz_cnot_layer_is_a_few_passes():
    # the 37-qubit RZ + CNOT-chain layer: 73 gates in a handful of code
    # passes.  Qubits 0..7 are in every tile and the default pass has five
    # more register qubits, so the 29 CNOT targets above qubit 7 need at
    # least 6 passes
    n = 37
    circ = W.rz_cnot_chain(n, 1, seed=37)
    order, blen, fused = schedule(n, "compact", circ)
    # a trailing gate may run alone when that moves fewer bytes than a pass
    assert len(blen) <= 8 and sum(b for b, f in zip(blen, fused) if f) >= len(circ) - 2, list(blen)
    # one register qubit fewer per pass: more passes
    _, blen6, _ = schedule(n, "compact", circ, fusion=6)
    assert len(blen6) > len(blen)


@pytest.mark.parametrize("enc,big_n", [("c128", 26), ("c64", 27), ("compact", 29)])
def test_deep_circuits_reorder_only_commuting_gates(enc, big_n):
    # many layers give the tile-slot search (on for states of 1 GiB and more)
    # room to pull later gates of some qubits ahead of earlier gates of
    # others; the result must stay the same unitary.  The circuits use the
    # low 14 qubits of a big state, so the oracle replays them on 14 qubits
    n = 14
    circs = [W.rz_cnot_chain(n, 25, seed=6)]
    if enc != "compact":  # Haar U(2) gates never run in code passes
        circs.append(W.layered_u2_cz(n, 25, seed=5))
    for circ in circs:
        order, blen, fused = schedule(big_n, enc, circ)
        assert sorted(order) == non_identity(circ)
        assert sum(fused) > 0
        rng = np.random.default_rng(3)
        psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
        psi /= np.linalg.norm(psi)
        a = O.run(psi.copy(), n, circ)
        b = O.run(psi.copy(), n, [circ[i] for i in order])
        assert O.rel_l2(b, a) < 1e-12


def test_tile_slot_search_shortens_rz_cnot_chains():
    # 40 layers of RZ + CNOT chain at N=30 (complex128: 7 free tile qubits per
    # pass).  Filling the slots first come, first served stalls on CNOTs
    # whose control is still behind (144 passes); letting a later qubit take
    # the slot of one that stalls early retires the circuit in 61-66 (the
    # search weighs passes against ops, and grouped diagonals make ops fewer)
    n = 30
    circ = W.rz_cnot_chain(n, 40, seed=7)
    order, blen, fused = schedule(n, "c128", circ)
    assert all(fused) and len(blen) <= 72, len(blen)
    # the layered Haar U(2) + CZ circuit: 62 passes before the search
    _, blen, fused = schedule(n, "c128", W.layered_u2_cz(n, 40, seed=2018))
    assert all(fused) and len(blen) <= 57, len(blen)


def test_search_switch_reaches_small_states():
    # the large-state steps (tile-slot search, register/lane split, lane
    # order) are on by default only for states of 1 GiB or more; the switch
    # turns them on at any size, which changes the passes of a deep circuit
    # at N=16, and off at any size, which reproduces the small-state plan
    n = 16
    circ = W.rz_cnot_chain(n, 12, seed=2) + W.layered_u2_cz(n, 6, seed=3)
    auto = jq.plan_steps(n, "c128", circ)
    on = jq.plan_steps(n, "c128", circ, search=jq.JQ_SEARCH_ON)
    off = jq.plan_steps(n, "c128", circ, search=jq.JQ_SEARCH_OFF)
    key = lambda st: [(s["fused"], s["reg_q"], s["lane_q"], s["n_gates"]) for s in st]
    assert key(auto) == key(off)
    assert key(on) != key(off)
    # at N=26 (1 GiB of complex128) the default is the searched plan
    big = 26
    assert key(jq.plan_steps(big, "c128", circ)) == key(jq.plan_steps(big, "c128", circ, search=jq.JQ_SEARCH_ON))
    assert key(jq.plan_steps(big, "c128", circ)) != key(jq.plan_steps(big, "c128", circ, search=jq.JQ_SEARCH_OFF))


def test_bad_options_are_rejected():
    circ = [("H", (0,), ())]
    for kw in ({"search": 3}, {"search": -1}):
        with pytest.raises(jq.JqError) as e:
            jq.plan_schedule(10, "c128", circ, **kw)
        assert e.value.code == jq.JQ_EINVAL
    opts = jq.exec_opts()
    opts.reserved[2] = 1
    arr, cnt = jq.gates(circ)
    n_steps = jq.ctypes.c_size_t()
    rc = jq.lib().jq_plan_steps(10, jq.JQ_C128, arr, cnt, jq.ctypes.byref(opts), None, 0, jq.ctypes.byref(n_steps))
    assert rc == jq.JQ_EINVAL


# per-slot diagonal tables: (encoding, options) -> (tag, 2^K fits the op)
TABLE_CASES = [("c128", {}, 1, True), ("c128", {"fusion": 5}, 1, False), ("c64", {}, 2, True),
               ("c64", {"fusion": 6}, 2, False), ("compact", {"compact_mode": PER_BLOCK}, 1, True),
               ("c128", SEARCH_ON, 1, True), ("c64", SEARCH_ON, 2, True)]


@pytest.mark.parametrize("enc,kw,tag,fits", TABLE_CASES)
def test_diagonal_tables_carry_the_kernel_element_type(enc, kw, tag, fits):
    # one-qubit diagonals on register qubits run as a table of their product
    # per slot in the fused kernel's element type (FP64 pairs for complex128
    # and the two-byte code's decoding kernel, at most 16 slots; FP32 pairs for
    # complex64, at most 32): where 2^K slots fit, some pass carries tables and
    # every tag is the kernel's; where they do not, no pass carries one
    n = 16
    circ = W.rz_cnot_chain(n, 4, seed=11)
    steps = [s for s in jq.plan_steps(n, enc, circ, **kw) if s["fused"]]
    assert steps
    for s in steps:
        assert s["table_tag"] in (0, tag), s
        assert (s["n_tables"] > 0) == (s["table_tag"] != 0), s
    if fits:
        assert any(s["n_tables"] for s in steps)
    else:
        assert not any(s["n_tables"] for s in steps)

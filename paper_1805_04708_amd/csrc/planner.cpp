// Fusion planner: groups consecutive gates into register-blocked tile passes.
//
// The paper notes that single- and two-qubit gates stream the whole state
// for a few flops per amplitude and proposes combining them into
// multi-qubit blocks to raise the arithmetic intensity (Sec. 5.2).  Here a
// pass loads a tile of 2^(6+K) amplitudes per wavefront - 64 lanes times
// 2^K registers - whose index bits are the F low bits (so eight or sixteen
// lanes read one 128-byte line), 6-F further lane qubits and K register
// qubits.  Any gate whose target lies in the tile can run in the pass:
// register targets in-thread, lane targets with cross-lane exchanges.
// Diagonal gates and controls need no tile bit at all: the index bits they
// test are known to each thread.
//
// Gates may be taken out of order only past gates they commute with: a
// gate joins the pass only if it shares no qubit with any gate skipped so
// far (diagonal gates may pass skipped diagonal gates).
//
// Which qubits take the free tile slots decides how far a pass gets: a scan
// that fills them first come, first served can spend a slot on a qubit that
// stalls at once (a CNOT from a qubit that is still behind, say).  Each pass
// therefore also tries scans that shut one of the chosen qubits out and keeps
// the one that retires the most work per unit of estimated pass time (a
// fixed streaming cost plus the arithmetic of its ops).
#include <algorithm>

#include "internal.hpp"

namespace jq {

namespace {

// Qubits 0..R+F-1 are always in the tile (R fixed register slots, then F
// fixed lane bits); the builder places the other targets.
struct PassBuilder {
    int n, F, K, max_ops, R;
    uint64_t banned;          // qubits this pass may not place
    std::vector<int> reg_q;   // qubits in the free register slots R..K-1
    std::vector<int> lane_q;  // qubits in lane bits F..5
    std::vector<int> taken;   // op indices
    uint64_t tile() const {
        uint64_t t = (1ull << (R + F)) - 1;
        for (int q : reg_q) t |= 1ull << q;
        for (int q : lane_q) t |= 1ull << q;
        return t;
    }
    bool holds(int q) const {
        return q < R + F || std::find(reg_q.begin(), reg_q.end(), q) != reg_q.end() ||
               std::find(lane_q.begin(), lane_q.end(), q) != lane_q.end();
    }
    // Can targets q0 and q1 (-1: none) be placed (or are they already)?
    // Places them if so (register slots first), else changes nothing.
    bool place(int q0, int q1 = -1) {
        int add[2], n_add = 0;
        for (int q : {q0, q1}) {
            if (q < 0 || holds(q) || (n_add == 1 && add[0] == q)) continue;
            if ((banned >> q) & 1) return false;
            add[n_add++] = q;
        }
        const int free_slots = (K - R - (int)reg_q.size()) + (6 - F - (int)lane_q.size());
        if (n_add > free_slots) return false;
        for (int i = 0; i < n_add; ++i) {
            if ((int)reg_q.size() < K - R) reg_q.push_back(add[i]);
            else lane_q.push_back(add[i]);
        }
        return true;
    }
};

double touched_fraction(const GateOp& op, int n) {
    return std::ldexp((double)op.touched(n), -n);
}

// A SWAP (controls allowed): the two-qubit dense op whose matrix exchanges
// |01> and |10>.  It is a permutation, so it runs in a pass as three
// controlled X ops (exact on the two-byte code too).
bool is_swap(const GateOp& op) {
    if (op.kind != OP_DENSE2) return false;
    for (int i = 0; i < 16; ++i) {
        const double want = (i == 0 || i == 6 || i == 9 || i == 15) ? 1.0 : 0.0;
        if (op.m[i].re != want || op.m[i].im != 0.0) return false;
    }
    return true;
}

// Index bits whose values an op changes (none for a diagonal op).
uint64_t changed_bits(const GateOp& op) {
    if (op.kind == OP_DIAG) return 0;
    uint64_t t = 1ull << op.t0;
    if (op.kind == OP_DENSE2) t |= 1ull << op.t1;
    return t;
}

// Can the op run inside a fused pass?  Two-qubit dense ops other than SWAP
// never do; on the two-byte code with per-gate quantisation only the ops
// that are exact on the codes do: permutations (SWAP included) and phase
// shifts by a non-tie integer.
bool fusable(const GateOp& op, const PlanConfig& cfg) {
    if (op.kind == OP_DENSE2) return is_swap(op);
    if (!cfg.code_domain) return true;
    if (op.kind == OP_PERMX) return true;
    double d[4];
    return op.kind == OP_DIAG && op.keeps_modulus && phase_code_shifts(op, d);
}

// Bytes the op moves as a per-gate kernel, in units of one fused pass
// (state vector: the touched amplitudes read and written; two-byte code: a
// permutation reads and writes both planes of the touched amplitudes, a phase
// shift reads the modulus plane and reads and writes the phase plane).
double single_cost(const GateOp& op, const PlanConfig& cfg) {
    const double t = touched_fraction(op, cfg.n);
    // a SWAP alone runs the two-qubit dense kernel (the two-byte code:
    // decode, 4x4 product, encode), which costs more than a pass
    if (is_swap(op)) return 2.0 * t;
    if (!cfg.code_domain) return t;
    return op.kind == OP_PERMX ? t : 0.75 * t;
}

FOp lower_fop(const GateOp& op, const FPass& p, int F, int K, int nmux = 0, const int* mux = nullptr,
              const cd (*mats)[4] = nullptr, bool code_domain = false) {
    FOp f{};
    auto reg_of = [&](int q) {
        for (int j = 0; j < K; j++) if (p.reg_q[j] == q) return j;
        return -1;
    };
    auto lane_of = [&](int q) {
        for (int b = 0; b < 6; b++) if (p.lane_q[b] == q) return b;
        return -1;
    };
    uint64_t reg_bits = 0;
    for (int j = 0; j < K; j++) reg_bits |= 1ull << p.reg_q[j];
    f.thr_ctrl = op.cmask & ~reg_bits;
    f.reg_ctrl = 0;
    for (int j = 0; j < K; j++) if (op.cmask & (1ull << p.reg_q[j])) f.reg_ctrl |= 1u << j;
    f.has_ctrl = op.cmask != 0;
    f.sel_reg[0] = f.sel_reg[1] = -1;
    f.sel_glob[0] = f.sel_glob[1] = -1;
    if (op.kind == OP_DENSE1 || op.kind == OP_PERMX) {
        const bool ctrl = op.cmask != 0;
        int j = reg_of(op.t0);
        if (j >= 0) {
            f.kind = op.kind == OP_DENSE1 ? (ctrl ? F_CDENSE_REG : F_DENSE_REG) : F_PERM_REG;
            f.slot = j;
        } else {
            int b = lane_of(op.t0);
            if (b < 0) fail(JQ_EDEVICE, "planner: target outside the tile");
            f.kind = op.kind == OP_DENSE1 ? (ctrl ? F_CDENSE_LANE : F_DENSE_LANE) : F_PERM_LANE;
            f.slot = b;
        }
        for (int i = 0; i < 4; i++) {
            f.m[2 * i] = op.m[i].re;
            f.m[2 * i + 1] = op.m[i].im;
        }
        if (nmux > 0) {
            f.kind = (f.kind == F_DENSE_REG) ? F_MDENSE_REG : F_MDENSE_LANE;
            f.nsel = nmux;
            for (int i = 0; i < nmux; i++) {
                int jr = reg_of(mux[i]);
                if (jr >= 0) f.sel_reg[i] = jr;
                else f.sel_glob[i] = mux[i];
                if (jr < 0 && lane_of(mux[i]) >= 0) f.sel_lane |= 1 << i;
            }
            for (int v = 0; v < (1 << nmux); v++)
                for (int i = 0; i < 4; i++) {
                    f.m[8 * v + 2 * i] = mats[v][i].re;
                    f.m[8 * v + 2 * i + 1] = mats[v][i].im;
                }
        }
        return f;
    }
    if (op.kind == OP_DIAG && code_domain) {
        // integer phase-code shift per selector value (rint of a non-tie shift)
        f.kind = F_CSHIFT;
        f.nsel = op.nsel;
        int sel[2] = {op.t0, op.t1};
        for (int i = 0; i < op.nsel; i++) {
            int j = reg_of(sel[i]);
            if (j >= 0) f.sel_reg[i] = j;
            else f.sel_glob[i] = sel[i];
        }
        double d[4];
        phase_code_shifts(op, d);
        int64_t m[4];
        for (int i = 0; i < 4; i++) {
            f.m[i] = std::rint(d[i]);
            m[i] = (int64_t)f.m[i];
        }
        // the shift for selector values (v0, v1) (first selector the MSB) is
        // m[2 v0 + v1] = A + B v0 + C v1 + D v0 v1 (one selector: m[v0] =
        // A + B v0), each term added where its selector bits are 1; the sums
        // are exact integers and only their value mod 256 is kept
        int64_t coef[4] = {m[0], 0, 0, 0};
        if (op.nsel == 1) coef[1] = m[1] - m[0];
        if (op.nsel == 2) {
            coef[1] = m[2] - m[0];
            coef[2] = m[1] - m[0];
            coef[3] = m[3] - m[2] - m[1] + m[0];
        }
        // term t holds the selectors of its bits (bit 0: first, bit 1: second)
        f.cs_n = 0;
        for (int t = 0; t < 4; t++) {
            const uint32_t add = (uint32_t)(coef[t] & 255) << 8;
            if (add == 0) continue;
            uint32_t rm = f.reg_ctrl;
            uint64_t tm = f.thr_ctrl;
            for (int i = 0; i < 2; i++) {
                if (!(t >> i & 1)) continue;
                if (f.sel_reg[i] >= 0) rm |= 1u << f.sel_reg[i];
                else tm |= 1ull << f.sel_glob[i];
            }
            f.cs_reg[f.cs_n] = rm;
            f.cs_thr[f.cs_n] = tm;
            f.cs_add[f.cs_n] = add;
            f.cs_n++;
        }
        return f;
    }
    if (op.kind == OP_DIAG) {
        f.kind = F_DIAG;
        if (op.nsel == 0) f.kind = (op.m[0].re == -1.0 && op.m[0].im == 0.0) ? F_NEG : F_PHASE;
        f.nsel = op.nsel;
        int sel[2] = {op.t0, op.t1};
        for (int i = 0; i < op.nsel; i++) {
            int j = reg_of(sel[i]);
            if (j >= 0) f.sel_reg[i] = j;
            else f.sel_glob[i] = sel[i];
            if (j < 0 && lane_of(sel[i]) >= 0) f.sel_lane |= 1 << i;
        }
        for (int i = 0; i < 4; i++) {
            f.m[2 * i] = op.m[i].re;
            f.m[2 * i + 1] = op.m[i].im;
        }
        return f;
    }
    fail(JQ_EDEVICE, "planner: op kind cannot run in a fused pass");
}

// A gate of a pass with its multiplexer: for each value v of the selector
// qubits (sel[0] the most significant bit) the 2x2 matrix mats[v].
struct PassOp {
    GateOp op;
    int nsel = 0;
    int sel[2] = {-1, -1};
    cd mats[4][4];
    bool alive = true;
};

// Value of a diagonal op at a full assignment of its qubits (bit q of idx).
cd diag_value(const GateOp& d, uint64_t idx) {
    if ((idx & d.cmask) != d.cmask) return {1.0, 0.0};
    int sel = 0;
    if (d.nsel >= 1) sel = (int)((idx >> d.t0) & 1);
    if (d.nsel == 2) sel = 2 * sel + (int)((idx >> d.t1) & 1);
    return d.m[sel];
}

cd cmulh(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

// Fold diagonal op d into the uncontrolled dense op u on target t in its
// support: for every value of the other qubits of d, d acts on t as
// diag(f0, f1), so u*d (d applied first) has matrix m[r][c] * f_c and d*u
// has f_r * m[r][c].  The other qubits of d become (further) multiplexer
// selectors of u.  Returns false if that would need more than two.
bool absorb(PassOp& u, const GateOp& d, bool d_first, uint64_t reg_bits) {
    const int t = u.op.t0;
    uint64_t q = d.support() & ~(1ull << t);
    int sel[2] = {u.sel[0], u.sel[1]};
    int nsel = u.nsel;
    for (int b = 0; b < 64; ++b) {
        if (!(q & (1ull << b))) continue;
        if ((nsel >= 1 && sel[0] == b) || (nsel == 2 && sel[1] == b)) continue;
        if (nsel == 2) return false;
        sel[nsel++] = b;
    }
    // the kernel resolves selectors per thread: none may be a register slot
    for (int i = 0; i < nsel; ++i)
        if ((reg_bits >> sel[i]) & 1) return false;
    cd mats[4][4];
    for (int v = 0; v < (1 << nsel); ++v) {
        uint64_t idx = 0;
        for (int i = 0; i < nsel; ++i)
            if ((v >> (nsel - 1 - i)) & 1) idx |= 1ull << sel[i];
        // matrix of u for this selector value
        int vo = 0;
        for (int i = 0; i < u.nsel; ++i) vo = 2 * vo + (int)((idx >> u.sel[i]) & 1);
        const cd* m = u.mats[vo];
        const cd f0 = diag_value(d, idx), f1 = diag_value(d, idx | (1ull << t));
        const cd f[2] = {f0, f1};
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) mats[v][2 * r + c] = d_first ? cmulh(m[2 * r + c], f[c]) : cmulh(f[r], m[2 * r + c]);
    }
    u.nsel = nsel;
    u.sel[0] = sel[0];
    u.sel[1] = sel[1];
    std::memcpy(u.mats, mats, sizeof(mats));
    return true;
}

bool absorbable(const PassOp& p) {
    return p.alive && p.op.kind == OP_DENSE1 && p.op.cmask == 0;
}

// The ops of a pass in emission order: a single pass op, or a group of
// uncontrolled one-qubit diagonals on lane or outer qubits that runs as one
// F_DGROUP op (one factor per thread).  Such diagonals on a qubit outside
// the tile commute with every op of the pass (none changes that bit): they
// all run together at its end.  Those on lane qubits group with the
// diagonals around them, up to the next non-diagonal op, and so do those on
// register qubits when the op can hold a table of their product per slot
// (reg_table: 16 slots of double pairs, or 32 of float pairs for complex64);
// otherwise they stay ops of their own.
struct PassItem {
    int pop = -1;
    std::vector<int> group;
};

std::vector<PassItem> emit_order(const std::vector<PassOp>& pops, uint64_t tile_bits, uint64_t reg_bits,
                                 bool code_domain, bool reg_table) {
    std::vector<PassItem> out;
    std::vector<int> run, outer;
    auto put_group = [&](const std::vector<int>& g, bool always) {
        if (g.size() == 1 && !always) {
            out.push_back(PassItem{g[0], {}});
            return;
        }
        for (size_t i = 0; i < g.size(); i += kMaxOdiag) {
            PassItem it;
            it.group.assign(g.begin() + i, g.begin() + std::min(g.size(), i + kMaxOdiag));
            out.push_back(it);
        }
    };
    for (int i = 0; i < (int)pops.size(); ++i) {
        const PassOp& po = pops[i];
        if (!po.alive) continue;
        const bool one = !code_domain && po.op.kind == OP_DIAG && po.op.cmask == 0 && po.op.nsel == 1 &&
                         (reg_table || !((reg_bits >> po.op.t0) & 1));
        if (one && !((tile_bits >> po.op.t0) & 1)) {
            outer.push_back(i);
        } else if (one) {
            run.push_back(i);
        } else if (po.op.kind == OP_DIAG) {
            out.push_back(PassItem{i, {}});
        } else {
            put_group(run, false);
            run.clear();
            out.push_back(PassItem{i, {}});
        }
    }
    put_group(run, false);
    put_group(outer, true);
    return out;
}

// Move each diagonal op of the pass onto a neighbouring uncontrolled dense
// op that acts on one of its qubits, past ops whose (non-diagonal) target
// lies outside its support; such ops commute with it.
void absorb_diagonals(std::vector<PassOp>& ops, uint64_t reg_bits) {
    for (size_t i = 0; i < ops.size(); ++i) {
        if (!ops[i].alive || ops[i].op.kind != OP_DIAG) continue;
        const GateOp d = ops[i].op;
        const uint64_t q = d.support();
        bool done = false;
        for (size_t j = i + 1; j < ops.size() && !done; ++j) {
            PassOp& u = ops[j];
            if (!u.alive || u.op.kind == OP_DIAG) continue;
            if (!(q & changed_bits(u.op))) continue;
            if (absorbable(u) && absorb(u, d, true, reg_bits)) done = true;
            break;
        }
        for (size_t j = i; j-- > 0 && !done;) {
            PassOp& u = ops[j];
            if (!u.alive || u.op.kind == OP_DIAG) continue;
            if (!(q & changed_bits(u.op))) continue;
            if (absorbable(u) && absorb(u, d, false, reg_bits)) done = true;
            break;
        }
        if (done) ops[i].alive = false;
    }
}

uint64_t lane_bits_of(const FPass& p) {
    uint64_t m = 0;
    for (int b = 0; b < 6; ++b) m |= 1ull << p.lane_q[b];
    return m;
}

uint64_t sel_mask(const PassOp& p) {
    uint64_t m = 0;
    for (int i = 0; i < p.nsel; ++i) m |= 1ull << p.sel[i];
    return m;
}

// Every qubit an op reads or changes: target(s), controls, diagonal
// selectors, multiplexer selectors.
uint64_t involved(const PassOp& p) { return p.op.support() | sel_mask(p); }

// b after a on the same target (both uncontrolled dense): one multiplexed
// 2x2 whose matrix for selector value v is B(v) A(v).  False if the union of
// their selectors has more than two bits.
bool merge_into(PassOp& b, const PassOp& a) {
    int sel[2] = {b.sel[0], b.sel[1]};
    int nsel = b.nsel;
    for (int i = 0; i < a.nsel; ++i) {
        const int q = a.sel[i];
        if ((nsel >= 1 && sel[0] == q) || (nsel == 2 && sel[1] == q)) continue;
        if (nsel == 2) return false;
        sel[nsel++] = q;
    }
    cd mats[4][4];
    for (int v = 0; v < (1 << nsel); ++v) {
        uint64_t idx = 0;
        for (int i = 0; i < nsel; ++i)
            if ((v >> (nsel - 1 - i)) & 1) idx |= 1ull << sel[i];
        int va = 0, vb = 0;
        for (int i = 0; i < a.nsel; ++i) va = 2 * va + (int)((idx >> a.sel[i]) & 1);
        for (int i = 0; i < b.nsel; ++i) vb = 2 * vb + (int)((idx >> b.sel[i]) & 1);
        const cd* A = a.mats[va];
        const cd* B = b.mats[vb];
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) {
                const cd x = cmulh(B[2 * r], A[c]), y = cmulh(B[2 * r + 1], A[2 + c]);
                mats[v][2 * r + c] = {x.re + y.re, x.im + y.im};
            }
    }
    b.nsel = nsel;
    b.sel[0] = sel[0];
    b.sel[1] = sel[1];
    std::memcpy(b.mats, mats, sizeof(mats));
    return true;
}

// Merge each uncontrolled dense op into the next uncontrolled dense op on
// the same target when every op in between leaves the target and the
// first op's selectors alone (then the first op commutes with all of them).
void merge_same_target(std::vector<PassOp>& ops) {
    for (size_t i = 0; i < ops.size(); ++i) {
        PassOp& a = ops[i];
        if (!absorbable(a)) continue;
        const int t = a.op.t0;
        const uint64_t tb = 1ull << t, sa = sel_mask(a);
        for (size_t j = i + 1; j < ops.size(); ++j) {
            PassOp& c = ops[j];
            if (!c.alive) continue;
            if (absorbable(c) && c.op.t0 == t) {
                if (merge_into(c, a)) a.alive = false;
                break;
            }
            if (involved(c) & tb) break;
            if (sa & changed_bits(c.op)) break;
        }
    }
}

}  // namespace

namespace {

// A gate that every fused pass lowers to an op of kLiteKinds: an
// uncontrolled one-qubit dense gate (a 2x2, or a multiplexed 2x2 once
// diagonals fold into it) or a controlled Z on two or more qubits (a
// negation, or a selector of a multiplexed 2x2).
bool lowers_to_reduced_kinds(const GateOp& op) {
    if (op.kind == OP_DENSE1) return op.cmask == 0;
    return op.kind == OP_DIAG && op.nsel == 0 && __builtin_popcountll(op.cmask) >= 2 && op.m[0].re == -1.0 &&
           op.m[0].im == 0.0;
}

}  // namespace

Plan make_plan(const std::vector<GateOp>& ops, const PlanConfig& cfg_in, const StepSink& on_step) {
    // Passes that hold any other op run the kernel compiled for every kind,
    // whose registers at a wider width leave 2-3 waves per SIMD (complex128
    // with 2^5 slots: 217 VGPRs, passes twice as slow as with 2^4): keep
    // such circuits at the width where it still runs 4.
    PlanConfig cfg = cfg_in;
    if (cfg.fuse && !cfg.k_explicit && cfg.k_general_max > 0 && cfg.k_reg > cfg.k_general_max &&
        !std::all_of(ops.begin(), ops.end(), lowers_to_reduced_kinds))
        cfg.k_reg = cfg.k_general_max;
    Plan plan;
    auto emit = [&](Step&& s) {
        plan.steps.push_back(std::move(s));
        if (on_step) on_step(plan);
    };
    const int n = cfg.n, F = cfg.fixed_lane_bits, K = cfg.k_reg;
    if (cfg.table_elem != 4 && cfg.table_elem != 8) fail(JQ_EINVAL, "planner: table element must be 4 or 8 bytes");
    // per-slot tables of register diagonals: in the fused kernel's element
    // type, when all 2^K slots fit one op
    const int table_tag = cfg.table_elem == 4 ? kDgTableF32 : kDgTableF64;
    const bool reg_table = (1 << K) <= (cfg.table_elem == 4 ? kDgSlotsF32 : kDgSlotsF64);
    const bool can_fuse = cfg.fuse && K >= 1 && K >= cfg.fixed_reg_bits && n >= 6 + K && 6 + K <= kMaxTileBits;
    if (!can_fuse) {
        for (const auto& op : ops) {
            Step s;
            s.op = op;
            s.n_gates = 1;
            s.gates.push_back((int)plan.steps.size());
            emit(std::move(s));
        }
        return plan;
    }
    std::vector<int> remaining(ops.size());
    for (size_t i = 0; i < ops.size(); i++) remaining[i] = (int)i;
    const size_t window = 4096;
    std::vector<char> fus(ops.size());
    for (size_t i = 0; i < ops.size(); ++i) fus[i] = fusable(ops[i], cfg);
    // One scan: take every gate, in order, that can join the pass; targets
    // take the free tile slots first come, first served.
    auto scan = [&](uint64_t banned) {
        PassBuilder pb{n, F, K, cfg.max_ops, cfg.fixed_reg_bits, banned, {}, {}, {}};
        uint64_t blk_any = 0, blk_diag = 0;
        size_t scanned = 0;
        for (size_t r = 0; r < remaining.size() && scanned < window; r++, scanned++) {
            const GateOp& op = ops[remaining[r]];
            const uint64_t sup = op.support();
            const bool diag = op.kind == OP_DIAG;
            // on the two-byte code with per-gate quantisation no gate may move
            // past one that decodes: the scan ends there
            if (cfg.code_domain && !fus[remaining[r]]) break;
            if ((sup & blk_any) || (!diag && (sup & blk_diag))) {
                (diag ? blk_diag : blk_any) |= sup;
                continue;
            }
            bool ok = true;
            if (!fus[remaining[r]]) {
                ok = false;  // two-qubit dense blocks run unfused
            } else if (!diag) {
                ok = pb.place(op.t0, op.kind == OP_DENSE2 ? op.t1 : -1);
            }
            if (!ok) {
                (diag ? blk_diag : blk_any) |= sup;
                continue;
            }
            pb.taken.push_back(remaining[r]);
            if ((int)pb.taken.size() >= cfg.max_ops) break;
        }
        return pb;
    };
    // Work a pass retires: non-diagonal gates count four times as much as
    // diagonal ones, which need no tile slot.
    auto work = [&](const PassBuilder& b) {
        int w = 0;
        for (int i : b.taken) w += ops[i].kind == OP_DIAG ? 1 : 4;
        return w;
    };
    const int R = cfg.fixed_reg_bits;
    // The pass layout for a builder (unused slots take the lowest qubits
    // outside the tile) and its op list after folding diagonals and merging
    // same-target gates; n_ops counts the kernel ops (a SWAP is three).
    struct Layout {
        FPass p;
        std::vector<PassOp> pops;
        int n_ops;
    };
    auto layout = [&](PassBuilder pb) {
        Layout L;
        uint64_t t = pb.tile();
        auto next_free = [&]() {
            for (int q = 0; q < n; q++)
                if (!(t & (1ull << q))) { t |= 1ull << q; return q; }
            fail(JQ_EDEVICE, "planner: no free qubit");
        };
        while ((int)pb.lane_q.size() < 6 - F) pb.lane_q.push_back(next_free());
        while ((int)pb.reg_q.size() < K - R) pb.reg_q.push_back(next_free());
        FPass& p = L.p;
        std::memset(&p, 0, sizeof(p));
        for (int j = 0; j < 8; j++) p.reg_q[j] = j < R ? j : j < K ? pb.reg_q[j - R] : -1;
        for (int b = 0; b < 6; b++) p.lane_q[b] = b < F ? R + b : pb.lane_q[b - F];
        std::vector<int> tb;
        for (int b = 0; b < 6; b++) tb.push_back(p.lane_q[b]);
        for (int j = 0; j < K; j++) tb.push_back(p.reg_q[j]);
        std::sort(tb.begin(), tb.end());
        p.n_tile = (int)tb.size();
        for (int i = 0; i < p.n_tile; i++) p.tile_sorted[i] = tb[i];
        L.pops.resize(pb.taken.size());
        for (size_t i = 0; i < pb.taken.size(); ++i) {
            L.pops[i].op = ops[pb.taken[i]];
            for (int e = 0; e < 4; ++e) L.pops[i].mats[0][e] = L.pops[i].op.m[e];
        }
        uint64_t reg_bits = 0;
        for (int j = 0; j < K; ++j) reg_bits |= 1ull << p.reg_q[j];
        if (cfg.absorb) {
            absorb_diagonals(L.pops, reg_bits);
            merge_same_target(L.pops);
        }
        L.n_ops = 0;
        for (const auto& it : emit_order(L.pops, reg_bits | lane_bits_of(p), reg_bits, cfg.code_domain, reg_table))
            L.n_ops += it.pop >= 0 && is_swap(L.pops[it.pop].op) ? 3 : 1;
        return L;
    };
    // Work per unit of pass time, the time being pass_ops (the pass's
    // streaming, in units of one op's arithmetic) plus its ops.
    auto rate = [&](const PassBuilder& b, const Layout& L) {
        return (double)work(b) / (cfg.pass_ops + L.n_ops);
    };
    while (!remaining.empty()) {
        // First come, first served can fill the tile with qubits that block
        // early (a gate coupling them to a qubit outside the tile that is
        // still behind); shutting one placed qubit out of the pass lets a
        // later one in.  Keep the scan with the best rate, a few times over.
        PassBuilder pb = scan(0);
        Layout L;
        if (!pb.taken.empty()) L = layout(pb);
        for (int it = 0; it < cfg.search_rounds && !pb.taken.empty(); ++it) {
            std::vector<int> placed = pb.reg_q;
            placed.insert(placed.end(), pb.lane_q.begin(), pb.lane_q.end());
            const uint64_t banned = pb.banned;
            double best = rate(pb, L);
            bool moved = false;
            for (int q : placed) {
                PassBuilder c = scan(banned | (1ull << q));
                if (c.taken.empty()) continue;
                Layout Lc = layout(c);
                const double rc = rate(c, Lc);
                if (rc > best) {
                    best = rc;
                    pb = std::move(c);
                    L = std::move(Lc);
                    moved = true;
                }
            }
            if (!moved) break;
        }
        // Which placed qubits sit in register slots and which in lane bits
        // decides what folds: a multiplexer selector must not be a register
        // slot, so a CZ to a register qubit stays an op of its own and keeps
        // the gates on either side of it from merging.  When a diagonal is
        // left over next to a foldable gate, try other splits and keep the
        // one with fewer ops, one swap at a time.
        if (cfg.search_rounds > 0 && cfg.absorb && !pb.taken.empty()) {
            bool dense = false, diag_left = false;
            for (const auto& po : L.pops) {
                if (!po.alive) continue;
                dense = dense || absorbable(po);
                diag_left = diag_left || po.op.kind == OP_DIAG;
            }
            // swap a register qubit with a lane qubit while that saves ops
            for (bool better = dense && diag_left; better;) {
                better = false;
                for (size_t i = 0; i < pb.reg_q.size() && !better; ++i)
                    for (size_t j = 0; j < pb.lane_q.size() && !better; ++j) {
                        PassBuilder c = pb;
                        std::swap(c.reg_q[i], c.lane_q[j]);
                        Layout Lc = layout(c);
                        if (Lc.n_ops < L.n_ops) {
                            pb = std::move(c);
                            L = std::move(Lc);
                            better = true;
                        }
                    }
            }
        }
        // Lane bit 5 exchanges through the LDS crossbar (a permute), the
        // lower lane bits by swizzles: give the highest lane bits to the
        // qubits that carry the fewest ops.
        if (cfg.search_rounds > 0 && pb.lane_q.size() > 1) {
            auto lane_ops = [&](int q) {
                int c = 0;
                for (const auto& po : L.pops)
                    if (po.alive && po.op.kind != OP_DIAG && po.op.t0 == q) ++c;
                return c;
            };
            std::vector<int> lq = pb.lane_q;
            std::stable_sort(lq.begin(), lq.end(), [&](int a, int b) { return lane_ops(a) > lane_ops(b); });
            if (lq != pb.lane_q) {
                pb.lane_q = lq;
                L = layout(pb);
            }
        }
        if (pb.taken.empty()) {
            // the first remaining gate cannot run fused: run it alone
            Step s;
            s.op = ops[remaining[0]];
            s.n_gates = 1;
            s.gates.push_back(remaining[0]);
            emit(std::move(s));
            remaining.erase(remaining.begin());
            continue;
        }
        // emit singles when they move fewer bytes than one full pass
        double singles = 0;
        for (int i : pb.taken) singles += single_cost(ops[i], cfg);
        std::vector<char> is_taken(ops.size(), 0);
        for (int i : pb.taken) is_taken[i] = 1;
        std::vector<int> rest;
        rest.reserve(remaining.size());
        for (int i : remaining) if (!is_taken[i]) rest.push_back(i);
        remaining.swap(rest);
        if (!cfg.always_pass && singles <= 1.0) {
            for (int i : pb.taken) {
                Step s;
                s.op = ops[i];
                s.n_gates = 1;
                s.gates.push_back(i);
                emit(std::move(s));
            }
            continue;
        }
        Step s;
        s.fused = true;
        s.k_reg = K;
        s.pass = L.p;
        s.pass.table_tag = 0;
        const FPass& p = s.pass;
        s.first_fop = plan.fops.size();
        int n_ops = 0;
        uint64_t reg_bits = 0;
        for (int j = 0; j < K; ++j) reg_bits |= 1ull << p.reg_q[j];
        for (const PassItem& it : emit_order(L.pops, reg_bits | lane_bits_of(p), reg_bits, cfg.code_domain, reg_table)) {
            if (it.pop < 0) {
                FOp f{};
                f.kind = F_DGROUP;
                f.sel_reg[0] = f.sel_reg[1] = f.sel_glob[0] = f.sel_glob[1] = -1;
                // register components: their product per slot
                cd table[kDgSlotsF32];
                for (auto& e : table) e = {1.0, 0.0};
                for (int g : it.group) {
                    const GateOp& d = L.pops[g].op;
                    for (int j = 0; j < K; ++j) {
                        if (p.reg_q[j] != d.t0) continue;
                        // emit_order groups register diagonals only when the
                        // table holds every slot
                        if (!reg_table) fail(JQ_EINVAL, "planner: register table exceeds its capacity");
                        f.slot = table_tag;
                        for (int s = 0; s < (1 << K); ++s) table[s] = cmulh(table[s], d.m[(s >> j) & 1]);
                    }
                }
                if (f.slot == kDgTableF32) {
                    float t32[2 * kDgSlotsF32];
                    for (int s = 0; s < (1 << K); ++s) {
                        t32[2 * s] = (float)table[s].re;
                        t32[2 * s + 1] = (float)table[s].im;
                    }
                    static_assert(sizeof(t32) <= sizeof(FOp::m), "float table fits the op");
                    std::memcpy(f.m, t32, sizeof(float) * 2 * (1 << K));
                } else if (f.slot == kDgTableF64) {
                    static_assert(2 * kDgSlotsF64 <= sizeof(FOp::m) / sizeof(double), "double table fits the op");
                    for (int s = 0; s < (1 << K); ++s) {
                        f.m[2 * s] = table[s].re;
                        f.m[2 * s + 1] = table[s].im;
                    }
                }
                if (f.slot) s.pass.table_tag = f.slot;
                f.n_od = 0;
                for (int g : it.group) {
                    const GateOp& d = L.pops[g].op;
                    if ((reg_bits >> d.t0) & 1) continue;
                    const int c = f.n_od++;
                    f.od_where[c] = 2;
                    f.od_idx[c] = d.t0;
                    for (int b = 0; b < 6; ++b)
                        if (p.lane_q[b] == d.t0) f.od_where[c] = 1, f.od_idx[c] = b;
                    f.od_m[4 * c] = d.m[0].re;
                    f.od_m[4 * c + 1] = d.m[0].im;
                    f.od_m[4 * c + 2] = d.m[1].re;
                    f.od_m[4 * c + 3] = d.m[1].im;
                }
                plan.fops.push_back(f);
                ++n_ops;
                continue;
            }
            PassOp& po = L.pops[it.pop];
            if (is_swap(po.op)) {
                // SWAP(a, b) = X on b where a = 1, X on a where b = 1, X on b
                // where a = 1 (each with the SWAP's own controls as well)
                const int a = po.op.t0, b = po.op.t1;
                GateOp xb;
                xb.kind = OP_PERMX;
                xb.t0 = b;
                xb.cmask = po.op.cmask | (1ull << a);
                xb.keeps_modulus = true;
                GateOp xa = xb;
                xa.t0 = a;
                xa.cmask = po.op.cmask | (1ull << b);
                for (const GateOp* x : {&xb, &xa, &xb})
                    plan.fops.push_back(lower_fop(*x, p, F, K, 0, nullptr, nullptr, cfg.code_domain));
                n_ops += 3;
                continue;
            }
            // a diagonal on the target alone folds into the matrix itself
            if (po.op.kind == OP_DENSE1 && po.nsel == 0)
                for (int e = 0; e < 4; ++e) po.op.m[e] = po.mats[0][e];
            plan.fops.push_back(lower_fop(po.op, p, F, K, po.nsel, po.sel, po.mats, cfg.code_domain));
            ++n_ops;
        }
        s.pass.n_ops = n_ops;
        s.pass.kinds = 0;
        for (size_t i = s.first_fop; i < plan.fops.size(); ++i) s.pass.kinds |= 1u << plan.fops[i].kind;
        s.n_gates = pb.taken.size();
        s.gates = pb.taken;
        emit(std::move(s));
    }
    return plan;
}

void check_table_tag(const FPass& p, int tag_of_kernel) {
    if (p.table_tag != 0 && p.table_tag != tag_of_kernel)
        fail(JQ_EINVAL, "fused pass: its diagonal tables are not in the kernel's element type");
}

}  // namespace jq

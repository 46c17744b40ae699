// Named instructions -> jq_gate, and jq_gate -> canonical device op.
//
// The instruction set is App. A of the paper.  Multi-qubit matrices are
// written in the basis |first listed qubit, ...> with the first qubit as the
// most significant bit, as App. A states for CNOT, U(k) and TOFFOLI.
#include <cmath>
#include <string>

#include "internal.hpp"

namespace jq {

namespace {

constexpr double kPi = 3.14159265358979323846;

void zero(jq_gate* g) {
    std::memset(g, 0, sizeof(*g));
}

void set(jq_gate* g, int idx, double re, double im) {
    g->m[2 * idx] = re;
    g->m[2 * idx + 1] = im;
}

void dense1(jq_gate* g, int q, cd a, cd b, cd c, cd d) {
    g->kind = JQ_DENSE;
    g->nq = 1;
    g->qubits[0] = q;
    set(g, 0, a.re, a.im);
    set(g, 1, b.re, b.im);
    set(g, 2, c.re, c.im);
    set(g, 3, d.re, d.im);
}

void diag1(jq_gate* g, int q, cd d0, cd d1) {
    g->kind = JQ_DIAGONAL;
    g->nq = 1;
    g->qubits[0] = q;
    set(g, 0, d0.re, d0.im);
    set(g, 1, d1.re, d1.im);
}

void diag2_phase(jq_gate* g, int a, int b, cd ph) {
    // diag(1, 1, 1, ph) on |a, b>
    g->kind = JQ_DIAGONAL;
    g->nq = 2;
    g->qubits[0] = a;
    g->qubits[1] = b;
    set(g, 0, 1, 0);
    set(g, 1, 1, 0);
    set(g, 2, 1, 0);
    set(g, 3, ph.re, ph.im);
}

cd expi(double a) { return {std::cos(a), std::sin(a)}; }
cd mul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
cd scale(double s, cd a) { return {s * a.re, s * a.im}; }

bool is_finite(const jq_gate& g) {
    for (double v : g.m)
        if (!std::isfinite(v)) return false;
    return true;
}

}  // namespace

int gate_named(const char* name_c, const int* q, int nq, const double* p, int np, jq_gate* out) {
    if (!name_c || !out || (nq > 0 && !q) || (np > 0 && !p) || nq < 0 || np < 0)
        fail(JQ_EINVAL, "jq_gate_named: null argument");
    std::string name(name_c);
    for (auto& ch : name) ch = (char)std::toupper((unsigned char)ch);
    zero(out);
    auto need = [&](int wq, int wp) {
        if (nq != wq || np != wp)
            fail(JQ_EINVAL, "jq_gate_named: " + name + " takes " + std::to_string(wq) + " qubit(s) and " +
                                std::to_string(wp) + " parameter(s)");
    };
    const double s2 = 1.0 / std::sqrt(2.0);
    if (name == "I") {
        need(1, 0);
        out->nq = 0;  // identity: nothing to do (App. A: a no-op)
        out->qubits[0] = q[0];
        return JQ_OK;
    }
    if (name == "H") { need(1, 0); dense1(out, q[0], {s2, 0}, {s2, 0}, {s2, 0}, {-s2, 0}); return JQ_OK; }
    if (name == "X") { need(1, 0); out->kind = JQ_PERM_X; out->nq = 1; out->qubits[0] = q[0]; return JQ_OK; }
    if (name == "Y") { need(1, 0); dense1(out, q[0], {0, 0}, {0, -1}, {0, 1}, {0, 0}); return JQ_OK; }
    if (name == "Z") { need(1, 0); diag1(out, q[0], {1, 0}, {-1, 0}); return JQ_OK; }
    if (name == "S") { need(1, 0); diag1(out, q[0], {1, 0}, {0, 1}); return JQ_OK; }
    if (name == "S+") { need(1, 0); diag1(out, q[0], {1, 0}, {0, -1}); return JQ_OK; }
    if (name == "T") { need(1, 0); diag1(out, q[0], {1, 0}, {s2, s2}); return JQ_OK; }
    if (name == "T+") { need(1, 0); diag1(out, q[0], {1, 0}, {s2, -s2}); return JQ_OK; }
    if (name == "U1") { need(1, 1); diag1(out, q[0], {1, 0}, expi(p[0])); return JQ_OK; }
    if (name == "RZ") { need(1, 1); diag1(out, q[0], expi(-p[0] / 2), expi(p[0] / 2)); return JQ_OK; }
    if (name == "R") {
        need(1, 1);
        long k = std::lround(p[0]);
        double ang = (k < 0 ? -1.0 : 1.0) * 2.0 * kPi / std::ldexp(1.0, (int)std::labs(k));
        diag1(out, q[0], {1, 0}, expi(ang));
        return JQ_OK;
    }
    if (name == "U2") {
        need(1, 2);
        double phi = p[0], lam = p[1];
        cd b = expi(lam);
        dense1(out, q[0], {s2, 0}, scale(-s2, b), scale(s2, expi(phi)), scale(s2, expi(phi + lam)));
        return JQ_OK;
    }
    if (name == "U3") {
        need(1, 3);
        double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2);
        dense1(out, q[0], {c, 0}, scale(-s, expi(p[2])), scale(s, expi(p[1])), scale(c, expi(p[1] + p[2])));
        return JQ_OK;
    }
    if (name == "+X") { need(1, 0); dense1(out, q[0], {s2, 0}, {0, s2}, {0, s2}, {s2, 0}); return JQ_OK; }
    if (name == "-X") { need(1, 0); dense1(out, q[0], {s2, 0}, {0, -s2}, {0, -s2}, {s2, 0}); return JQ_OK; }
    if (name == "+Y") { need(1, 0); dense1(out, q[0], {s2, 0}, {s2, 0}, {-s2, 0}, {s2, 0}); return JQ_OK; }
    if (name == "-Y") { need(1, 0); dense1(out, q[0], {s2, 0}, {-s2, 0}, {s2, 0}, {s2, 0}); return JQ_OK; }
    if (name == "MAT1") {
        need(1, 8);
        out->kind = JQ_DENSE;
        out->nq = 1;
        out->qubits[0] = q[0];
        for (int i = 0; i < 8; i++) out->m[i] = p[i];
        return JQ_OK;
    }
    if (name == "CNOT") {
        need(2, 0);
        out->kind = JQ_PERM_X;
        out->nq = 1;
        out->qubits[0] = q[1];
        out->nc = 1;
        out->controls[0] = q[0];
        return JQ_OK;
    }
    if (name == "TOFFOLI") {
        need(3, 0);
        out->kind = JQ_PERM_X;
        out->nq = 1;
        out->qubits[0] = q[2];
        out->nc = 2;
        out->controls[0] = q[0];
        out->controls[1] = q[1];
        return JQ_OK;
    }
    if (name == "U") {
        need(2, 1);
        long k = std::lround(p[0]);
        double ang = (k < 0 ? -1.0 : 1.0) * 2.0 * kPi / std::ldexp(1.0, (int)std::labs(k));
        diag2_phase(out, q[0], q[1], expi(ang));
        return JQ_OK;
    }
    if (name == "CZ") { need(2, 0); diag2_phase(out, q[0], q[1], {-1, 0}); return JQ_OK; }
    if (name == "CP") { need(2, 1); diag2_phase(out, q[0], q[1], expi(p[0])); return JQ_OK; }
    if (name == "SWAP" || name == "MAT2") {
        if (name == "SWAP") need(2, 0); else need(2, 32);
        out->kind = JQ_DENSE;
        out->nq = 2;
        out->qubits[0] = q[0];
        out->qubits[1] = q[1];
        if (name == "SWAP") {
            set(out, 0, 1, 0);
            set(out, 6, 1, 0);   // row 1, col 2
            set(out, 9, 1, 0);   // row 2, col 1
            set(out, 15, 1, 0);
        } else {
            for (int i = 0; i < 32; i++) out->m[i] = p[i];
        }
        return JQ_OK;
    }
    fail(JQ_EINVAL, "jq_gate_named: unknown instruction '" + name + "'");
}

namespace {

bool is_one(cd a) { return a.re == 1.0 && a.im == 0.0; }

// Is the 2^k x 2^k matrix (row-major interleaved) a permutation with exact
// 0/1 entries, or diagonal with every entry of modulus 1 (to 1e-12)?  These
// gates leave every modulus of the state unchanged.
bool keeps_modulus_dense(const double* m, int K) {
    bool perm = true;
    for (int r = 0; r < K && perm; r++) {
        int ones = 0;
        for (int c = 0; c < K; c++) {
            double re = m[2 * (r * K + c)], im = m[2 * (r * K + c) + 1];
            if (im != 0.0 || (re != 0.0 && re != 1.0)) { perm = false; break; }
            ones += re == 1.0;
        }
        if (ones != 1) perm = false;
    }
    if (perm) {
        for (int c = 0; c < K; c++) {
            int ones = 0;
            for (int r = 0; r < K; r++) ones += m[2 * (r * K + c)] == 1.0;
            if (ones != 1) { perm = false; break; }
        }
    }
    if (perm) return true;
    for (int r = 0; r < K; r++)
        for (int c = 0; c < K; c++) {
            double re = m[2 * (r * K + c)], im = m[2 * (r * K + c) + 1];
            if (r != c) {
                if (re != 0.0 || im != 0.0) return false;
            } else if (std::fabs(std::sqrt(re * re + im * im) - 1.0) > 1e-12) {
                return false;
            }
        }
    return true;
}

}  // namespace

GateOp canonicalize(const jq_gate& g, int n) {
    GateOp op;
    if (g.kind < JQ_DENSE || g.kind > JQ_PERM_X) fail(JQ_EINVAL, "gate: unknown kind " + std::to_string(g.kind));
    if (g.nq < 1 || g.nq > 2) fail(JQ_EINVAL, "gate: nq must be 1 or 2");
    if (g.kind == JQ_PERM_X && g.nq != 1) fail(JQ_EINVAL, "gate: PERM_X takes one target");
    if (g.nc < 0 || g.nc > JQ_MAX_CONTROLS) fail(JQ_EINVAL, "gate: too many controls");
    uint64_t seen = 0;
    auto take = [&](int q) {
        if (q < 0 || q >= n) fail(JQ_EINVAL, "gate: qubit " + std::to_string(q) + " out of range for N=" + std::to_string(n));
        if (seen & (1ull << q)) fail(JQ_EINVAL, "gate: qubit " + std::to_string(q) + " used twice");
        seen |= 1ull << q;
    };
    for (int i = 0; i < g.nq; i++) take(g.qubits[i]);
    for (int i = 0; i < g.nc; i++) {
        take(g.controls[i]);
        op.cmask |= 1ull << g.controls[i];
    }
    if (!is_finite(g)) fail(JQ_EINVAL, "gate: matrix has a non-finite entry");
    const int K = 1 << g.nq;
    auto at = [&](int i) { return cd{g.m[2 * i], g.m[2 * i + 1]}; };
    if (g.kind == JQ_PERM_X) {
        op.kind = OP_PERMX;
        op.t0 = g.qubits[0];
        op.keeps_modulus = true;
        return op;
    }
    if (g.kind == JQ_DENSE) {
        op.kind = g.nq == 1 ? OP_DENSE1 : OP_DENSE2;
        op.t0 = g.qubits[0];
        op.t1 = g.nq == 2 ? g.qubits[1] : -1;
        for (int i = 0; i < K * K; i++) op.m[i] = at(i);
        op.keeps_modulus = keeps_modulus_dense(g.m, K);
        return op;
    }
    // diagonal: entries d[i], i over the target bits (qubits[0] the MSB)
    {
        double full[32] = {};
        for (int i = 0; i < K; i++) {
            full[2 * (i * K + i)] = g.m[2 * i];
            full[2 * (i * K + i) + 1] = g.m[2 * i + 1];
        }
        op.keeps_modulus = keeps_modulus_dense(full, K);
    }
    op.kind = OP_DIAG;
    if (g.nq == 1) {
        int t = g.qubits[0];
        if (is_one(at(0))) {
            op.nsel = 0;
            op.cmask |= 1ull << t;
            op.m[0] = at(1);
        } else {
            op.nsel = 1;
            op.t0 = t;
            op.m[0] = at(0);
            op.m[1] = at(1);
        }
        return op;
    }
    int a = g.qubits[0], b = g.qubits[1];
    cd d0 = at(0), d1 = at(1), d2 = at(2), d3 = at(3);
    if (is_one(d0) && is_one(d1) && is_one(d2)) {
        op.nsel = 0;
        op.cmask |= (1ull << a) | (1ull << b);
        op.m[0] = d3;
    } else if (is_one(d0) && is_one(d1)) {  // acts only where a = 1: diag(d2, d3) on b
        op.nsel = 1;
        op.t0 = b;
        op.cmask |= 1ull << a;
        op.m[0] = d2;
        op.m[1] = d3;
    } else if (is_one(d0) && is_one(d2)) {  // acts only where b = 1: diag(d1, d3) on a
        op.nsel = 1;
        op.t0 = a;
        op.cmask |= 1ull << b;
        op.m[0] = d1;
        op.m[1] = d3;
    } else {
        op.nsel = 2;
        op.t0 = a;
        op.t1 = b;
        op.m[0] = d0;
        op.m[1] = d1;
        op.m[2] = d2;
        op.m[3] = d3;
    }
    return op;
}

bool phase_code_shifts(const GateOp& op, double d[4]) {
    constexpr double kPi = 3.14159265358979323846;
    bool clear = true;
    for (int i = 0; i < 4; ++i) {
        d[i] = (128.0 * std::atan2(op.m[i].im, op.m[i].re)) / kPi;
        const double f = d[i] - std::floor(d[i]);
        clear = clear && !(std::fabs(f - 0.5) < 1e-6);
    }
    return clear;
}

}  // namespace jq

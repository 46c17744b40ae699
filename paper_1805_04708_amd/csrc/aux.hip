// Amplitudes by the auxiliary-variable method (Sec. 4.2, Eqs. appa2-appa7).
//
// Each controlled phase shift U(a) (Eq. appa4) becomes a two-valued
// variable s via the discrete Hubbard-Stratonovich identity (Eqs. appa5,
// appa6): U(a) = (1/2) sum_s exp(i (sigma^z_0 + sigma^z_1)(x s - a/4)) with
// cos 2x = exp(ia/2), i.e. a diagonal single-qubit factor on each of its two
// qubits; CNOT is H_t U(pi) H_t.  For one assignment of the P variables
// every qubit then evolves alone from |0> (Eq. appa1), and an amplitude
// <b|psi> is 2^-P times the sum over assignments of the product of the
// qubits' components b_j (Eq. appa7).
//
// GPU mapping: one thread per assignment (grid-stride); the per-qubit item
// lists are uniform across threads and read through the scalar cache; each
// thread multiplies the components of up to kAuxChunk requested basis states
// into registers, and the sums over assignments are reduced in a fixed order
// (wave and block trees, then the blocks in order), so results are
// deterministic.  Memory is O(N + M) per thread.
#include <complex>

#include "device_common.hpp"

namespace jq {

namespace {

constexpr int kAuxChunk = 8;       // amplitudes per launch
constexpr int kAuxMaxVars = 40;
constexpr unsigned kAuxMaxBlocks = 4096;

using cplx = std::complex<double>;

struct AuxItem {
    int32_t kind;   // 0: 2x2 matrix, 1: factor of variable `index`
    int32_t index;  // matrix or variable number
};

// factor of a variable on one qubit: |0> times f[s], |1> times g[s] (s = 0
// for the variable value +1, 1 for -1)
struct AuxVar {
    double f[2][2];  // (re, im) of exp(i(+-x - a/4))
    double g[2][2];  // (re, im) of exp(-i(+-x - a/4))
};

struct AuxProgram {
    std::vector<std::vector<AuxItem>> items;  // per qubit
    std::vector<cplx> mats;                   // 4 entries per matrix, row-major
    std::vector<AuxVar> vars;
    cplx global{1.0, 0.0};
};

void add_matrix(AuxProgram& P, int q, const cplx m[4]) {
    auto& it = P.items[q];
    if (!it.empty() && it.back().kind == 0) {
        // fold into the previous matrix of this qubit: new = m * prev
        cplx* p = &P.mats[4 * it.back().index];
        const cplx r[4] = {m[0] * p[0] + m[1] * p[2], m[0] * p[1] + m[1] * p[3], m[2] * p[0] + m[3] * p[2],
                           m[2] * p[1] + m[3] * p[3]};
        for (int k = 0; k < 4; ++k) p[k] = r[k];
        return;
    }
    it.push_back({0, (int32_t)(P.mats.size() / 4)});
    for (int k = 0; k < 4; ++k) P.mats.push_back(m[k]);
}

void add_diag(AuxProgram& P, int q, cplx d0, cplx d1) {
    const cplx m[4] = {d0, 0.0, 0.0, d1};
    add_matrix(P, q, m);
}

// controlled phase with exp(ia) = e on qubits q0, q1 (Eqs. appa4-appa6)
void add_phase(AuxProgram& P, int q0, int q1, cplx e) {
    if ((int)P.vars.size() >= kAuxMaxVars) fail(JQ_EUNSUPPORTED, "jq_aux_amplitudes: more than 40 entangling gates");
    const cplx I(0.0, 1.0);
    const cplx a = -I * std::log(e);
    const cplx x = std::acos(std::exp(0.5 * I * a)) / 2.0;
    AuxVar v{};
    for (int s = 0; s < 2; ++s) {
        const cplx arg = (s == 0 ? x : -x) - a / 4.0;
        const cplx f = std::exp(I * arg), g = std::exp(-I * arg);
        v.f[s][0] = f.real();
        v.f[s][1] = f.imag();
        v.g[s][0] = g.real();
        v.g[s][1] = g.imag();
    }
    const int32_t p = (int32_t)P.vars.size();
    P.vars.push_back(v);
    P.items[q0].push_back({1, p});
    P.items[q1].push_back({1, p});
}

cplx c(const cd& z) { return cplx(z.re, z.im); }

int single_bit(uint64_t m) { return __builtin_ctzll(m); }

AuxProgram build(int n, const jq_gate* gates, size_t count) {
    AuxProgram P;
    P.items.resize(n);
    const cplx h = 1.0 / std::sqrt(2.0);
    const cplx H[4] = {h, h, h, -h};
    for (size_t i = 0; i < count; ++i) {
        if (gates[i].nq == 0) continue;  // identity
        GateOp op;
        try {
            op = canonicalize(gates[i], n);
        } catch (const Error& e) {
            fail(e.code, "gate " + std::to_string(i) + ": " + e.what());
        }
        const int nc = __builtin_popcountll(op.cmask);
        const std::string where = "gate " + std::to_string(i) + ": ";
        if (op.kind == OP_DENSE1) {
            if (nc) fail(JQ_EUNSUPPORTED, where + "controlled dense gates are not supported");
            const cplx m[4] = {c(op.m[0]), c(op.m[1]), c(op.m[2]), c(op.m[3])};
            add_matrix(P, op.t0, m);
        } else if (op.kind == OP_PERMX) {
            if (nc == 0) {
                const cplx X[4] = {0.0, 1.0, 1.0, 0.0};
                add_matrix(P, op.t0, X);
            } else if (nc == 1) {
                // CNOT = H_t U(pi) H_t
                add_matrix(P, op.t0, H);
                add_phase(P, single_bit(op.cmask), op.t0, cplx(-1.0, 0.0));
                add_matrix(P, op.t0, H);
            } else {
                fail(JQ_EUNSUPPORTED, where + "X with more than one control is not supported");
            }
        } else if (op.kind == OP_DIAG) {
            if (op.nsel == 0) {
                // multiply the subspace where every cmask bit is 1 by m[0]
                if (nc == 1) add_diag(P, single_bit(op.cmask), 1.0, c(op.m[0]));
                else if (nc == 2) {
                    const int q0 = single_bit(op.cmask), q1 = single_bit(op.cmask & (op.cmask - 1));
                    add_phase(P, q0, q1, c(op.m[0]));
                } else {
                    fail(JQ_EUNSUPPORTED, where + "phases on more than two qubits are not supported");
                }
            } else if (op.nsel == 1) {
                const cplx d0 = c(op.m[0]), d1 = c(op.m[1]);
                if (nc == 0) {
                    add_diag(P, op.t0, d0, d1);
                } else if (nc == 1) {
                    // diag(d0, d1) on t0 where the control is 1: diag(1, d0) on
                    // the control, then the phase d1/d0 on (control, t0)
                    if (d0 == 0.0) fail(JQ_EUNSUPPORTED, where + "zero diagonal entry");
                    const int cq = single_bit(op.cmask);
                    add_diag(P, cq, 1.0, d0);
                    add_phase(P, cq, op.t0, d1 / d0);
                } else {
                    fail(JQ_EUNSUPPORTED, where + "diagonal gates with several controls are not supported");
                }
            } else {
                if (nc) fail(JQ_EUNSUPPORTED, where + "controlled two-qubit diagonal gates are not supported");
                // diag(d00, d01, d10, d11), index 2 bit(t0) + bit(t1): d00 times
                // diag(1, d01/d00) on t1, diag(1, d10/d00) on t0 and the phase
                // d11 d00 / (d01 d10) on (t0, t1)
                const cplx d00 = c(op.m[0]), d01 = c(op.m[1]), d10 = c(op.m[2]), d11 = c(op.m[3]);
                if (d00 == 0.0 || d01 == 0.0 || d10 == 0.0) fail(JQ_EUNSUPPORTED, where + "zero diagonal entry");
                P.global *= d00;
                add_diag(P, op.t1, 1.0, d01 / d00);
                add_diag(P, op.t0, 1.0, d10 / d00);
                add_phase(P, op.t0, op.t1, d11 * d00 / (d01 * d10));
            }
        } else {
            fail(JQ_EUNSUPPORTED, where + "two-qubit dense gates are not supported");
        }
    }
    return P;
}

}  // namespace

// One thread per assignment c (bit p of c set: variable p is -1).  For the
// chunk's basis states b_k, acc_k = prod_j v_j[bit j of b_k].
__global__ __launch_bounds__(kBlock) void k_aux(int n, const AuxItem* __restrict__ items,
                                                 const int32_t* __restrict__ first, const double* __restrict__ mats,
                                                 const AuxVar* __restrict__ vars, uint64_t nconf,
                                                 const uint64_t* __restrict__ basis, int nb,
                                                 double* __restrict__ partial) {
    __shared__ double lds[kBlock / 64];
    double sr[kAuxChunk], si[kAuxChunk];
#pragma unroll
    for (int k = 0; k < kAuxChunk; ++k) sr[k] = si[k] = 0.0;
    for (uint64_t cf = (uint64_t)blockIdx.x * kBlock + threadIdx.x; cf < nconf; cf += (uint64_t)gridDim.x * kBlock) {
        double ar[kAuxChunk], ai[kAuxChunk];
#pragma unroll
        for (int k = 0; k < kAuxChunk; ++k) {
            ar[k] = 1.0;
            ai[k] = 0.0;
        }
        for (int j = 0; j < n; ++j) {
            double v0r = 1.0, v0i = 0.0, v1r = 0.0, v1i = 0.0;
            for (int t = first[j]; t < first[j + 1]; ++t) {
                const AuxItem it = items[t];
                if (it.kind == 0) {
                    const double* m = mats + 8 * it.index;
                    const double w0r = m[0] * v0r - m[1] * v0i + m[2] * v1r - m[3] * v1i;
                    const double w0i = m[0] * v0i + m[1] * v0r + m[2] * v1i + m[3] * v1r;
                    const double w1r = m[4] * v0r - m[5] * v0i + m[6] * v1r - m[7] * v1i;
                    const double w1i = m[4] * v0i + m[5] * v0r + m[6] * v1i + m[7] * v1r;
                    v0r = w0r;
                    v0i = w0i;
                    v1r = w1r;
                    v1i = w1i;
                } else {
                    const int s = (int)((cf >> it.index) & 1);
                    const AuxVar& V = vars[it.index];
                    const double fr = s ? V.f[1][0] : V.f[0][0], fi = s ? V.f[1][1] : V.f[0][1];
                    const double gr = s ? V.g[1][0] : V.g[0][0], gi = s ? V.g[1][1] : V.g[0][1];
                    const double t0r = v0r * fr - v0i * fi, t0i = v0r * fi + v0i * fr;
                    const double t1r = v1r * gr - v1i * gi, t1i = v1r * gi + v1i * gr;
                    v0r = t0r;
                    v0i = t0i;
                    v1r = t1r;
                    v1i = t1i;
                }
            }
#pragma unroll
            for (int k = 0; k < kAuxChunk; ++k) {
                if (k >= nb) break;
                const bool one = (basis[k] >> j) & 1;
                const double cr = one ? v1r : v0r, ci = one ? v1i : v0i;
                const double nr = ar[k] * cr - ai[k] * ci, ni = ar[k] * ci + ai[k] * cr;
                ar[k] = nr;
                ai[k] = ni;
            }
        }
#pragma unroll
        for (int k = 0; k < kAuxChunk; ++k) {
            sr[k] += ar[k];
            si[k] += ai[k];
        }
    }
    for (int k = 0; k < kAuxChunk; ++k) {
        const double r = block_sum(sr[k], lds);
        const double i = block_sum(si[k], lds);
        if (threadIdx.x == 0) {
            partial[(2 * k) * gridDim.x + blockIdx.x] = r;
            partial[(2 * k + 1) * gridDim.x + blockIdx.x] = i;
        }
    }
}

// out[k] = scale * sum over blocks of partial (in block order)
__global__ void k_aux_final(const double* __restrict__ partial, unsigned blocks, int nb, double scale_r,
                            double scale_i, double* __restrict__ out) {
    const int k = threadIdx.x;
    if (blockIdx.x != 0 || k >= nb) return;
    double r = 0.0, i = 0.0;
    for (unsigned b = 0; b < blocks; ++b) {
        r += partial[(2 * k) * blocks + b];
        i += partial[(2 * k + 1) * blocks + b];
    }
    out[2 * k] = scale_r * r - scale_i * i;
    out[2 * k + 1] = scale_r * i + scale_i * r;
}

}  // namespace jq

using namespace jq;

extern "C" {

int jq_aux_amplitudes(int n_qubits, const jq_gate* gates, size_t count, const uint64_t* basis, size_t m,
                      double* out) {
    void* dev = nullptr;
    try {
        set_last_error("");
        if (n_qubits < 1 || n_qubits > JQ_MAX_QUBITS) fail(JQ_EINVAL, "jq_aux_amplitudes: N must be in [1, 63]");
        if (count && !gates) fail(JQ_EINVAL, "jq_aux_amplitudes: null gates");
        if (m && (!basis || !out)) fail(JQ_EINVAL, "jq_aux_amplitudes: null array");
        for (size_t k = 0; k < m; ++k)
            if (n_qubits < 64 && (basis[k] >> n_qubits)) fail(JQ_EINVAL, "jq_aux_amplitudes: basis index out of range");
        AuxProgram P = build(n_qubits, gates, count);
        if (m == 0) return JQ_OK;
        // flatten
        std::vector<AuxItem> items;
        std::vector<int32_t> first(n_qubits + 1, 0);
        for (int j = 0; j < n_qubits; ++j) {
            first[j] = (int32_t)items.size();
            items.insert(items.end(), P.items[j].begin(), P.items[j].end());
        }
        first[n_qubits] = (int32_t)items.size();
        std::vector<double> mats(2 * P.mats.size() + 8);
        for (size_t k = 0; k < P.mats.size(); ++k) {
            mats[2 * k] = P.mats[k].real();
            mats[2 * k + 1] = P.mats[k].imag();
        }
        const int nv = (int)P.vars.size();
        const uint64_t nconf = 1ull << nv;
        unsigned blocks = (unsigned)std::min<uint64_t>((nconf + kBlock - 1) / kBlock, kAuxMaxBlocks);
        if (blocks == 0) blocks = 1;
        const size_t bytes_items = std::max<size_t>(items.size(), 1) * sizeof(AuxItem);
        const size_t bytes_first = first.size() * sizeof(int32_t);
        const size_t bytes_mats = mats.size() * sizeof(double);
        const size_t bytes_vars = std::max<size_t>(P.vars.size(), 1) * sizeof(AuxVar);
        const size_t bytes_basis = kAuxChunk * sizeof(uint64_t);
        const size_t bytes_part = 2 * kAuxChunk * (size_t)blocks * sizeof(double);
        const size_t bytes_out = 2 * kAuxChunk * sizeof(double);
        auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
        const size_t total = al(bytes_items) + al(bytes_first) + al(bytes_mats) + al(bytes_vars) + al(bytes_basis) +
                             al(bytes_part) + al(bytes_out);
        JQ_HIP(hipMalloc(&dev, total));
        char* p = (char*)dev;
        auto take = [&](size_t b) {
            char* r = p;
            p += al(b);
            return r;
        };
        AuxItem* d_items = (AuxItem*)take(bytes_items);
        int32_t* d_first = (int32_t*)take(bytes_first);
        double* d_mats = (double*)take(bytes_mats);
        AuxVar* d_vars = (AuxVar*)take(bytes_vars);
        uint64_t* d_basis = (uint64_t*)take(bytes_basis);
        double* d_part = (double*)take(bytes_part);
        double* d_out = (double*)take(bytes_out);
        if (!items.empty()) JQ_HIP(hipMemcpy(d_items, items.data(), items.size() * sizeof(AuxItem), hipMemcpyHostToDevice));
        JQ_HIP(hipMemcpy(d_first, first.data(), bytes_first, hipMemcpyHostToDevice));
        JQ_HIP(hipMemcpy(d_mats, mats.data(), bytes_mats, hipMemcpyHostToDevice));
        if (nv) JQ_HIP(hipMemcpy(d_vars, P.vars.data(), P.vars.size() * sizeof(AuxVar), hipMemcpyHostToDevice));
        const cplx scale = P.global / std::ldexp(1.0, nv);
        for (size_t k0 = 0; k0 < m; k0 += kAuxChunk) {
            const int nb = (int)std::min<size_t>(kAuxChunk, m - k0);
            JQ_HIP(hipMemcpy(d_basis, basis + k0, nb * sizeof(uint64_t), hipMemcpyHostToDevice));
            hipLaunchKernelGGL(k_aux, dim3(blocks), dim3(kBlock), 0, 0, n_qubits, d_items, d_first, d_mats, d_vars,
                               nconf, d_basis, nb, d_part);
            hipLaunchKernelGGL(k_aux_final, dim3(1), dim3(64), 0, 0, d_part, blocks, nb, scale.real(), scale.imag(),
                               d_out);
            JQ_HIP(hipGetLastError());
            JQ_HIP(hipMemcpy(out + 2 * k0, d_out, 2 * nb * sizeof(double), hipMemcpyDeviceToHost));
        }
        JQ_HIP(hipFree(dev));
        return JQ_OK;
    } catch (const Error& e) {
        if (dev) (void)hipFree(dev);
        set_last_error(e.what());
        return e.code;
    } catch (const std::exception& e) {
        if (dev) (void)hipFree(dev);
        set_last_error(e.what());
        return JQ_EDEVICE;
    }
}

}  // extern "C"

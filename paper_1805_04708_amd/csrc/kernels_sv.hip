// HIP kernels for complex128 / complex64 state vectors on gfx950.
//
// Per-gate kernels implement the in-place group updates of Sec. 2 (pairs
// for one target, Eq. NUM2; groups of four for two targets), restricted to
// the subspace where the controls are 1.  Each thread handles IT groups;
// consecutive threads take consecutive group indices, so with the target
// above the low index bits every load instruction of a wavefront reads
// contiguous 128-byte lines.  The fused kernel runs a whole pass of gates on
// a register/lane tile (see planner.cpp).  Reductions accumulate in FP64 in
// a fixed order (per-thread sums, a fixed tree per block, then the block
// partials in index order) so repeated calls give identical bits.
#include "device_common.hpp"

namespace jq {

// ------------------------------------------------------------ per gate --

template <typename R>
__global__ __launch_bounds__(kBlock) void k_dense1(typename Vec<R>::T* __restrict__ psi, uint64_t ngroups,
                                                    Ins ins, uint64_t tbit, M4<R> m) {
    const uint64_t g0 = (uint64_t)blockIdx.x * (kIt * kBlock) + threadIdx.x;
    uint64_t i0[kIt];
    Cx<R> a[kIt], b[kIt];
#pragma unroll
    for (int u = 0; u < kIt; ++u) {
        const uint64_t g = g0 + (uint64_t)u * kBlock;
        if (g < ngroups) {
            i0[u] = expand(g, ins);
            a[u] = ld<R>(psi, i0[u]);
            b[u] = ld<R>(psi, i0[u] | tbit);
        }
    }
#pragma unroll
    for (int u = 0; u < kIt; ++u) {
        const uint64_t g = g0 + (uint64_t)u * kBlock;
        if (g < ngroups) {
            st<R>(psi, i0[u], mac2(m.e[0], a[u], m.e[1], b[u]));
            st<R>(psi, i0[u] | tbit, mac2(m.e[2], a[u], m.e[3], b[u]));
        }
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_dense2(typename Vec<R>::T* __restrict__ psi, uint64_t ngroups,
                                                    Ins ins, uint64_t hbit, uint64_t lbit, M16<R> m) {
    const uint64_t g0 = (uint64_t)blockIdx.x * (2 * kBlock) + threadIdx.x;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const uint64_t g = g0 + (uint64_t)u * kBlock;
        if (g >= ngroups) continue;
        const uint64_t i = expand(g, ins);
        const uint64_t idx[4] = {i, i | lbit, i | hbit, i | hbit | lbit};
        Cx<R> x[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) x[c] = ld<R>(psi, idx[c]);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Cx<R> s = cmul(m.e[4 * r], x[0]);
#pragma unroll
            for (int c = 1; c < 4; ++c) s = cadd(s, cmul(m.e[4 * r + c], x[c]));
            st<R>(psi, idx[r], s);
        }
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_diag(typename Vec<R>::T* __restrict__ psi, uint64_t ngroups,
                                                  Ins ins, int nsel, int s0, int s1, M4<R> d) {
    const uint64_t g0 = (uint64_t)blockIdx.x * (kIt * kBlock) + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kIt; ++u) {
        const uint64_t g = g0 + (uint64_t)u * kBlock;
        if (g >= ngroups) continue;
        const uint64_t i = expand(g, ins);
        int sel = 0;
        if (nsel >= 1) sel = (int)((i >> s0) & 1);
        if (nsel == 2) sel = 2 * sel + (int)((i >> s1) & 1);
        Cx<R> f = d.e[0];
        f = csel(sel == 1, d.e[1], f);
        f = csel(sel == 2, d.e[2], f);
        f = csel(sel == 3, d.e[3], f);
        st<R>(psi, i, cmul(f, ld<R>(psi, i)));
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_permx(typename Vec<R>::T* __restrict__ psi, uint64_t ngroups,
                                                   Ins ins, uint64_t tbit) {
    const uint64_t g0 = (uint64_t)blockIdx.x * (kIt * kBlock) + threadIdx.x;
    uint64_t i0[kIt];
    typename Vec<R>::T a[kIt], b[kIt];
#pragma unroll
    for (int u = 0; u < kIt; ++u) {
        const uint64_t g = g0 + (uint64_t)u * kBlock;
        if (g < ngroups) {
            i0[u] = expand(g, ins);
            a[u] = psi[i0[u]];
            b[u] = psi[i0[u] | tbit];
        }
    }
#pragma unroll
    for (int u = 0; u < kIt; ++u) {
        const uint64_t g = g0 + (uint64_t)u * kBlock;
        if (g < ngroups) {
            psi[i0[u]] = b[u];
            psi[i0[u] | tbit] = a[u];
        }
    }
}

// ---------------------------------------------------------- fused pass --

// Keep the scheduler from interleaving the arithmetic of different register
// slots: interleaving buys latency the other waves already hide and costs a
// full set of temporaries per slot.
#define JQ_SLOT_FENCE() __builtin_amdgcn_sched_barrier(0)

template <typename R>
struct M2x2 {
    Cx<R> m0, m1, m2, m3;
};

template <typename R>
__device__ __forceinline__ M2x2<R> load_m(const FOp* op) {
    return {{(R)op->m[0], (R)op->m[1]}, {(R)op->m[2], (R)op->m[3]},
            {(R)op->m[4], (R)op->m[5]}, {(R)op->m[6], (R)op->m[7]}};
}

template <typename R>
__device__ __forceinline__ M2x2<R> load_m_v(const FOp* op, int v) {
    const double* m = op->m + 8 * v;
    return {{(R)m[0], (R)m[1]}, {(R)m[2], (R)m[3]}, {(R)m[4], (R)m[5]}, {(R)m[6], (R)m[7]}};
}

template <typename R>
__device__ __forceinline__ M2x2<R> msel(bool c, const M2x2<R>& x, const M2x2<R>& y) {
    return {csel(c, x.m0, y.m0), csel(c, x.m1, y.m1), csel(c, x.m2, y.m2), csel(c, x.m3, y.m3)};
}

// A multiplexed op's selectors are thread index bits (lane or outer bits;
// the planner never uses register slots for them): one matrix per thread.
template <typename R>
__device__ __forceinline__ M2x2<R> mux_thread(const FOp* op, uint64_t base) {
    const int g0 = (int)((base >> op->sel_glob[0]) & 1);
    if (op->nsel == 1) return msel(g0 == 1, load_m_v<R>(op, 1), load_m_v<R>(op, 0));
    const int v = 2 * g0 + (int)((base >> op->sel_glob[1]) & 1);
    M2x2<R> m = load_m_v<R>(op, 0);
    m = msel(v == 1, load_m_v<R>(op, 1), m);
    m = msel(v == 2, load_m_v<R>(op, 2), m);
    return msel(v == 3, load_m_v<R>(op, 3), m);
}

// Multiplexed 2x2 on register slot J: the matrix depends on 1-2 selector
// bits (a diagonal gate folded into this one).
template <typename R, int K, int J>
__device__ __forceinline__ void reg_mdense(Cx<R> (&a)[1 << K], const FOp* op, uint64_t base) {
    const M2x2<R> m = mux_thread<R>(op, base);
#pragma unroll
    for (int s = 0; s < (1 << K); ++s) {
        if (s & (1 << J)) continue;
        const Cx<R> x = a[s], y = a[s | (1 << J)];
        a[s] = mac2(m.m0, x, m.m1, y);
        a[s | (1 << J)] = mac2(m.m2, x, m.m3, y);
        JQ_SLOT_FENCE();
    }
}

// Dense 2x2 on register slot J.  CTRL: only where the thread's index bits
// and the slot's register bits satisfy the controls.
template <typename R, int K, int J, bool CTRL>
__device__ __forceinline__ void reg_dense(Cx<R> (&a)[1 << K], const FOp* op, bool thr_ok) {
    const M2x2<R> m = load_m<R>(op);
    const uint32_t rc = op->reg_ctrl;
#pragma unroll
    for (int s = 0; s < (1 << K); ++s) {
        if (s & (1 << J)) continue;
        const Cx<R> x = a[s], y = a[s | (1 << J)];
        const Cx<R> nx = mac2(m.m0, x, m.m1, y), ny = mac2(m.m2, x, m.m3, y);
        if constexpr (CTRL) {
            const bool ok = thr_ok && (((uint32_t)s & rc) == rc);
            a[s] = csel(ok, nx, x);
            a[s | (1 << J)] = csel(ok, ny, y);
        } else {
            a[s] = nx;
            a[s | (1 << J)] = ny;
        }
        JQ_SLOT_FENCE();
    }
}

template <typename R, int K, int J>
__device__ __forceinline__ void reg_perm(Cx<R> (&a)[1 << K], const FOp* op, bool thr_ok) {
    const uint32_t rc = op->reg_ctrl;
    if (!op->has_ctrl) {
#pragma unroll
        for (int s = 0; s < (1 << K); ++s) {
            if (s & (1 << J)) continue;
            const Cx<R> x = a[s];
            a[s] = a[s | (1 << J)];
            a[s | (1 << J)] = x;
        }
        return;
    }
#pragma unroll
    for (int s = 0; s < (1 << K); ++s) {
        if (s & (1 << J)) continue;
        const bool ok = thr_ok && (((uint32_t)s & rc) == rc);
        const Cx<R> x = a[s], y = a[s | (1 << J)];
        a[s] = csel(ok, y, x);
        a[s | (1 << J)] = csel(ok, x, y);
    }
}

// Exchange of a 32-bit value with lane ^ (1 << B): DPP quad permutations
// (VALU) for the two lowest lane bits, swizzles within 32 lanes (LDS pipe,
// no VALU issue) for bits 2-4, and a permute through the LDS crossbar for
// bit 5.
template <int B>
__device__ __forceinline__ int xor_lane(int v) {
    if constexpr (B == 0) {
        return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);  // quad_perm 1,0,3,2
    } else if constexpr (B == 1) {
        return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);  // quad_perm 2,3,0,1
    } else if constexpr (B == 2) {
        return __builtin_amdgcn_ds_swizzle(v, 0x101F);  // bitmask mode, xor 4
    } else if constexpr (B == 3) {
        return __builtin_amdgcn_ds_swizzle(v, 0x201F);  // bitmask mode, xor 8
    } else if constexpr (B == 4) {
        return __builtin_amdgcn_ds_swizzle(v, 0x401F);  // bitmask mode, xor 16
    } else {
        return __shfl_xor(v, 32, 64);
    }
}

template <int B>
__device__ __forceinline__ double xor_lane_d(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(xor_lane<B>(hi), xor_lane<B>(lo));
}
template <int B>
__device__ __forceinline__ float xor_lane_d(float v) {
    return __int_as_float(xor_lane<B>(__float_as_int(v)));
}

template <typename R, int B>
__device__ __forceinline__ Cx<R> xor_lane_c(Cx<R> v) {
    return {xor_lane_d<B>(v.re), xor_lane_d<B>(v.im)};
}

// Dense 2x2 (or X) on lane bit B: the partner amplitude lives in lane ^ 2^B,
// same register slot.  A lane with bit B = 0 computes row 0, one with bit
// B = 1 row 1 (m11 x + m10 y with x its own, y the partner's value).
template <typename R, int K, int B, int KIND>
__device__ __forceinline__ void lane_op_b(Cx<R> (&a)[1 << K], const FOp* op, int lane, bool thr_ok, uint64_t base) {
    const uint32_t rc = op->reg_ctrl;
    if constexpr (KIND == F_PERM_LANE) {
#pragma unroll
        for (int s = 0; s < (1 << K); ++s) {
            const Cx<R> y = xor_lane_c<R, B>(a[s]);
            const bool ok = thr_ok && (((uint32_t)s & rc) == rc);
            a[s] = csel(ok, y, a[s]);
            if ((s & 3) == 3) JQ_SLOT_FENCE();
        }
    } else if constexpr (KIND == F_MDENSE_LANE) {
        const bool hi = (lane >> B) & 1;
        const M2x2<R> m = mux_thread<R>(op, base);
        const Cx<R> cs = csel(hi, m.m3, m.m0), co = csel(hi, m.m2, m.m1);
#pragma unroll
        for (int s = 0; s < (1 << K); ++s) {
            const Cx<R> y = xor_lane_c<R, B>(a[s]);
            a[s] = mac2(cs, a[s], co, y);
            if ((s & 3) == 3) JQ_SLOT_FENCE();
        }
    } else {
        const M2x2<R> m = load_m<R>(op);
        const bool hi = (lane >> B) & 1;
        const Cx<R> cs = csel(hi, m.m3, m.m0), co = csel(hi, m.m2, m.m1);
#pragma unroll
        for (int s = 0; s < (1 << K); ++s) {
            const Cx<R> y = xor_lane_c<R, B>(a[s]);
            const Cx<R> nv = mac2(cs, a[s], co, y);
            if constexpr (KIND == F_CDENSE_LANE) {
                const bool ok = thr_ok && (((uint32_t)s & rc) == rc);
                a[s] = csel(ok, nv, a[s]);
            } else {
                a[s] = nv;
            }
            if ((s & 3) == 3) JQ_SLOT_FENCE();
        }
    }
}

// Multiply the controlled subset by d0 (F_PHASE) or negate it (F_NEG).  The
// thread's part of the control test is folded into a per-thread factor
// once; the register part is uniform per slot and becomes a branch.
template <typename R, int K, bool NEG>
__device__ __forceinline__ void phase_op(Cx<R> (&a)[1 << K], const FOp* op, bool thr_ok) {
    const uint32_t rc = op->reg_ctrl;
    if constexpr (NEG) {
        const R sg = thr_ok ? (R)-1 : (R)1;
        if (rc == 0) {
#pragma unroll
            for (int s = 0; s < (1 << K); ++s) {
                a[s].re *= sg;
                a[s].im *= sg;
            }
        } else {
#pragma unroll
            for (int s = 0; s < (1 << K); ++s) {
                const R f = (((uint32_t)s & rc) == rc) ? sg : (R)1;
                a[s].re *= f;
                a[s].im *= f;
            }
        }
    } else {
        const Cx<R> d{(R)op->m[0], (R)op->m[1]};
        const Cx<R> f = csel(thr_ok, d, Cx<R>{(R)1, (R)0});
        if (rc == 0) {
#pragma unroll
            for (int s = 0; s < (1 << K); ++s) {
                a[s] = cmulf(f, a[s]);
                JQ_SLOT_FENCE();
            }
        } else {
#pragma unroll
            for (int s = 0; s < (1 << K); ++s) {
                const Cx<R> fs = (((uint32_t)s & rc) == rc) ? f : Cx<R>{(R)1, (R)0};
                a[s] = cmulf(fs, a[s]);
                JQ_SLOT_FENCE();
            }
        }
    }
}

// General diagonal: factor d[sel], sel from one or two selector bits that
// are register slots (uniform per slot) or thread index bits.
template <typename R, int K>
__device__ __forceinline__ void diag_op(Cx<R> (&a)[1 << K], const FOp* op, uint64_t base, bool thr_ok) {
    Cx<R> d[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) d[i] = Cx<R>{(R)op->m[2 * i], (R)op->m[2 * i + 1]};
    const int nsel = op->nsel;
    const int r0 = op->sel_reg[0], r1 = op->sel_reg[1];
    const int g0 = op->sel_glob[0] >= 0 ? (int)((base >> op->sel_glob[0]) & 1) : 0;
    const int g1 = op->sel_glob[1] >= 0 ? (int)((base >> op->sel_glob[1]) & 1) : 0;
    const uint32_t rc = op->reg_ctrl;
    if (r0 < 0 && r1 < 0) {
        // every selector is a thread index bit: one factor per thread
        const int sel = nsel == 1 ? g0 : 2 * g0 + g1;
        Cx<R> f = d[0];
        f = csel(sel == 1, d[1], f);
        f = csel(sel == 2, d[2], f);
        f = csel(sel == 3, d[3], f);
        f = csel(thr_ok, f, Cx<R>{(R)1, (R)0});
        if (rc == 0) {
#pragma unroll
            for (int s = 0; s < (1 << K); ++s) {
                a[s] = cmulf(f, a[s]);
                JQ_SLOT_FENCE();
            }
            return;
        }
#pragma unroll
        for (int s = 0; s < (1 << K); ++s) {
            const Cx<R> fs = (((uint32_t)s & rc) == rc) ? f : Cx<R>{(R)1, (R)0};
            a[s] = cmulf(fs, a[s]);
            JQ_SLOT_FENCE();
        }
        return;
    }
#pragma unroll
    for (int s = 0; s < (1 << K); ++s) {
        const int b0 = r0 >= 0 ? ((s >> r0) & 1) : g0;
        const int b1 = r1 >= 0 ? ((s >> r1) & 1) : g1;
        const int sel = nsel == 1 ? b0 : 2 * b0 + b1;
        Cx<R> f = d[0];
        f = csel(sel == 1, d[1], f);
        f = csel(sel == 2, d[2], f);
        f = csel(sel == 3, d[3], f);
        const bool ok = thr_ok && (((uint32_t)s & rc) == rc);
        a[s] = csel(ok, cmulf(f, a[s]), a[s]);
        JQ_SLOT_FENCE();
    }
}

template <typename R, int K, int KIND>
__device__ __forceinline__ void reg_dispatch(Cx<R> (&a)[1 << K], const FOp* op, bool thr_ok, uint64_t base) {
    switch (op->slot) {
#define JQ_CASE(J)                                                                       \
    case J:                                                                              \
        if constexpr (J < K) {                                                           \
                                                            \
            if constexpr (KIND == F_DENSE_REG) reg_dense<R, K, J, false>(a, op, thr_ok); \
            else if constexpr (KIND == F_CDENSE_REG) reg_dense<R, K, J, true>(a, op, thr_ok); \
            else if constexpr (KIND == F_MDENSE_REG) reg_mdense<R, K, J>(a, op, base);   \
            else reg_perm<R, K, J>(a, op, thr_ok);                                       \
        }                                                                                \
        break;
        JQ_CASE(0)
        JQ_CASE(1)
        JQ_CASE(2)
        JQ_CASE(3)
        JQ_CASE(4)
        JQ_CASE(5)
#undef JQ_CASE
        default:
            break;
    }
}

template <typename R, int K, int KIND>
__device__ __forceinline__ void lane_dispatch(Cx<R> (&a)[1 << K], const FOp* op, int lane, bool thr_ok,
                                              uint64_t base = 0) {
    switch (op->slot) {
#define JQ_LCASE(B)                                             \
    case B:                                                     \
                                  \
        lane_op_b<R, K, B, KIND>(a, op, lane, thr_ok, base);    \
        break;
        JQ_LCASE(0)
        JQ_LCASE(1)
        JQ_LCASE(2)
        JQ_LCASE(3)
        JQ_LCASE(4)
        JQ_LCASE(5)
#undef JQ_LCASE
        default:
            break;
    }
}

#ifndef JQ_NT
#define JQ_NT 1
#endif

template <typename R>
struct NVec;
template <>
struct NVec<double> {
    typedef double T __attribute__((ext_vector_type(2)));
};
template <>
struct NVec<float> {
    typedef float T __attribute__((ext_vector_type(2)));
};

// Streaming access: each amplitude of the pass is read once and written
// once, so the loads and stores carry the non-temporal hint.
template <typename R>
__device__ __forceinline__ Cx<R> ld_stream(const typename Vec<R>::T* p, uint64_t i) {
#if JQ_NT
    const typename NVec<R>::T v = __builtin_nontemporal_load(reinterpret_cast<const typename NVec<R>::T*>(p) + i);
    return {v.x, v.y};
#else
    return ld<R>(p, i);
#endif
}

template <typename R>
__device__ __forceinline__ void st_stream(typename Vec<R>::T* p, uint64_t i, Cx<R> a) {
#if JQ_NT
    typename NVec<R>::T v;
    v.x = a.re;
    v.y = a.im;
    __builtin_nontemporal_store(v, reinterpret_cast<typename NVec<R>::T*>(p) + i);
#else
    st<R>(p, i, a);
#endif
}

template <typename R, int K>
__device__ __forceinline__ void run_ops(Cx<R> (&a)[1 << K], const FOp* __restrict__ ops, int n_ops, uint64_t base,
                                        int lane) {
    for (int k = 0; k < n_ops; ++k) {
        const FOp* op = ops + k;
        const bool thr_ok = (base & op->thr_ctrl) == op->thr_ctrl;
        switch (op->kind) {
            case F_DENSE_REG:
                reg_dispatch<R, K, F_DENSE_REG>(a, op, thr_ok, base);
                break;
            case F_CDENSE_REG:
                reg_dispatch<R, K, F_CDENSE_REG>(a, op, thr_ok, base);
                break;
            case F_PERM_REG:
                reg_dispatch<R, K, F_PERM_REG>(a, op, thr_ok, base);
                break;
            case F_DENSE_LANE:
                lane_dispatch<R, K, F_DENSE_LANE>(a, op, lane, thr_ok);
                break;
            case F_CDENSE_LANE:
                lane_dispatch<R, K, F_CDENSE_LANE>(a, op, lane, thr_ok);
                break;
            case F_PERM_LANE:
                lane_dispatch<R, K, F_PERM_LANE>(a, op, lane, thr_ok);
                break;
            case F_MDENSE_REG:
                reg_dispatch<R, K, F_MDENSE_REG>(a, op, thr_ok, base);
                break;
            case F_MDENSE_LANE:
                lane_dispatch<R, K, F_MDENSE_LANE>(a, op, lane, thr_ok, base);
                break;
            case F_PHASE:
                phase_op<R, K, false>(a, op, thr_ok);
                break;
            case F_NEG:
                phase_op<R, K, true>(a, op, thr_ok);
                break;
            case F_DIAG:
                diag_op<R, K>(a, op, base, thr_ok);
                break;
            default:
                break;
        }
    }
}

// Index of lane `lane`'s first amplitude in tile w: the tile number fills
// the index bits outside the tile, the lane number the lane bits.
__device__ __forceinline__ uint64_t tile_base(const FPass& P, uint64_t w, uint64_t lane_off) {
    uint64_t o = w;
    for (int i = 0; i < P.n_tile; ++i) {
        const int p = P.tile_sorted[i];
        o = ((o >> p) << (p + 1)) | (o & ((1ull << p) - 1));
    }
    return o | lane_off;
}

// One tile per wavefront.
template <typename R, int K, int F>
__global__ __launch_bounds__(kBlock) void k_fused(typename Vec<R>::T* __restrict__ psi, FPass P,
                                                   const FOp* __restrict__ ops) {
    constexpr int S = 1 << K;
    const int lane = threadIdx.x & 63;
    const uint64_t waves_per_block = blockDim.x >> 6;
    const uint64_t wave = (uint64_t)blockIdx.x * waves_per_block +
                          (uint64_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint64_t lane_off = (uint64_t)(lane & ((1 << F) - 1));
#pragma unroll
    for (int b = F; b < 6; ++b) lane_off |= (uint64_t)((lane >> b) & 1) << P.lane_q[b];
    uint64_t base = tile_base(P, wave, lane_off);
    uint64_t stride[K];
#pragma unroll
    for (int j = 0; j < K; ++j) stride[j] = 1ull << P.reg_q[j];
    Cx<R> a[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        uint64_t off = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (s & (1 << j)) off += stride[j];
        a[s] = ld_stream<R>(psi, base + off);
    }
    run_ops<R, K>(a, ops, P.n_ops, base, lane);
    // recompute the store addresses instead of keeping 2^K of them live
    asm volatile("" : "+v"(base));
#pragma unroll
    for (int s = 0; s < S; ++s) {
        uint64_t off = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (s & (1 << j)) off += stride[j];
        st_stream<R>(psi, base + off, a[s]);
    }
}

// ------------------------------------------------------- init / scale --

template <typename R>
__global__ __launch_bounds__(kBlock) void k_init(typename Vec<R>::T* __restrict__ psi, uint64_t dim, int mode,
                                                  uint64_t basis, double value) {
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < dim; i += (uint64_t)gridDim.x * kBlock) {
        typename Vec<R>::T v;
        v.x = (R)(mode == JQ_INIT_UNIFORM ? value : (i == basis ? 1.0 : 0.0));
        v.y = (R)0;
        psi[i] = v;
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_scale(typename Vec<R>::T* __restrict__ psi, uint64_t dim, double f) {
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < dim; i += (uint64_t)gridDim.x * kBlock) {
        typename Vec<R>::T v = psi[i];
        v.x = (R)((double)v.x * f);
        v.y = (R)((double)v.y * f);
        psi[i] = v;
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_to_c128(const typename Vec<R>::T* __restrict__ psi, uint64_t first,
                                                     uint64_t count, double2* __restrict__ dst) {
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (uint64_t)gridDim.x * kBlock) {
        typename Vec<R>::T v = psi[first + i];
        dst[i] = make_double2((double)v.x, (double)v.y);
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_from_c128(typename Vec<R>::T* __restrict__ psi, uint64_t first,
                                                       uint64_t count, const double2* __restrict__ src) {
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (uint64_t)gridDim.x * kBlock) {
        double2 v = src[i];
        typename Vec<R>::T w;
        w.x = (R)v.x;
        w.y = (R)v.y;
        psi[first + i] = w;
    }
}

// ---------------------------------------------------------- reductions --

// Loader for the reduction kernels: amplitudes as FP64.
template <typename R>
struct LoaderSV {
    const typename Vec<R>::T* psi;
    __device__ void prepare() {}
    __device__ __forceinline__ Cx<double> amp(uint64_t i) const {
        const Cx<R> v = ld<R>(psi, i);
        return {(double)v.re, (double)v.im};
    }
    __device__ __forceinline__ double modulus2(uint64_t i) const {
        const Cx<R> v = ld<R>(psi, i);
        const double re = v.re, im = v.im;
        return re * re + im * im;
    }
};

__global__ void k_sum_parts(const double* __restrict__ partial, uint64_t nbins, uint32_t parts,
                            double* __restrict__ out) {
    const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbins) return;
    double s = 0.0;
    for (uint32_t p = 0; p < parts; ++p) s += partial[b * parts + p];
    out[b] = s;
}

__global__ void k_expect_final(const double* __restrict__ partial, uint32_t parts, int q, int n,
                               double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s[4];
    for (int c = 0; c < 4; ++c) {
        double t = 0.0;
        for (uint32_t p = 0; p < parts; ++p) t += partial[(uint64_t)c * parts + p];
        s[c] = t;
    }
    out[q] = (1.0 - s[0] / s[3]) / 2.0;
    out[n + q] = (1.0 - s[1] / s[3]) / 2.0;
    out[2 * n + q] = (1.0 - s[2] / s[3]) / 2.0;
}

// ------------------------------------------------------------ launchers --

Ins make_ins(uint64_t zero_bits, uint64_t ones) {
    Ins s{};
    s.ones = ones;
    s.cnt = 0;
    for (int p = 0; p < 64; ++p)
        if (zero_bits & (1ull << p)) {
            if (s.cnt >= 7) fail(JQ_EINVAL, "too many fixed bits");
            s.pos[s.cnt++] = p;
        }
    return s;
}

unsigned blocks_for(uint64_t items, uint64_t per_block) {
    uint64_t b = (items + per_block - 1) / per_block;
    if (b == 0) b = 1;
    if (b > 0x7fffffffull) fail(JQ_EINVAL, "grid too large");
    return (unsigned)b;
}

unsigned grid_stride_blocks(uint64_t dim) {
    uint64_t b = (dim + kBlock - 1) / kBlock;
    return (unsigned)(b < 8192 ? (b ? b : 1) : 8192);
}

namespace {

template <typename R>
void apply_op_t(typename Vec<R>::T* psi, int n, const GateOp& op, hipStream_t st) {
    const int fixed = __builtin_popcountll(op.cmask);
    switch (op.kind) {
        case OP_DENSE1: {
            const uint64_t tb = 1ull << op.t0;
            const uint64_t ng = 1ull << (n - 1 - fixed);
            M4<R> m;
            for (int i = 0; i < 4; ++i) m.e[i] = {(R)op.m[i].re, (R)op.m[i].im};
            hipLaunchKernelGGL(k_dense1<R>, dim3(blocks_for(ng, kIt * kBlock)), dim3(kBlock), 0, st, psi, ng,
                               make_ins(op.cmask | tb, op.cmask), tb, m);
            break;
        }
        case OP_DENSE2: {
            const uint64_t hb = 1ull << op.t0, lb = 1ull << op.t1;
            const uint64_t ng = 1ull << (n - 2 - fixed);
            M16<R> m;
            for (int i = 0; i < 16; ++i) m.e[i] = {(R)op.m[i].re, (R)op.m[i].im};
            hipLaunchKernelGGL(k_dense2<R>, dim3(blocks_for(ng, 2 * kBlock)), dim3(kBlock), 0, st, psi, ng,
                               make_ins(op.cmask | hb | lb, op.cmask), hb, lb, m);
            break;
        }
        case OP_DIAG: {
            const uint64_t ng = 1ull << (n - fixed);
            M4<R> d;
            for (int i = 0; i < 4; ++i) d.e[i] = {(R)op.m[i].re, (R)op.m[i].im};
            hipLaunchKernelGGL(k_diag<R>, dim3(blocks_for(ng, kIt * kBlock)), dim3(kBlock), 0, st, psi, ng,
                               make_ins(op.cmask, op.cmask), op.nsel, op.t0 < 0 ? 0 : op.t0,
                               op.t1 < 0 ? 0 : op.t1, d);
            break;
        }
        case OP_PERMX: {
            const uint64_t tb = 1ull << op.t0;
            const uint64_t ng = 1ull << (n - 1 - fixed);
            hipLaunchKernelGGL(k_permx<R>, dim3(blocks_for(ng, kIt * kBlock)), dim3(kBlock), 0, st, psi, ng,
                               make_ins(op.cmask | tb, op.cmask), tb);
            break;
        }
        default:
            fail(JQ_EINVAL, "unknown op");
    }
    JQ_HIP(hipGetLastError());
}

template <typename R, int K, int F>
void launch_fused(typename Vec<R>::T* psi, int n, const FPass& p, hipStream_t st) {
    const uint64_t waves = 1ull << (n - 6 - K);
    const uint64_t wpb = waves < 4 ? waves : 4;
    hipLaunchKernelGGL((k_fused<R, K, F>), dim3(blocks_for(waves, wpb)), dim3(64 * wpb), 0, st, psi, p, p.ops);
    JQ_HIP(hipGetLastError());
}

template <typename R, int F>
void fused_dispatch(typename Vec<R>::T* psi, int n, const FPass& p, int k, hipStream_t st) {
    if (n < 6 + k) fail(JQ_EINVAL, "fused pass: tile larger than the state");
    switch (k) {
        case 2: launch_fused<R, 2, F>(psi, n, p, st); break;
        case 3: launch_fused<R, 3, F>(psi, n, p, st); break;
        case 4: launch_fused<R, 4, F>(psi, n, p, st); break;
        case 5: launch_fused<R, 5, F>(psi, n, p, st); break;
        case 6:
            if constexpr (sizeof(R) == 4) { launch_fused<R, 6, F>(psi, n, p, st); break; }
            [[fallthrough]];
        default:
            fail(JQ_EINVAL, "fused pass: unsupported register width " + std::to_string(k));
    }
}

}  // namespace

size_t probabilities_partial_count(int n, int nq) {
    (void)n;
    return (size_t)(4096 + (1ull << nq)) + 8192;
}

void sv_init(int enc, void* psi, int n, int mode, uint64_t basis, hipStream_t st) {
    const uint64_t dim = 1ull << n;
    const double v = uniform_amplitude(n);
    if (enc == JQ_C128)
        hipLaunchKernelGGL(k_init<double>, dim3(grid_stride_blocks(dim)), dim3(kBlock), 0, st, (double2*)psi, dim,
                           mode, basis, v);
    else
        hipLaunchKernelGGL(k_init<float>, dim3(grid_stride_blocks(dim)), dim3(kBlock), 0, st, (float2*)psi, dim, mode,
                           basis, v);
    JQ_HIP(hipGetLastError());
}

void sv_apply_op(int enc, void* psi, int n, const GateOp& op, hipStream_t st) {
    if (enc == JQ_C128) apply_op_t<double>((double2*)psi, n, op, st);
    else apply_op_t<float>((float2*)psi, n, op, st);
}

void sv_apply_fused(int enc, void* psi, int n, const FPass& pass, int k_reg, int fixed_lane_bits, hipStream_t st) {
    if (enc == JQ_C128) {
        if (fixed_lane_bits != 3) fail(JQ_EINVAL, "c128 fused pass expects 3 fixed lane bits");
        fused_dispatch<double, 3>((double2*)psi, n, pass, k_reg, st);
    } else {
        if (fixed_lane_bits != 4) fail(JQ_EINVAL, "c64 fused pass expects 4 fixed lane bits");
        fused_dispatch<float, 4>((float2*)psi, n, pass, k_reg, st);
    }
}

void sv_probabilities(int enc, const void* psi, int n, const int* qubits, int nq, double* out, double* partial,
                      size_t cap, hipStream_t st) {
    if (enc == JQ_C128) launch_probs(LoaderSV<double>{(const double2*)psi}, n, qubits, nq, out, partial, cap, st);
    else launch_probs(LoaderSV<float>{(const float2*)psi}, n, qubits, nq, out, partial, cap, st);
}

void sv_expectations(int enc, const void* psi, int n, double* out, double* partial, size_t cap, hipStream_t st) {
    if (enc == JQ_C128) launch_expect(LoaderSV<double>{(const double2*)psi}, n, out, partial, cap, st);
    else launch_expect(LoaderSV<float>{(const float2*)psi}, n, out, partial, cap, st);
}

void sv_scale(int enc, void* psi, int n, double f, hipStream_t st) {
    const uint64_t dim = 1ull << n;
    if (enc == JQ_C128)
        hipLaunchKernelGGL(k_scale<double>, dim3(grid_stride_blocks(dim)), dim3(kBlock), 0, st, (double2*)psi, dim, f);
    else
        hipLaunchKernelGGL(k_scale<float>, dim3(grid_stride_blocks(dim)), dim3(kBlock), 0, st, (float2*)psi, dim, f);
    JQ_HIP(hipGetLastError());
}

void sv_to_c128(int enc, const void* psi, uint64_t first, uint64_t count, double* dst, hipStream_t st) {
    if (enc == JQ_C128)
        hipLaunchKernelGGL(k_to_c128<double>, dim3(grid_stride_blocks(count)), dim3(kBlock), 0, st,
                           (const double2*)psi, first, count, (double2*)dst);
    else
        hipLaunchKernelGGL(k_to_c128<float>, dim3(grid_stride_blocks(count)), dim3(kBlock), 0, st,
                           (const float2*)psi, first, count, (double2*)dst);
    JQ_HIP(hipGetLastError());
}

void sv_from_c128(int enc, void* psi, uint64_t first, uint64_t count, const double* src, hipStream_t st) {
    if (enc == JQ_C128)
        hipLaunchKernelGGL(k_from_c128<double>, dim3(grid_stride_blocks(count)), dim3(kBlock), 0, st, (double2*)psi,
                           first, count, (const double2*)src);
    else
        hipLaunchKernelGGL(k_from_c128<float>, dim3(grid_stride_blocks(count)), dim3(kBlock), 0, st, (float2*)psi,
                           first, count, (const double2*)src);
    JQ_HIP(hipGetLastError());
}

}  // namespace jq

// Register/lane tile operations of the fused pass, shared by the
// state-vector kernels and the two-byte-code kernels.  A wavefront holds
// 2^K amplitudes per lane; ops act on register slots (in-thread) or lane
// bits (cross-lane exchange), see planner.cpp.
#pragma once

#include "device_common.hpp"

namespace jq {

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

// Matrix v read per lane (v may differ between lanes): four 16-byte vector
// loads from the op record (FOp::m is 16-byte aligned, see internal.hpp).
template <typename R>
__device__ __forceinline__ M2x2<R> load_m_lane(const FOp* op, int v) {
    const double2* m = reinterpret_cast<const double2*>(op->m) + 4 * v;
    const double2 e0 = m[0], e1 = m[1], e2 = m[2], e3 = m[3];
    return {{(R)e0.x, (R)e0.y}, {(R)e1.x, (R)e1.y}, {(R)e2.x, (R)e2.y}, {(R)e3.x, (R)e3.y}};
}

template <typename R>
__device__ __forceinline__ M2x2<R> msel(bool c, const M2x2<R>& x, const M2x2<R>& y) {
    return {csel(c, x.m0, y.m0), csel(c, x.m1, y.m1), csel(c, x.m2, y.m2), csel(c, x.m3, y.m3)};
}

// A multiplexed op's selectors are thread index bits (lane or outer bits;
// the planner never uses register slots for them): one matrix per thread.
// An outer bit is the same in every lane of the wave (read from the tile
// base ubase), so its part of the choice is made once for the wave, with
// the matrix read by scalar loads; only lane-bit selectors choose per lane.
// One lane selector chooses between two scalar-loaded matrices in
// registers.  With two, the matrix is loaded per lane instead: a chain of
// three selects held two candidate sets live at once and set the fused
// kernel's peak register count (98 instead of 94 VGPRs for complex128 with
// the op set of kLiteKinds).
template <typename R>
__device__ __forceinline__ M2x2<R> mux_thread(const FOp* op, uint64_t base, uint64_t ubase) {
    const int lm = op->sel_lane;
    const int s0 = op->sel_glob[0];
    if (op->nsel == 1) {
        if (!(lm & 1)) return load_m_v<R>(op, (int)((ubase >> s0) & 1));
        return msel(((base >> s0) & 1) != 0, load_m_v<R>(op, 1), load_m_v<R>(op, 0));
    }
    const int s1 = op->sel_glob[1];
    if (!(lm & 3)) return load_m_v<R>(op, 2 * (int)((ubase >> s0) & 1) + (int)((ubase >> s1) & 1));
    if (!(lm & 1)) {
        const int v0 = 2 * (int)((ubase >> s0) & 1);
        return msel(((base >> s1) & 1) != 0, load_m_v<R>(op, v0 + 1), load_m_v<R>(op, v0));
    }
    if (!(lm & 2)) {
        const int v1 = (int)((ubase >> s1) & 1);
        return msel(((base >> s0) & 1) != 0, load_m_v<R>(op, 2 + v1), load_m_v<R>(op, v1));
    }
    return load_m_lane<R>(op, 2 * (int)((base >> s0) & 1) + (int)((base >> s1) & 1));
}

// Multiplexed 2x2 on register slot J: the matrix depends on 1-2 selector
// bits (a diagonal gate folded into this one).
template <typename R, int K, int J>
__device__ __forceinline__ void reg_mdense(Cx<R> (&a)[1 << K], const FOp* op, uint64_t base, uint64_t ubase) {
    const M2x2<R> m = mux_thread<R>(op, base, ubase);
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
__device__ __forceinline__ void lane_op_b(Cx<R> (&a)[1 << K], const FOp* op, int lane, bool thr_ok, uint64_t base,
                                          uint64_t ubase) {
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
        const M2x2<R> m = mux_thread<R>(op, base, ubase);
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

// x with its sign bit XORed with bit 31 of f (f is 0 or 0x80000000):
// -x bit for bit when f is set, x otherwise
__device__ __forceinline__ double flip_sign(double x, uint32_t f) {
    const uint64_t b = (uint64_t)__builtin_bit_cast(uint64_t, x) ^ ((uint64_t)f << 32);
    return __builtin_bit_cast(double, b);
}
__device__ __forceinline__ float flip_sign(float x, uint32_t f) {
    return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, x) ^ f);
}

// Multiply the controlled subset by d0 (F_PHASE) or negate it (F_NEG).  The
// thread's part of the control test is folded into a per-thread factor
// once; the register part is uniform per slot and becomes a branch.
template <typename R, int K, bool NEG>
__device__ __forceinline__ void phase_op(Cx<R> (&a)[1 << K], const FOp* op, bool thr_ok) {
    const uint32_t rc = op->reg_ctrl;
    if constexpr (NEG) {
        // negation flips the sign bit, the same bits as a product with -1
        // (signed zeros and NaNs included), with no factor per slot held
        // in registers
        const uint32_t sgn = thr_ok ? 0x80000000u : 0u;
#pragma unroll
        for (int s = 0; s < (1 << K); ++s) {
            const uint32_t f = (((uint32_t)s & rc) == rc) ? sgn : 0u;
            a[s].re = flip_sign(a[s].re, f);
            a[s].im = flip_sign(a[s].im, f);
            if ((s & 3) == 3) JQ_SLOT_FENCE();
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
__device__ __forceinline__ void diag_op(Cx<R> (&a)[1 << K], const FOp* op, uint64_t base, uint64_t ubase,
                                        bool thr_ok) {
    Cx<R> d[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) d[i] = Cx<R>{(R)op->m[2 * i], (R)op->m[2 * i + 1]};
    const int nsel = op->nsel;
    const int r0 = op->sel_reg[0], r1 = op->sel_reg[1];
    // a selector bit outside the lanes is the same in every lane: read it
    // from the wave-uniform tile base
    const int lm = op->sel_lane;
    const int g0 = op->sel_glob[0] >= 0 ? (int)(((lm & 1 ? base : ubase) >> op->sel_glob[0]) & 1) : 0;
    const int g1 = op->sel_glob[1] >= 0 ? (int)(((lm & 2 ? base : ubase) >> op->sel_glob[1]) & 1) : 0;
    const uint32_t rc = op->reg_ctrl;
    if (r0 < 0 && r1 < 0) {
        // every selector is a thread index bit: one factor per thread
        Cx<R> f;
        if (!(lm & 3)) {
            // no lane selector: the factor is the same in every lane
            const int sel = nsel == 1 ? g0 : 2 * g0 + g1;
            f = Cx<R>{(R)op->m[2 * sel], (R)op->m[2 * sel + 1]};
        } else {
            const int sel = nsel == 1 ? g0 : 2 * g0 + g1;
            f = d[0];
            f = csel(sel == 1, d[1], f);
            f = csel(sel == 2, d[2], f);
            f = csel(sel == 3, d[3], f);
        }
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
    if (!op->has_ctrl && !(lm & 3)) {
        // no controls and no lane selector: every factor is chosen per slot,
        // the same in every lane (an RZ on a register qubit, say)
#pragma unroll
        for (int s = 0; s < (1 << K); ++s) {
            const int b0 = r0 >= 0 ? ((s >> r0) & 1) : g0;
            const int b1 = r1 >= 0 ? ((s >> r1) & 1) : g1;
            const int sel = nsel == 1 ? b0 : 2 * b0 + b1;
            Cx<R> f = d[0];
            f = csel(sel == 1, d[1], f);
            f = csel(sel == 2, d[2], f);
            f = csel(sel == 3, d[3], f);
            a[s] = cmulf(f, a[s]);
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

// A group of uncontrolled one-qubit diagonals: one factor per thread, the
// product of the lane components (chosen per lane) and of the components
// on index bits outside the tile (the same in every lane, from the tile
// base, formed in FP64 once per wave); the register components come as a
// table of their product per slot, in the kernel's precision (slot holds
// the table's tag; the launcher has checked that it is R's).
template <typename R, int K>
__device__ __forceinline__ void dgroup_op(Cx<R> (&a)[1 << K], const FOp* op, int lane, uint64_t ubase) {
    const int n = op->n_od;
    Cx<double> w{1.0, 0.0};
    for (int c = 0; c < n; ++c) {
        if (op->od_where[c] != 2) continue;
        const int b = (int)((ubase >> op->od_idx[c]) & 1);
        w = cmul(w, Cx<double>{op->od_m[4 * c + 2 * b], op->od_m[4 * c + 2 * b + 1]});
    }
    Cx<R> t{(R)w.re, (R)w.im};
    for (int c = 0; c < n; ++c) {
        if (op->od_where[c] != 1) continue;
        const bool b = (lane >> op->od_idx[c]) & 1;
        const Cx<R> d0{(R)op->od_m[4 * c], (R)op->od_m[4 * c + 1]};
        const Cx<R> d1{(R)op->od_m[4 * c + 2], (R)op->od_m[4 * c + 3]};
        t = cmul(t, csel(b, d1, d0));
    }
    if constexpr ((1 << K) <= (sizeof(R) == 4 ? kDgSlotsF32 : kDgSlotsF64)) {
        if (op->slot == dg_table_tag<R>()) {
            // register components: the planner's product per slot, float
            // pairs for complex64, double pairs otherwise
            const R* tab = reinterpret_cast<const R*>(op->m);
#pragma unroll
            for (int s = 0; s < (1 << K); ++s) {
                const Cx<R> fs = cmul(t, Cx<R>{tab[2 * s], tab[2 * s + 1]});
                a[s] = cmulf(fs, a[s]);
                JQ_SLOT_FENCE();
            }
            return;
        }
    }
#pragma unroll
    for (int s = 0; s < (1 << K); ++s) {
        a[s] = cmulf(t, a[s]);
        JQ_SLOT_FENCE();
    }
}

template <typename R, int K, int KIND>
__device__ __forceinline__ void reg_dispatch(Cx<R> (&a)[1 << K], const FOp* op, bool thr_ok, uint64_t base,
                                             uint64_t ubase) {
    switch (op->slot) {
#define JQ_CASE(J)                                                                       \
    case J:                                                                              \
        if constexpr (J < K) {                                                           \
                                                            \
            if constexpr (KIND == F_DENSE_REG) reg_dense<R, K, J, false>(a, op, thr_ok); \
            else if constexpr (KIND == F_CDENSE_REG) reg_dense<R, K, J, true>(a, op, thr_ok); \
            else if constexpr (KIND == F_MDENSE_REG) reg_mdense<R, K, J>(a, op, base, ubase); \
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
                                              uint64_t base = 0, uint64_t ubase = 0) {
    switch (op->slot) {
#define JQ_LCASE(B)                                             \
    case B:                                                     \
                                  \
        lane_op_b<R, K, B, KIND>(a, op, lane, thr_ok, base, ubase); \
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

// base: index of the lane's first amplitude; ubase: the tile's base, the
// same in every lane (base without the lane bits)
// Op kinds of the reduced op loop (LITE): dense and multiplexed 2x2s on
// register slots and lane bits, and negations; what layers of one-qubit
// gates with CZs between them lower to.  A kernel compiled with every kind
// needs as many registers as its hungriest kind plus what the others keep
// live across the loop (121 VGPRs for complex128 with 2^4 register slots,
// 4 waves per SIMD); one compiled with these alone needs 94 (5 waves).
constexpr uint32_t kLiteKinds = (1u << F_DENSE_REG) | (1u << F_DENSE_LANE) | (1u << F_MDENSE_REG) |
                                (1u << F_MDENSE_LANE) | (1u << F_NEG);

// LITE: the op list holds only kinds of kLiteKinds (others are skipped).
template <typename R, int K, bool LITE = false>
__device__ __forceinline__ void run_ops(Cx<R> (&a)[1 << K], const FOp* __restrict__ ops, int n_ops, uint64_t base,
                                        uint64_t ubase, int lane) {
    for (int k = 0; k < n_ops; ++k) {
        const FOp* op = ops + k;
        const bool thr_ok = (base & op->thr_ctrl) == op->thr_ctrl;
        switch (op->kind) {
            case F_DENSE_REG:
                reg_dispatch<R, K, F_DENSE_REG>(a, op, thr_ok, base, ubase);
                break;
            case F_CDENSE_REG:
                if constexpr (!LITE) reg_dispatch<R, K, F_CDENSE_REG>(a, op, thr_ok, base, ubase);
                break;
            case F_PERM_REG:
                if constexpr (!LITE) reg_dispatch<R, K, F_PERM_REG>(a, op, thr_ok, base, ubase);
                break;
            case F_DENSE_LANE:
                lane_dispatch<R, K, F_DENSE_LANE>(a, op, lane, thr_ok);
                break;
            case F_CDENSE_LANE:
                if constexpr (!LITE) lane_dispatch<R, K, F_CDENSE_LANE>(a, op, lane, thr_ok);
                break;
            case F_PERM_LANE:
                if constexpr (!LITE) lane_dispatch<R, K, F_PERM_LANE>(a, op, lane, thr_ok);
                break;
            case F_MDENSE_REG:
                reg_dispatch<R, K, F_MDENSE_REG>(a, op, thr_ok, base, ubase);
                break;
            case F_MDENSE_LANE:
                lane_dispatch<R, K, F_MDENSE_LANE>(a, op, lane, thr_ok, base, ubase);
                break;
            case F_PHASE:
                if constexpr (!LITE) phase_op<R, K, false>(a, op, thr_ok);
                break;
            case F_NEG:
                phase_op<R, K, true>(a, op, thr_ok);
                break;
            case F_DIAG:
                if constexpr (!LITE) diag_op<R, K>(a, op, base, ubase, thr_ok);
                break;
            case F_DGROUP:
                if constexpr (!LITE) dgroup_op<R, K>(a, op, lane, ubase);
                break;
            default:
                break;
        }
    }
}

// A 64-bit value that is the same in every lane, held in scalar registers
// (readfirstlane returns int: each half goes through uint32_t).
__device__ __forceinline__ uint64_t wave_uniform(uint64_t x) {
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32)) << 32) |
           (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
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


}  // namespace jq

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
#include "fused_ops.hpp"

namespace jq {

// ------------------------------------------------------------ per gate --
//
// Blocks take chunks of IT * 256 groups (two-qubit: 2 * 256) and loop over
// chunks when the grid is capped (a launch holds at most 2^32 threads).
// Each amplitude is read and written once, so the accesses carry the
// non-temporal hint, except where controls leave parts of each line
// untouched.  IT is chosen per gate by the caller (measured at N=30
// complex128: one pair per thread streams fastest for targets below 17,
// four pairs above).
template <typename R, bool NT>
__device__ __forceinline__ Cx<R> ld_pg(const typename Vec<R>::T* p, uint64_t i) {
    if constexpr (NT) return ld_stream<R>(p, i);
    else return ld<R>(p, i);
}
template <typename R, bool NT>
__device__ __forceinline__ void st_pg(typename Vec<R>::T* p, uint64_t i, Cx<R> a) {
    if constexpr (NT) st_stream<R>(p, i, a);
    else st<R>(p, i, a);
}

// Chunk order: with ilv = 0 chunk c covers groups [c IT 256, (c+1) IT 256);
// with ilv = nchunks / 64 the chunks are dealt out in 64 interleaved
// streams (chunk c takes slot (c mod 64) ilv + c / 64), so that the
// requests in flight spread over the memory channels when a fixed control
// bit sits on an address bit that selects them (measured: CZ(t, t+1) at
// N=30 complex128 streams at 4.0-5.5 TB/s in order and 6.0-6.3 TB/s
// interleaved for t = 5, 6, 7, 15, 16, i.e. byte-address bits 10, 11 and
// 20; for other t the order is as fast or faster).
__device__ __forceinline__ uint64_t chunk_slot(uint64_t c, uint64_t ilv) {
    return ilv ? (c & 63) * ilv + (c >> 6) : c;
}

template <typename R, int IT, bool NT>
__global__ __launch_bounds__(kBlock) void k_dense1(typename Vec<R>::T* __restrict__ psi, uint64_t ngroups,
                                                    Ins ins, uint64_t tbit, M4<R> m, uint64_t ilv) {
    for (uint64_t chunk = blockIdx.x; chunk * (IT * kBlock) < ngroups; chunk += gridDim.x) {
        const uint64_t g0 = chunk_slot(chunk, ilv) * (IT * kBlock) + threadIdx.x;
        uint64_t i0[IT];
        Cx<R> a[IT], b[IT];
#pragma unroll
        for (int u = 0; u < IT; ++u) {
            const uint64_t g = g0 + (uint64_t)u * kBlock;
            if (g < ngroups) {
                i0[u] = expand(g, ins);
                a[u] = ld_pg<R, NT>(psi, i0[u]);
                b[u] = ld_pg<R, NT>(psi, i0[u] | tbit);
            }
        }
#pragma unroll
        for (int u = 0; u < IT; ++u) {
            const uint64_t g = g0 + (uint64_t)u * kBlock;
            if (g < ngroups) {
                st_pg<R, NT>(psi, i0[u], mac2(m.e[0], a[u], m.e[1], b[u]));
                st_pg<R, NT>(psi, i0[u] | tbit, mac2(m.e[2], a[u], m.e[3], b[u]));
            }
        }
    }
}

// An uncontrolled 2x2 or X on a target B below 3 (Eq. NUM2 with the pair
// inside one 128-byte line): consecutive threads take consecutive
// amplitudes, so every load and store instruction covers whole lines, and a
// lane gets its partner's value from lane ^ 2^B (DPP for B = 0, 1, a
// swizzle for B = 2).  A lane with bit B = 0 computes row 0 of the matrix,
// one with bit B = 1 row 1 (X: the partner's value).  Needs whole chunks of
// 256 amplitudes (2^N >= 256), so that every lane of a wave is active.
// Measured at N=30 complex128: 5.87-5.88 TB/s on targets 0-2, against
// 5.44-5.57 for the pair kernel, whose loads use half of every line.
template <typename R, int B, bool PERM>
__global__ __launch_bounds__(kBlock) void k_pair_lane(typename Vec<R>::T* __restrict__ psi, uint64_t dim, M4<R> m) {
    const int lane = threadIdx.x & 63;
    const bool hi = (lane >> B) & 1;
    const Cx<R> cs = csel(hi, m.e[3], m.e[0]), co = csel(hi, m.e[2], m.e[1]);
    for (uint64_t chunk = blockIdx.x; chunk * kBlock < dim; chunk += gridDim.x) {
        const uint64_t i = chunk * kBlock + threadIdx.x;
        const Cx<R> a = ld_stream<R>(psi, i);
        const Cx<R> y = xor_lane_c<R, B>(a);
        if constexpr (PERM) st_stream<R>(psi, i, y);
        else st_stream<R>(psi, i, mac2(cs, a, co, y));
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_dense2(typename Vec<R>::T* __restrict__ psi, uint64_t ngroups,
                                                    Ins ins, uint64_t hbit, uint64_t lbit, M16<R> m) {
    for (uint64_t chunk = blockIdx.x; chunk * (2 * kBlock) < ngroups; chunk += gridDim.x) {
        const uint64_t g0 = chunk * (2 * kBlock) + threadIdx.x;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const uint64_t g = g0 + (uint64_t)u * kBlock;
            if (g >= ngroups) continue;
            const uint64_t i = expand(g, ins);
            const uint64_t idx[4] = {i, i | lbit, i | hbit, i | hbit | lbit};
            Cx<R> x[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) x[c] = ld_stream<R>(psi, idx[c]);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                Cx<R> s = cmul(m.e[4 * r], x[0]);
#pragma unroll
                for (int c = 1; c < 4; ++c) s = cadd(s, cmul(m.e[4 * r + c], x[c]));
                st_stream<R>(psi, idx[r], s);
            }
        }
    }
}

// Uncontrolled two-qubit gate whose lower qubit LO lies inside a 128-byte
// line (below 3 for complex128, below 4 for complex64).  A thread
// holds the amplitudes i and i + 2^hi (hi the other qubit, i with bit hi
// clear; consecutive threads take consecutive i) and takes the two partners
// across bit LO from lane ^ 2^LO (DPP or swizzle), so every load and store
// covers whole lines.  LO_LSB: LO is the gate's second qubit (the least
// significant bit of the matrix index; the first listed is the most).  The
// coefficients of the lane's two rows are chosen once.  Needs whole chunks
// of 256 pairs (2^N >= 512), so that every lane of a wave is active.
// Measured at N=30 complex128: qubits (0, 1) 5.4 TB/s and (2, 5) 6.1 TB/s,
// against 1.5 and 4.0 TB/s for the four-amplitude kernel, whose loads use a
// quarter or half of each line per instruction.
template <typename R, int LO, bool LO_LSB>
__global__ __launch_bounds__(kBlock) void k_quad_lane(typename Vec<R>::T* __restrict__ psi, uint64_t npairs, int hi,
                                                       M16<R> m) {
    const int lane = threadIdx.x & 63;
    const bool l = (lane >> LO) & 1;
    // matrix index of (bit hi, bit LO)
    auto idx = [](int h, int v) { return LO_LSB ? 2 * h + v : 2 * v + h; };
    // row idx(h, l): coefficients of x_h (own, bit LO = l) and of y_h (from
    // the partner lane, bit LO = !l), chosen by the lane's bit LO
    Cx<R> cx[2][2], cy[2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int hc = 0; hc < 2; ++hc) {
            cx[h][hc] = csel(l, m.e[4 * idx(h, 1) + idx(hc, 1)], m.e[4 * idx(h, 0) + idx(hc, 0)]);
            cy[h][hc] = csel(l, m.e[4 * idx(h, 1) + idx(hc, 0)], m.e[4 * idx(h, 0) + idx(hc, 1)]);
        }
    const uint64_t low = (1ull << hi) - 1;
    for (uint64_t chunk = blockIdx.x; chunk * kBlock < npairs; chunk += gridDim.x) {
        const uint64_t g = chunk * kBlock + threadIdx.x;
        const uint64_t i = ((g & ~low) << 1) | (g & low), j = i | (low + 1);
        const Cx<R> x0 = ld_stream<R>(psi, i), x1 = ld_stream<R>(psi, j);
        const Cx<R> y0 = xor_lane_c<R, LO>(x0), y1 = xor_lane_c<R, LO>(x1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            Cx<R> acc = cmul(cx[h][0], x0);
            acc = cadd(acc, cmul(cx[h][1], x1));
            acc = cadd(acc, cmul(cy[h][0], y0));
            acc = cadd(acc, cmul(cy[h][1], y1));
            st_stream<R>(psi, h ? j : i, acc);
        }
    }
}

template <typename R, int IT, bool NT>
__global__ __launch_bounds__(kBlock) void k_diag(typename Vec<R>::T* __restrict__ psi, uint64_t ngroups,
                                                  Ins ins, int nsel, int s0, int s1, M4<R> d, uint64_t ilv) {
    for (uint64_t chunk = blockIdx.x; chunk * (IT * kBlock) < ngroups; chunk += gridDim.x) {
        const uint64_t g0 = chunk_slot(chunk, ilv) * (IT * kBlock) + threadIdx.x;
#pragma unroll
        for (int u = 0; u < IT; ++u) {
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
            st_pg<R, NT>(psi, i, cmul(f, ld_pg<R, NT>(psi, i)));
        }
    }
}

// A diagonal whose controls fix index bits inside a 128-byte line touches
// parts of every line it touches.  FULL: every amplitude is read and
// written (streaming), the factor applied where the controls hold (for a
// fixed bit 0 the touched pieces are 16 bytes apart and partial writes
// cost whole sectors); otherwise one thread per index, and only the
// threads whose index satisfies the controls load and store.
template <typename R, bool FULL>
__global__ __launch_bounds__(kBlock) void k_diag_lines(typename Vec<R>::T* __restrict__ psi, uint64_t dim,
                                                        uint64_t cmask, int nsel, int s0, int s1, M4<R> d) {
    for (uint64_t chunk = blockIdx.x; chunk * kBlock < dim; chunk += gridDim.x) {
        const uint64_t i = chunk * kBlock + threadIdx.x;
        if (i >= dim) continue;
        const bool hit = (i & cmask) == cmask;
        if (!FULL && !hit) continue;
        int sel = 0;
        if (nsel >= 1) sel = (int)((i >> s0) & 1);
        if (nsel == 2) sel = 2 * sel + (int)((i >> s1) & 1);
        Cx<R> f = d.e[0];
        f = csel(sel == 1, d.e[1], f);
        f = csel(sel == 2, d.e[2], f);
        f = csel(sel == 3, d.e[3], f);
        if constexpr (FULL) {
            const Cx<R> a = ld_stream<R>(psi, i);
            st_stream<R>(psi, i, csel(hit, cmul(f, a), a));
        } else {
            st<R>(psi, i, cmul(f, ld<R>(psi, i)));
        }
    }
}

template <typename R, int IT, bool NT>
__global__ __launch_bounds__(kBlock) void k_permx(typename Vec<R>::T* __restrict__ psi, uint64_t ngroups,
                                                   Ins ins, uint64_t tbit, uint64_t ilv) {
    for (uint64_t chunk = blockIdx.x; chunk * (IT * kBlock) < ngroups; chunk += gridDim.x) {
        const uint64_t g0 = chunk_slot(chunk, ilv) * (IT * kBlock) + threadIdx.x;
        uint64_t i0[IT];
        Cx<R> a[IT], b[IT];
#pragma unroll
        for (int u = 0; u < IT; ++u) {
            const uint64_t g = g0 + (uint64_t)u * kBlock;
            if (g < ngroups) {
                i0[u] = expand(g, ins);
                a[u] = ld_pg<R, NT>(psi, i0[u]);
                b[u] = ld_pg<R, NT>(psi, i0[u] | tbit);
            }
        }
#pragma unroll
        for (int u = 0; u < IT; ++u) {
            const uint64_t g = g0 + (uint64_t)u * kBlock;
            if (g < ngroups) {
                st_pg<R, NT>(psi, i0[u], b[u]);
                st_pg<R, NT>(psi, i0[u] | tbit, a[u]);
            }
        }
    }
}


// One tile per wavefront.  LITE: the pass holds only op kinds of
// kLiteKinds, and the op loop is compiled for those alone.  Fewer registers
// give more waves per SIMD to overlap one wave's loads and stores with
// another's arithmetic.  Measured at N=30 on layers of Haar-random U(2) and
// CZ gates: complex128 (2^4 slots) 94 instead of 121 VGPRs, 5 waves per
// SIMD instead of 4, the circuit 3.0% faster; complex64 (2^5 slots) 86
// instead of 112, 7.2% faster.
template <typename R, int K, int F, bool LITE>
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
    run_ops<R, K, LITE>(a, ops, P.n_ops, base, wave_uniform(tile_base(P, wave, 0)), lane);
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

// SHORBOX (App. A): amplitude a at index x + 2^n_x (y^x mod G) for every x
// of the n_x-qubit x-register; the state has been zeroed before.  Each
// thread raises y to its own x by square-and-multiply (G < 2^32, so every
// product fits in 64 bits).
__device__ __forceinline__ uint64_t pow_mod(uint64_t y, uint64_t e, uint64_t G) {
    uint64_t r = 1 % G, b = y % G;
    while (e) {
        if (e & 1) r = r * b % G;
        b = b * b % G;
        e >>= 1;
    }
    return r;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_shorbox(typename Vec<R>::T* __restrict__ psi, int n_x, uint64_t G,
                                                     uint64_t y, double a) {
    const uint64_t nx = 1ull << n_x;
    for (uint64_t x = (uint64_t)blockIdx.x * kBlock + threadIdx.x; x < nx; x += (uint64_t)gridDim.x * kBlock) {
        typename Vec<R>::T v;
        v.x = (R)a;
        v.y = (R)0;
        psi[x + (pow_mod(y, x, G) << n_x)] = v;
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

// Sampling prefixes (see device_common.hpp): one thread per super-block
__global__ void k_sample_block_prefix(const double* __restrict__ bsum, uint64_t nblocks, uint64_t nsuper,
                                      double* __restrict__ bp, double* __restrict__ ssum) {
    const uint64_t sb = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (sb >= nsuper) return;
    const uint64_t lo = sb << kSampleSuperBits;
    const uint64_t hi = lo + (1ull << kSampleSuperBits) < nblocks ? lo + (1ull << kSampleSuperBits) : nblocks;
    double r = 0.0;
    for (uint64_t b = lo; b < hi; ++b) {
        bp[b] = r;
        r = r + bsum[b];
    }
    ssum[sb] = r;
}

__global__ void k_sample_super_prefix(const double* __restrict__ ssum, uint64_t nsuper, double* __restrict__ sp) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double r = 0.0;
    for (uint64_t i = 0; i < nsuper; ++i) {
        sp[i] = r;
        r = r + ssum[i];
    }
    sp[nsuper] = r;
}

__global__ void k_sum_parts(const double* __restrict__ partial, uint64_t nbins, uint32_t parts,
                            double* __restrict__ out) {
    const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbins) return;
    double s = 0.0;
    for (uint32_t p = 0; p < parts; ++p) s += partial[b * parts + p];
    out[b] = s;
}

// The sum of n values in a fixed order by one wave: lane l adds values l,
// l + 64, ... in turn, then the lanes combine by halving distance.  Every
// lane must call it; lane 0 gets the sum.
__device__ __forceinline__ double wave_sum_fixed(const double* __restrict__ v, uint32_t n) {
    double s = 0.0;
    for (uint32_t p = threadIdx.x & 63; p < n; p += 64) s += v[p];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    return s;
}

// Many parts per bin: one 64-thread block (a wave) per bin.
__global__ void k_sum_parts_wave(const double* __restrict__ partial, uint32_t parts, double* __restrict__ out) {
    const double s = wave_sum_fixed(partial + (uint64_t)blockIdx.x * parts, parts);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// One 64-thread block.
__global__ void k_expect_final(const double* __restrict__ partial, uint32_t parts, int q, int n,
                               double* __restrict__ out) {
    double s[4];
    for (int c = 0; c < 4; ++c) s[c] = wave_sum_fixed(partial + (uint64_t)c * parts, parts);
    if (threadIdx.x != 0) return;
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


// A control bit inside a 128-byte line (below qubit 3 for complex128, 4
// for complex64) leaves parts of every line untouched: such gates keep
// plain (cached) accesses, measured faster there than the streaming hint.
template <typename R>
bool partial_lines(uint64_t cmask) {
    const uint64_t line_bits = sizeof(R) == 8 ? 3 : 4;
    return (cmask & ((1ull << line_bits) - 1)) != 0;
}

// The chunk interleave for a per-gate kernel (see chunk_slot): on when a
// fixed control bit of the op lies on byte-address bit 10, 11 or 20 (the
// bits measured to concentrate in-order requests on few channels) and the
// chunks are full and a multiple of 64.
template <typename R>
uint64_t chunk_interleave(uint64_t ngroups, uint64_t per_chunk, uint64_t cmask) {
    constexpr int lb = sizeof(R) == 8 ? 4 : 3;  // log2 of the amplitude's bytes
    const uint64_t channel_bits = (1ull << (10 - lb)) | (1ull << (11 - lb)) | (1ull << (20 - lb));
    if (!(cmask & channel_bits) || ngroups % per_chunk) return 0;
    const uint64_t nchunks = ngroups / per_chunk;
    return nchunks >= 64 && nchunks % 64 == 0 ? nchunks / 64 : 0;
}

unsigned chunk_blocks(uint64_t items, uint64_t per_block) {
    const uint64_t b = (items + per_block - 1) / per_block;
    return (unsigned)(b < 1 ? 1 : b < (1ull << 22) ? b : (1ull << 22));
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

// targets 0-2 of an uncontrolled 2x2 or X (2^n >= 256)
template <typename R, bool PERM>
void launch_pair_lane(typename Vec<R>::T* psi, int n, int t, const M4<R>& m, hipStream_t st) {
    const uint64_t dim = 1ull << n;
    const unsigned blocks = chunk_blocks(dim, kBlock);
    if (t == 0) hipLaunchKernelGGL((k_pair_lane<R, 0, PERM>), dim3(blocks), dim3(kBlock), 0, st, psi, dim, m);
    else if (t == 1) hipLaunchKernelGGL((k_pair_lane<R, 1, PERM>), dim3(blocks), dim3(kBlock), 0, st, psi, dim, m);
    else hipLaunchKernelGGL((k_pair_lane<R, 2, PERM>), dim3(blocks), dim3(kBlock), 0, st, psi, dim, m);
}

// uncontrolled two-qubit gate with its lower qubit inside a line (2^n >= 512)
template <typename R>
void launch_quad_lane(typename Vec<R>::T* psi, int n, const GateOp& op, const M16<R>& m, hipStream_t st) {
    const int lo = std::min(op.t0, op.t1), hi = std::max(op.t0, op.t1);
    const bool lsb = lo == op.t1;
    const uint64_t npairs = 1ull << (n - 1);
    const unsigned blocks = chunk_blocks(npairs, kBlock);
#define JQ_QUAD(L, B) hipLaunchKernelGGL((k_quad_lane<R, L, B>), dim3(blocks), dim3(kBlock), 0, st, psi, npairs, hi, m)
    if (lo == 0) { if (lsb) JQ_QUAD(0, true); else JQ_QUAD(0, false); }
    else if (lo == 1) { if (lsb) JQ_QUAD(1, true); else JQ_QUAD(1, false); }
    else if (lo == 2) { if (lsb) JQ_QUAD(2, true); else JQ_QUAD(2, false); }
    else { if (lsb) JQ_QUAD(3, true); else JQ_QUAD(3, false); }
#undef JQ_QUAD
}

// wide_mask: targets whose bit is set take four pairs per thread, the
// others one (measured at N=30 complex128: one pair is as fast or faster on
// almost every target; complex64 differs target by target)
template <typename R>
void apply_op_t(typename Vec<R>::T* psi, int n, const GateOp& op, uint64_t wide_mask, hipStream_t st) {
    const bool wide = (wide_mask >> op.t0) & 1;
    const int fixed = __builtin_popcountll(op.cmask);
    switch (op.kind) {
        case OP_DENSE1: {
            const uint64_t tb = 1ull << op.t0;
            const uint64_t ng = 1ull << (n - 1 - fixed);
            M4<R> m;
            for (int i = 0; i < 4; ++i) m.e[i] = {(R)op.m[i].re, (R)op.m[i].im};
            const Ins ins = make_ins(op.cmask | tb, op.cmask);
            if (op.cmask == 0 && op.t0 < 3 && n >= 8)
                launch_pair_lane<R, false>(psi, n, op.t0, m, st);
            else if (partial_lines<R>(op.cmask))
                hipLaunchKernelGGL((k_dense1<R, 4, false>), dim3(chunk_blocks(ng, 4 * kBlock)), dim3(kBlock), 0, st,
                                   psi, ng, ins, tb, m, uint64_t(0));
            else if (!wide)
                hipLaunchKernelGGL((k_dense1<R, 1, true>), dim3(chunk_blocks(ng, kBlock)), dim3(kBlock), 0, st, psi,
                                   ng, ins, tb, m, chunk_interleave<R>(ng, kBlock, op.cmask));
            else
                hipLaunchKernelGGL((k_dense1<R, 4, true>), dim3(chunk_blocks(ng, 4 * kBlock)), dim3(kBlock), 0, st,
                                   psi, ng, ins, tb, m, chunk_interleave<R>(ng, 4 * kBlock, op.cmask));
            break;
        }
        case OP_DENSE2: {
            const uint64_t hb = 1ull << op.t0, lb = 1ull << op.t1;
            const uint64_t ng = 1ull << (n - 2 - fixed);
            M16<R> m;
            for (int i = 0; i < 16; ++i) m.e[i] = {(R)op.m[i].re, (R)op.m[i].im};
            if (op.cmask == 0 && std::min(op.t0, op.t1) < (sizeof(R) == 4 ? 4 : 3) && n >= 9) {
                launch_quad_lane<R>(psi, n, op, m, st);
                break;
            }
            hipLaunchKernelGGL(k_dense2<R>, dim3(chunk_blocks(ng, 2 * kBlock)), dim3(kBlock), 0, st, psi, ng,
                               make_ins(op.cmask | hb | lb, op.cmask), hb, lb, m);
            break;
        }
        case OP_DIAG: {
            const uint64_t ng = 1ull << (n - fixed);
            M4<R> d;
            for (int i = 0; i < 4; ++i) d.e[i] = {(R)op.m[i].re, (R)op.m[i].im};
            const Ins ins = make_ins(op.cmask, op.cmask);
            const int s0 = op.t0 < 0 ? 0 : op.t0, s1 = op.t1 < 0 ? 0 : op.t1;
            if (partial_lines<R>(op.cmask)) {
                // controls inside the line (measured, CZ at N=30 complex128:
                // lowest qubit 0 1.64 TB/s of algorithmic bytes read and
                // written whole vs 1.24 touched only; lowest qubit 2 3.5 vs
                // 2.6 TB/s one thread per index)
                const uint64_t dim = 1ull << n;
                if (op.cmask & 1)
                    hipLaunchKernelGGL((k_diag_lines<R, true>), dim3(chunk_blocks(dim, kBlock)), dim3(kBlock), 0, st,
                                       psi, dim, op.cmask, op.nsel, s0, s1, d);
                else
                    hipLaunchKernelGGL((k_diag_lines<R, false>), dim3(chunk_blocks(dim, kBlock)), dim3(kBlock), 0, st,
                                       psi, dim, op.cmask, op.nsel, s0, s1, d);
            } else {
                hipLaunchKernelGGL((k_diag<R, 1, true>), dim3(chunk_blocks(ng, kBlock)), dim3(kBlock), 0, st, psi,
                                   ng, ins, op.nsel, s0, s1, d, chunk_interleave<R>(ng, kBlock, op.cmask));
            }
            break;
        }
        case OP_PERMX: {
            const uint64_t tb = 1ull << op.t0;
            const uint64_t ng = 1ull << (n - 1 - fixed);
            const Ins ins = make_ins(op.cmask | tb, op.cmask);
            if (op.cmask == 0 && op.t0 < 3 && n >= 8)
                launch_pair_lane<R, true>(psi, n, op.t0, M4<R>{}, st);
            else if (partial_lines<R>(op.cmask))
                hipLaunchKernelGGL((k_permx<R, 4, false>), dim3(chunk_blocks(ng, 4 * kBlock)), dim3(kBlock), 0, st,
                                   psi, ng, ins, tb, uint64_t(0));
            else if (!wide)
                hipLaunchKernelGGL((k_permx<R, 1, true>), dim3(chunk_blocks(ng, kBlock)), dim3(kBlock), 0, st, psi,
                                   ng, ins, tb, chunk_interleave<R>(ng, kBlock, op.cmask));
            else
                hipLaunchKernelGGL((k_permx<R, 4, true>), dim3(chunk_blocks(ng, 4 * kBlock)), dim3(kBlock), 0, st,
                                   psi, ng, ins, tb, chunk_interleave<R>(ng, 4 * kBlock, op.cmask));
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
    if (waves >= (1ull << 26)) fail(JQ_EUNSUPPORTED, "fused pass: too many tiles for one launch (use more register qubits)");
    if (p.kinds != 0 && (p.kinds & ~kLiteKinds) == 0)
        hipLaunchKernelGGL((k_fused<R, K, F, true>), dim3(blocks_for(waves, wpb)), dim3(64 * wpb), 0, st, psi, p, p.ops);
    else
        hipLaunchKernelGGL((k_fused<R, K, F, false>), dim3(blocks_for(waves, wpb)), dim3(64 * wpb), 0, st, psi, p, p.ops);
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

void sv_shorbox(int enc, void* psi, int n, int n_x, uint64_t G, uint64_t y, hipStream_t st) {
    sv_init(enc, psi, n, JQ_INIT_BASIS, ~0ull, st);  // no basis state matches: all zero
    const uint64_t nx = 1ull << n_x;
    const double a = uniform_amplitude(n_x);
    if (enc == JQ_C128)
        hipLaunchKernelGGL(k_shorbox<double>, dim3(grid_stride_blocks(nx)), dim3(kBlock), 0, st, (double2*)psi, n_x, G,
                           y, a);
    else
        hipLaunchKernelGGL(k_shorbox<float>, dim3(grid_stride_blocks(nx)), dim3(kBlock), 0, st, (float2*)psi, n_x, G,
                           y, a);
    JQ_HIP(hipGetLastError());
}

void sv_apply_op(int enc, void* psi, int n, const GateOp& op, uint64_t wide_mask, hipStream_t st) {
    if (enc == JQ_C128) apply_op_t<double>((double2*)psi, n, op, wide_mask, st);
    else apply_op_t<float>((float2*)psi, n, op, wide_mask, st);
}

void sv_apply_fused(int enc, void* psi, int n, const FPass& pass, int k_reg, int fixed_lane_bits, hipStream_t st) {
    check_table_tag(pass, enc == JQ_C128 ? dg_table_tag<double>() : dg_table_tag<float>());
    if ((1 << k_reg) > (enc == JQ_C128 ? kDgSlotsF64 : kDgSlotsF32) && pass.table_tag != 0)
        fail(JQ_EINVAL, "fused pass: diagonal table smaller than the register tile");
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

void sv_sample(int enc, const void* psi, int n, const double* u, uint64_t count, uint64_t* out, double* scratch,
               hipStream_t st) {
    if (enc == JQ_C128) launch_sample(LoaderSV<double>{(const double2*)psi}, n, u, count, out, scratch, st);
    else launch_sample(LoaderSV<float>{(const float2*)psi}, n, u, count, out, scratch, st);
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

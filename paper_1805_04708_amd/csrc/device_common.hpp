// Device helpers shared by the state-vector and two-byte-code kernels:
// complex arithmetic, index expansion, and the FP64 reduction kernels, which
// take a loader so that both storage formats reuse them.
#pragma once

#include "internal.hpp"

namespace jq {

constexpr int kBlock = 256;

template <typename R>
struct Vec;
template <>
struct Vec<double> {
    using T = double2;
};
template <>
struct Vec<float> {
    using T = float2;
};

template <typename R>
struct Cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ Cx<R> cadd(Cx<R> a, Cx<R> b) {
    return {a.re + b.re, a.im + b.im};
}
template <typename R>
__device__ __forceinline__ Cx<R> csel(bool c, Cx<R> a, Cx<R> b) {
    return {c ? a.re : b.re, c ? a.im : b.im};
}

template <typename R>
__device__ __forceinline__ Cx<R> ld(const typename Vec<R>::T* p, uint64_t i) {
    typename Vec<R>::T v = p[i];
    return {v.x, v.y};
}
template <typename R>
__device__ __forceinline__ void st(typename Vec<R>::T* p, uint64_t i, Cx<R> a) {
    typename Vec<R>::T v;
    v.x = a.re;
    v.y = a.im;
    p[i] = v;
}

// a*x + b*y as a chain of fused multiply-adds: 8 FP instructions per
// complex result, the minimum for a dense 2x2 row.
template <typename R>
__device__ __forceinline__ Cx<R> mac2(Cx<R> a, Cx<R> x, Cx<R> b, Cx<R> y) {
    R re = a.re * x.re;
    re = fma(-a.im, x.im, re);
    re = fma(b.re, y.re, re);
    re = fma(-b.im, y.im, re);
    R im = a.re * x.im;
    im = fma(a.im, x.re, im);
    im = fma(b.re, y.im, im);
    im = fma(b.im, y.re, im);
    return {re, im};
}

template <typename R>
__device__ __forceinline__ Cx<R> cmulf(Cx<R> a, Cx<R> x) {
    R re = a.re * x.re;
    re = fma(-a.im, x.im, re);
    R im = a.re * x.im;
    im = fma(a.im, x.re, im);
    return {re, im};
}

// Insert zero bits at sorted positions, then set the bits of `ones`.
struct Ins {
    int32_t cnt;
    int32_t pos[7];
    uint64_t ones;
};

__device__ __forceinline__ uint64_t expand(uint64_t g, const Ins& s) {
    for (int i = 0; i < s.cnt; ++i) {
        const int p = s.pos[i];
        g = ((g >> p) << (p + 1)) | (g & ((1ull << p) - 1));
    }
    return g | s.ones;
}

template <typename R>
struct M4 {
    Cx<R> e[4];
};
template <typename R>
struct M16 {
    Cx<R> e[16];
};



// Insert zero bits at up to 32 sorted positions (reductions over many qubits).
struct InsN {
    int32_t cnt;
    int32_t pos[32];
};

__device__ __forceinline__ uint64_t expand_n(uint64_t g, const InsN& s) {
    for (int i = 0; i < s.cnt; ++i) {
        const int p = s.pos[i];
        g = ((g >> p) << (p + 1)) | (g & ((1ull << p) - 1));
    }
    return g;
}

// Fixed-order block sum: within the wave by halving distance, then the
// waves in order.  Every thread must call it; thread 0 gets the sum.
__device__ __forceinline__ double block_sum(double v, double* lds) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += lds[i];
    __syncthreads();
    return s;
}

struct Dep {
    int32_t nq;
    int32_t q[30];
};

// Marginal distribution: block (bin, part) sums |a|^2 over the indices whose
// selected bits spell `bin`, for its contiguous share of the other bits.
// With W > 1 (every selected qubit at position log2(W) or above) a thread
// takes W consecutive amplitudes at a time (loader method modulus2_w).
template <class L, int W>
__global__ __launch_bounds__(kBlock) void k_probs(L ldr, InsN others, Dep sel, uint64_t n_others, uint32_t parts,
                                                   double* __restrict__ partial) {
    __shared__ double lds[kBlock / 64];
    ldr.prepare();
    const uint64_t bin = blockIdx.x / parts;
    const uint64_t part = blockIdx.x % parts;
    const uint64_t n_w = n_others / W;
    const uint64_t chunk = (n_w + parts - 1) / parts;
    const uint64_t lo = part * chunk;
    const uint64_t hi = lo + chunk < n_w ? lo + chunk : n_w;
    uint64_t binoff = 0;
    for (int m = 0; m < sel.nq; ++m) binoff |= ((bin >> m) & 1ull) << sel.q[m];
    auto term = [&](uint64_t o) {
        if constexpr (W == 1) return ldr.modulus2(expand_n(o, others) | binoff);
        else return ldr.template modulus2_w<W>(expand_n(o * W, others) | binoff);
    };
    // eight loads in flight per thread; the sum still runs in index order
    double acc = 0.0;
    uint64_t o = lo + threadIdx.x;
    for (; o + 7 * kBlock < hi; o += 8 * kBlock) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = term(o + u * kBlock);
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += t[u];
    }
    for (; o < hi; o += kBlock) acc += term(o);
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Few other bits: one thread per bin sums its 2^(N-nq) entries in order.
template <class L>
__global__ __launch_bounds__(kBlock) void k_probs_by_bin(L ldr, InsN others, Dep sel, uint64_t n_others,
                                                          uint64_t nbins, double* __restrict__ out) {
    ldr.prepare();
    const uint64_t bin = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (bin >= nbins) return;
    uint64_t binoff = 0;
    for (int m = 0; m < sel.nq; ++m) binoff |= ((bin >> m) & 1ull) << sel.q[m];
    double acc = 0.0;
    for (uint64_t o = 0; o < n_others; ++o) acc += ldr.modulus2(expand_n(o, others) | binoff);
    out[bin] = acc;
}

__global__ void k_sum_parts(const double* __restrict__ partial, uint64_t nbins, uint32_t parts,
                            double* __restrict__ out);
__global__ void k_sum_parts_wave(const double* __restrict__ partial, uint32_t parts, double* __restrict__ out);

// Sums over amplitude pairs (i, j = i | 2^q) of 2 Re(conj(a_i) a_j),
// 2 Im(conj(a_i) a_j), |a_i|^2 - |a_j|^2 and |a_i|^2 + |a_j|^2: the
// expectations of sigma^x, sigma^y, sigma^z on qubit q and the norm.
template <class L>
__global__ __launch_bounds__(kBlock) void k_expect(L ldr, Ins ins, uint64_t qbit, uint64_t npairs, uint32_t parts,
                                                    double* __restrict__ partial) {
    __shared__ double lds[kBlock / 64];
    ldr.prepare();
    const uint64_t chunk = (npairs + parts - 1) / parts;
    const uint64_t lo = (uint64_t)blockIdx.x * chunk;
    const uint64_t hi = lo + chunk < npairs ? lo + chunk : npairs;
    double sx = 0, sy = 0, sz = 0, nr = 0;
    auto add = [&](const Cx<double>& a, const Cx<double>& b) {
        sx += 2.0 * (a.re * b.re + a.im * b.im);
        sy += 2.0 * (a.re * b.im - a.im * b.re);
        const double pa = a.re * a.re + a.im * a.im, pb = b.re * b.re + b.im * b.im;
        sz += pa - pb;
        nr += pa + pb;
    };
    // four pairs (eight loads) in flight per thread, summed in index order
    uint64_t g = lo + threadIdx.x;
    for (; g + 3 * kBlock < hi; g += 4 * kBlock) {
        Cx<double> a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t i = expand(g + u * kBlock, ins);
            a[u] = ldr.amp(i);
            b[u] = ldr.amp(i | qbit);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) add(a[u], b[u]);
    }
    for (; g < hi; g += kBlock) {
        const uint64_t i = expand(g, ins);
        add(ldr.amp(i), ldr.amp(i | qbit));
    }
    double r[4] = {sx, sy, sz, nr};
    for (int c = 0; c < 4; ++c) {
        const double s = block_sum(r[c], lds);
        if (threadIdx.x == 0) partial[(uint64_t)c * parts + blockIdx.x] = s;
    }
}

// ------------------------------------------------------------ sampling --
//
// Inverse-CDF sampling of basis states (App. A, GENERATE EVENTS).  The
// cumulative probability of amplitude i is a sum of sums at four levels:
// 16 amplitudes per thread, 256 threads per block (4096 amplitudes), 4096
// blocks per super-block, then the super-blocks; every level's total is the
// sequential sum (from 0.0) of its children's totals, and the running value
// at i is SP[sb] + (BP[b] + (T_t + w_k)).  At each level's end the running
// value therefore equals the next start exactly, so it never decreases and
// the search for the first value above a target ends inside the block the
// prefix search chose.


template <class L>
__global__ __launch_bounds__(kBlock) void k_sample_block_sums(L ldr, uint64_t dim, uint64_t nblocks,
                                                              double* __restrict__ bsum) {
    __shared__ double cs[kBlock];
    ldr.prepare();
    for (uint64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
        const uint64_t first = (blk << kSampleBlockBits) + (uint64_t)threadIdx.x * kSampleLeaf;
        double w = 0.0;
#pragma unroll
        for (int k = 0; k < kSampleLeaf; ++k)
            if (first + k < dim) w = w + ldr.modulus2(first + k);
        cs[threadIdx.x] = w;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int j = 0; j < kBlock; ++j) t = t + cs[j];
            bsum[blk] = t;
        }
        __syncthreads();
    }
}

// one thread per super-block: exclusive running sums of its blocks
__global__ void k_sample_block_prefix(const double* __restrict__ bsum, uint64_t nblocks, uint64_t nsuper,
                                      double* __restrict__ bp, double* __restrict__ ssum);
// one thread: exclusive running sums of the super-blocks, then the total
__global__ void k_sample_super_prefix(const double* __restrict__ ssum, uint64_t nsuper, double* __restrict__ sp);

// One workgroup per draw (grid-stride over the draws).
template <class L>
__global__ __launch_bounds__(kBlock) void k_sample(L ldr, uint64_t dim, const double* __restrict__ sp,
                                                    uint64_t nsuper, const double* __restrict__ bp, uint64_t nblocks,
                                                    const double* __restrict__ u, uint64_t count,
                                                    uint64_t* __restrict__ out) {
    __shared__ double pv[kBlock * kSampleLeaf];
    __shared__ double cs[kBlock];
    ldr.prepare();
    const double total = sp[nsuper];
    for (uint64_t d = blockIdx.x; d < count; d += gridDim.x) {
        const double target = u[d] * total;
        // last super-block, then last block in it, whose start is <= target
        uint64_t lo = 0, hi = nsuper - 1;
        while (lo < hi) {
            const uint64_t mid = (lo + hi + 1) / 2;
            if (sp[mid] <= target) lo = mid; else hi = mid - 1;
        }
        const uint64_t sb = lo;
        const double s0 = sp[sb];
        uint64_t blo = sb << kSampleSuperBits;
        uint64_t bhi = blo + (1ull << kSampleSuperBits) < nblocks ? blo + (1ull << kSampleSuperBits) - 1 : nblocks - 1;
        while (blo < bhi) {
            const uint64_t mid = (blo + bhi + 1) / 2;
            if (s0 + bp[mid] <= target) blo = mid; else bhi = mid - 1;
        }
        const uint64_t blk = blo;
        const double b0 = bp[blk];
        const uint64_t first = (blk << kSampleBlockBits) + (uint64_t)threadIdx.x * kSampleLeaf;
        double w = 0.0;
#pragma unroll
        for (int k = 0; k < kSampleLeaf; ++k) {
            const double p = first + k < dim ? ldr.modulus2(first + k) : 0.0;
            pv[threadIdx.x * kSampleLeaf + k] = p;
            w = w + p;
        }
        cs[threadIdx.x] = w;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t idx = ~0ull;
            double t = 0.0;
            for (int j = 0; j < kBlock && idx == ~0ull; ++j) {
                if (s0 + (b0 + (t + cs[j])) > target) {
                    double wk = 0.0;
                    for (int k = 0; k < kSampleLeaf; ++k) {
                        wk = wk + pv[j * kSampleLeaf + k];
                        if (s0 + (b0 + (t + wk)) > target) {
                            idx = (blk << kSampleBlockBits) + (uint64_t)(j * kSampleLeaf + k);
                            break;
                        }
                    }
                }
                t = t + cs[j];
            }
            if (idx == ~0ull) {
                // target at the very top (u rounded up to the total): the last
                // amplitude of the block with non-zero probability
                idx = blk << kSampleBlockBits;
                for (int e = kBlock * kSampleLeaf - 1; e >= 0; --e)
                    if (pv[e] > 0.0) {
                        idx = (blk << kSampleBlockBits) + (uint64_t)e;
                        break;
                    }
            }
            out[d] = idx;
        }
        __syncthreads();
    }
}

__global__ void k_expect_final(const double* __restrict__ partial, uint32_t parts, int q, int n,
                               double* __restrict__ out);

Ins make_ins(uint64_t zero_bits, uint64_t ones);
unsigned blocks_for(uint64_t items, uint64_t per_block);
unsigned grid_stride_blocks(uint64_t dim);

// W: amplitudes per loader access in the main kernel (1, or 16 when the
// loader has modulus2_w<16>; used only if no selected qubit is below 4)
template <class L, int W = 1>
void launch_probs(const L& ldr, int n, const int* qubits, int nq, double* out, double* partial, size_t cap,
                  hipStream_t st) {
    uint64_t selmask = 0;
    Dep d{};
    d.nq = nq;
    for (int m = 0; m < nq; ++m) {
        selmask |= 1ull << qubits[m];
        d.q[m] = qubits[m];
    }
    const uint64_t nbins = 1ull << nq;
    const uint64_t n_others = 1ull << (n - nq);
    InsN others{};
    for (int p = 0; p < n; ++p)
        if (selmask & (1ull << p)) others.pos[others.cnt++] = p;
    if (n_others <= 64) {
        hipLaunchKernelGGL(k_probs_by_bin<L>, dim3(blocks_for(nbins, kBlock)), dim3(kBlock), 0, st, ldr, others, d,
                           n_others, nbins, out);
        JQ_HIP(hipGetLastError());
        return;
    }
    bool wide = W > 1 && n_others >= (uint64_t)W * kBlock;
    for (int m = 0; m < nq && wide; ++m) wide = (1ull << qubits[m]) >= (uint64_t)W;
    // Blocks: one resident round of the device for up to 64 bins (each block
    // streams one long chunk), two rounds for more bins, whose zero-bit
    // insertion costs more arithmetic per amplitude (both measured).
    int dev = 0, cus = 0, per_cu = 0;
    JQ_HIP(hipGetDevice(&dev));
    JQ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    JQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, wide ? (const void*)k_probs<L, W> : (const void*)k_probs<L, 1>, kBlock, 0));
    const uint64_t round = (uint64_t)(cus > 0 ? cus : 1) * (uint64_t)(per_cu > 0 ? per_cu : 1);
    uint64_t parts = n_others / (kBlock * 16);
    if (parts < 1) parts = 1;
    uint64_t want = (nbins <= 64 ? round : 2 * round) / nbins;
    if (want < 1) want = 1;
    if (parts > want) parts = want;
    if (nbins * parts > cap) parts = cap / nbins;
    if (parts < 1) fail(JQ_EINVAL, "reduction scratch too small");
    if (wide) {
        if constexpr (W > 1)
            hipLaunchKernelGGL((k_probs<L, W>), dim3((unsigned)(nbins * parts)), dim3(kBlock), 0, st, ldr, others, d,
                               n_others, (uint32_t)parts, partial);
    } else {
        hipLaunchKernelGGL((k_probs<L, 1>), dim3((unsigned)(nbins * parts)), dim3(kBlock), 0, st, ldr, others, d,
                           n_others, (uint32_t)parts, partial);
    }
    JQ_HIP(hipGetLastError());
    // the parts of a bin in a fixed order: by one thread when they are few,
    // by one wave per bin otherwise (64 times shorter a chain of loads)
    if (parts < 64)
        hipLaunchKernelGGL(k_sum_parts, dim3(blocks_for(nbins, 64)), dim3(64), 0, st, partial, nbins,
                           (uint32_t)parts, out);
    else
        hipLaunchKernelGGL(k_sum_parts_wave, dim3((unsigned)nbins), dim3(64), 0, st, partial, (uint32_t)parts, out);
    JQ_HIP(hipGetLastError());
}

// u_dev: count draws in [0, 1) (device); out_dev: count indices (device).
template <class L>
void launch_sample(const L& ldr, int n, const double* u_dev, uint64_t count, uint64_t* out_dev, double* scratch,
                   hipStream_t st) {
    const uint64_t dim = 1ull << n;
    const uint64_t nblocks = n > kSampleBlockBits ? 1ull << (n - kSampleBlockBits) : 1;
    const uint64_t nsuper = (nblocks + (1ull << kSampleSuperBits) - 1) >> kSampleSuperBits;
    double* bsum = scratch;
    double* bp = bsum + nblocks;
    double* ssum = bp + nblocks;
    double* sp = ssum + nsuper;
    hipLaunchKernelGGL(k_sample_block_sums<L>, dim3((unsigned)(nblocks < (1ull << 20) ? nblocks : (1ull << 20))),
                       dim3(kBlock), 0, st, ldr, dim, nblocks, bsum);
    hipLaunchKernelGGL(k_sample_block_prefix, dim3(blocks_for(nsuper, 64)), dim3(64), 0, st, bsum, nblocks, nsuper,
                       bp, ssum);
    hipLaunchKernelGGL(k_sample_super_prefix, dim3(1), dim3(64), 0, st, ssum, nsuper, sp);
    if (count) {
        const unsigned grid = (unsigned)(count < 16384 ? count : 16384);
        hipLaunchKernelGGL(k_sample<L>, dim3(grid), dim3(kBlock), 0, st, ldr, dim, sp, nsuper, bp, nblocks, u_dev,
                           count, out_dev);
    }
    JQ_HIP(hipGetLastError());
}

template <class L>
void launch_expect(const L& ldr, int n, double* out, double* partial, size_t cap, hipStream_t st) {
    const uint64_t npairs = 1ull << (n - 1);
    uint64_t parts = npairs / (kBlock * 16);
    if (parts < 1) parts = 1;
    if (parts > 2048) parts = 2048;
    if (4 * parts > cap) parts = cap / 4;
    for (int q = 0; q < n; ++q) {
        const uint64_t qb = 1ull << q;
        hipLaunchKernelGGL(k_expect<L>, dim3((unsigned)parts), dim3(kBlock), 0, st, ldr, make_ins(qb, 0), qb, npairs,
                           (uint32_t)parts, partial);
        hipLaunchKernelGGL(k_expect_final, dim3(1), dim3(64), 0, st, partial, (uint32_t)parts, q, n, out);
    }
    JQ_HIP(hipGetLastError());
}

}  // namespace jq

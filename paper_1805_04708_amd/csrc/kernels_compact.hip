// HIP kernels for the adaptive two-byte polar code of Sec. 4.1.
//
// Storage: plane b0 (modulus codes) then plane b1 (phase codes), one int8
// per amplitude each, plus the FP64 range (r0, r1) in device memory.
// Decoding: b0 = -128 is 0, b0 = 127 is modulus 1, other codes give
// r = (b0+127)(r1-r0)/253 + r0; the phase is pi*b1/128.  After a gate the
// range is recomputed as the min and max of |z| over 0 < |z| < 1 (a
// modulus >= 1 - 1e-12 counts as one) and every amplitude is re-encoded;
// a gate that cannot change any modulus (permutation, or diagonal with
// modulus-one entries) keeps the range.
//
// A general gate takes two sweeps with no host round trip: k_cp_gate in
// range mode decodes, applies the gate in FP64 and reduces min/max |z'|
// into two ordered 64-bit patterns (atomic min/max: order independent and
// exact); k_cp_resolve turns them into the new range (or keeps the old one
// when no modulus lies strictly inside (0, 1)); k_cp_gate in apply mode
// decodes with the old range, applies, and encodes with the new one.
// Permutations swap code pairs; modulus-preserving diagonal gates rewrite
// the phase codes of the touched amplitudes only, by an integer shift of
// the code unless the shift is a half-integer.
//
// This file is compiled with -ffp-contract=off: each product and sum
// rounds on its own, in the order written, so the codes do not depend on
// fused multiply-adds.
#include "fused_ops.hpp"

namespace jq {

constexpr double kOneTol = 1e-12;
constexpr double kPiD = 3.14159265358979323846;

// cos/sin(pi*c/128) for c = -128..127, filled from the host C library
__constant__ double c_cos[256];
__constant__ double c_sin[256];

struct Range {
    double r0, r1;
};

__device__ __forceinline__ Cx<double> decode(int c0, int c1, Range g) {
    if (c0 == -128) return {0.0, 0.0};
    const double r = c0 == 127 ? 1.0 : ((double)(c0 + 127) * (g.r1 - g.r0)) / 253.0 + g.r0;
    return {r * c_cos[c1 + 128], r * c_sin[c1 + 128]};
}

__device__ __forceinline__ double modulus(Cx<double> z) {
    return sqrt(z.re * z.re + z.im * z.im);
}

__device__ __forceinline__ int encode_mod(double a, Range g) {
    if (a == 0.0) return -128;
    if (a >= 1.0 - kOneTol) return 127;
    if (g.r1 == g.r0) return -127;
    const double q = rint((253.0 * (a - g.r0)) / (g.r1 - g.r0));
    double v = -127.0 + q;
    v = v < -127.0 ? -127.0 : v;
    v = v > 126.0 ? 126.0 : v;
    return (int)v;
}

__device__ __forceinline__ int encode_phase(Cx<double> z) {
    int t = (int)rint((128.0 * atan2(z.im, z.re)) / kPiD);
    if (t >= 128) t -= 256;
    if (t < -128) t += 256;
    return t;
}

// ordered bit pattern of a non-negative double: integer order = numeric order
__device__ __forceinline__ unsigned long long dbits(double x) { return (unsigned long long)__double_as_longlong(x); }

__device__ __forceinline__ void range_update(double a, double& lo, double& hi) {
    if (a > 0.0 && a < 1.0 - kOneTol) {
        lo = a < lo ? a : lo;
        hi = a > hi ? a : hi;
    }
}

__device__ __forceinline__ void range_flush(double lo, double hi, unsigned long long* acc) {
    // wave-level min/max, then one atomic pair per wave
    for (int off = 32; off > 0; off >>= 1) {
        const double l2 = __shfl_xor(lo, off, 64), h2 = __shfl_xor(hi, off, 64);
        lo = l2 < lo ? l2 : lo;
        hi = h2 > hi ? h2 : hi;
    }
    if ((threadIdx.x & 63) == 0 && hi > 0.0) {
        atomicMin(&acc[0], dbits(lo));
        atomicMax(&acc[1], dbits(hi));
    }
}

// ------------------------------------------------ fast codec paths --
//
// The codes are defined by the FP64 formulas above.  The kernels below take
// them through cheaper routes that give the same code:
// * decode reads r(b0) from a per-block LDS table holding the decode
//   formula's value for each of the 256 codes, and cos/sin of the phase
//   code from LDS;
// * the range is reduced over x = re^2 + im^2: the correctly rounded square
//   root is monotone, so min/max of sqrt(x) are sqrt of min/max of x, and
//   sqrt(x) < 1 - kOneTol holds exactly when x < c_x_one, the least double
//   whose square root reaches 1 - kOneTol (found on the host);
// * an estimate of the code's real-valued argument (the modulus ratio from
//   a refined hardware reciprocal square root, the phase from an FP32
//   atan2 of the power-of-two-scaled amplitude) decides the code when it
//   lies farther from a rounding boundary than a bound on the estimate's
//   error; otherwise the FP64 formula runs.

__constant__ double c_x_one;

// r(b0) per modulus code, (cos, sin) per phase code as one 16-byte entry
// (one LDS read each)
struct DecodeTab {
    double r[256];
    double2 cs[256];
};

// every thread of the block calls this (it ends with a barrier)
__device__ __forceinline__ void decode_tab_fill(DecodeTab& T, Range g) {
    for (int k = (int)threadIdx.x; k < 256; k += (int)blockDim.x) {
        const int c0 = k - 128;
        T.r[k] = c0 == -128 ? 0.0 : c0 == 127 ? 1.0 : ((double)(c0 + 127) * (g.r1 - g.r0)) / 253.0 + g.r0;
        T.cs[k] = make_double2(c_cos[k], c_sin[k]);
    }
    __syncthreads();
}

__device__ __forceinline__ Cx<double> decode_tab(const DecodeTab& T, int c0, int c1) {
    const double r = T.r[c0 + 128];
    const double2 cs = T.cs[c1 + 128];
    return {r * cs.x, r * cs.y};
}

__device__ __forceinline__ double modulus2(Cx<double> z) { return z.re * z.re + z.im * z.im; }

__device__ __forceinline__ void range_update_x(double x, double& lo, double& hi) {
    if (x > 0.0 && x < c_x_one) {
        lo = x < lo ? x : lo;
        hi = x > hi ? x : hi;
    }
}

__device__ __forceinline__ void range_flush_x(double lo, double hi, unsigned long long* acc) {
    for (int off = 32; off > 0; off >>= 1) {
        const double l2 = __shfl_xor(lo, off, 64), h2 = __shfl_xor(hi, off, 64);
        lo = l2 < lo ? l2 : lo;
        hi = h2 > hi ? h2 : hi;
    }
    if ((threadIdx.x & 63) == 0 && hi > 0.0) {
        atomicMin(&acc[0], dbits(sqrt(lo)));
        atomicMax(&acc[1], dbits(sqrt(hi)));
    }
}

struct EncParams {
    double r0, r1;
    double inv;  // 253 / (r1 - r0)
};

__device__ __forceinline__ EncParams enc_params(Range g) {
    return {g.r0, g.r1, g.r1 > g.r0 ? 253.0 / (g.r1 - g.r0) : 0.0};
}

// The FP64 formulas out of line: they run only for the few amplitudes the
// estimates cannot decide, and inlining them into every register slot of
// an unrolled tile would multiply the kernel's code size.
__device__ __attribute__((noinline)) int encode_mod_slow(double x, double r0, double r1) {
    return encode_mod(sqrt(x), Range{r0, r1});
}

__device__ __attribute__((noinline)) int encode_phase_slow(double re, double im) {
    return encode_phase(Cx<double>{re, im});
}

// b0 of an amplitude with x = re^2 + im^2: encode_mod(sqrt(x)).
__device__ __forceinline__ int encode_mod_x(double x, const EncParams& p) {
    if (x == 0.0) return -128;
    if (x >= c_x_one) return 127;
    if (p.r1 == p.r0) return -127;
    if (x >= 0x1p-900) {
        // v_rsq_f64 (relative error far below 2^-20) and one Goldschmidt
        // step: a within 2^-40 relative of sqrt(x)
        const double y = __builtin_amdgcn_rsq(x);
        double a = x * y;
        const double h = 0.5 * y;
        a = fma(a, fma(-h, a, 0.5), a);
        // the FP64 formula's argument differs from q by less than
        // inv * a * 2^-43 + 2^-42
        const double q = (a - p.r0) * p.inv;
        const double f = q - floor(q);
        if (fabs(f - 0.5) > p.inv * a * 0x1p-36 + 1e-9) {
            double v = -127.0 + rint(q);
            v = v < -127.0 ? -127.0 : v;
            v = v > 126.0 ? 126.0 : v;
            return (int)v;
        }
    }
    return encode_mod_slow(x, p.r0, p.r1);
}

// b1 of a non-zero amplitude: encode_phase(z).  The phase in code units,
// t = 128 atan2(im, re) / pi, is estimated in FP32 from the octant: with
// r = min(|x|, |y|) / max(|x|, |y|) in [0, 1], atan(r) 128/pi is the odd
// polynomial below (coefficients fitted to it on [0, 1]; largest error
// 6.8e-5 code units), mirrored about 32 code units when |y| > |x|, then
// about 64 for x < 0 and negated for y < 0.  Error of t: the polynomial,
// the FP32 conversions (2^-24 relative each), the reciprocal and product
// (2^-23), Horner's rounding (41 * 6 * 2^-24) and the mirroring (2^-17
// each): below 1.2e-4 code units.  The estimate decides the code when its
// fractional part is farther than 1e-3 from 1/2; otherwise, and for
// amplitudes below 2^-100 (FP32 would lose them), the FP64 formula runs.
constexpr float kAtanC[6] = {40.74273725441187f, -13.552273111704942f, 7.88554333160211f,
                             -4.743638602227283f, 2.145042417363906f, -0.477479010596689f};

__device__ __forceinline__ int encode_phase_fast(Cx<double> z) {
    if (!(fmax(fabs(z.re), fabs(z.im)) >= 0x1p-100)) return encode_phase_slow(z.re, z.im);
    const float xf = (float)z.re, yf = (float)z.im;
    const float ax = fabsf(xf), ay = fabsf(yf);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float r = mn * __builtin_amdgcn_rcpf(mx);
    const float q = r * r;
    float p = kAtanC[5];
    p = p * q + kAtanC[4];
    p = p * q + kAtanC[3];
    p = p * q + kAtanC[2];
    p = p * q + kAtanC[1];
    p = p * q + kAtanC[0];
    float t = p * r;
    t = ay > ax ? 64.0f - t : t;
    t = xf < 0.0f ? 128.0f - t : t;
    t = yf < 0.0f ? -t : t;
    const float fl = floorf(t);
    const float f = t - fl;
    if (fabsf(f - 0.5f) > 1e-3f) {
        int c = (int)fl + (f > 0.5f ? 1 : 0);
        if (c >= 128) c -= 256;
        if (c < -128) c += 256;
        return c;
    }
    return encode_phase_slow(z.re, z.im);
}

struct CpGate {
    int32_t kind;     // OP_DENSE1, OP_DENSE2, OP_DIAG
    int32_t nsel;
    int32_t t0, t1;
    uint64_t cmask;
    Cx<double> m[16];
};

// Group of the gate: pairs (DENSE1), quads (DENSE2) or single amplitudes
// (DIAG), over the whole state (controls are tested per group, so that
// amplitudes outside the controlled subspace are decoded, counted in the
// range and re-encoded like all others).
template <int KIND>
__global__ __launch_bounds__(kBlock) void k_cp_gate(int8_t* __restrict__ b0, int8_t* __restrict__ b1, uint64_t ngroups,
                                                     Ins ins, uint64_t hbit, uint64_t lbit, CpGate g,
                                                     const double* __restrict__ rng_old,
                                                     const double* __restrict__ rng_new,
                                                     unsigned long long* __restrict__ acc, int apply) {
    constexpr int A = KIND == OP_DENSE2 ? 4 : KIND == OP_DENSE1 ? 2 : 1;
    const Range ro{rng_old[0], rng_old[1]};
    Range rn = ro;
    if (apply) rn = Range{rng_new[0], rng_new[1]};
    const EncParams ep = enc_params(rn);
    __shared__ DecodeTab tab;
    decode_tab_fill(tab, ro);
    double lo = 2.0, hi = 0.0;
    for (uint64_t gi = (uint64_t)blockIdx.x * kBlock + threadIdx.x; gi < ngroups;
         gi += (uint64_t)gridDim.x * kBlock) {
        const uint64_t i = expand(gi, ins);
        uint64_t idx[A];
        if constexpr (A == 1) {
            idx[0] = i;
        } else if constexpr (A == 2) {
            idx[0] = i;
            idx[1] = i | lbit;
        } else {
            idx[0] = i;
            idx[1] = i | lbit;
            idx[2] = i | hbit;
            idx[3] = i | hbit | lbit;
        }
        Cx<double> z[A], w[A];
#pragma unroll
        for (int c = 0; c < A; ++c) z[c] = decode_tab(tab, b0[idx[c]], b1[idx[c]]);
        const bool on = (i & g.cmask) == g.cmask;
        if constexpr (KIND == OP_DIAG) {
            int sel = 0;
            if (g.nsel >= 1) sel = (int)((i >> g.t0) & 1);
            if (g.nsel == 2) sel = 2 * sel + (int)((i >> g.t1) & 1);
            w[0] = csel(on, cmul(g.m[sel], z[0]), z[0]);
        } else {
#pragma unroll
            for (int r = 0; r < A; ++r) {
                // left-to-right sum of row r, as sum_c m[r][c] z[c]
                Cx<double> s = cmul(g.m[A * r], z[0]);
#pragma unroll
                for (int c = 1; c < A; ++c) s = cadd(s, cmul(g.m[A * r + c], z[c]));
                w[r] = csel(on, s, z[r]);
            }
        }
        if (!apply) {
#pragma unroll
            for (int c = 0; c < A; ++c) range_update_x(modulus2(w[c]), lo, hi);
        } else {
#pragma unroll
            for (int c = 0; c < A; ++c) {
                const int c0 = encode_mod_x(modulus2(w[c]), ep);
                b0[idx[c]] = (int8_t)c0;
                b1[idx[c]] = (int8_t)(c0 == -128 ? 0 : encode_phase_fast(w[c]));
            }
        }
    }
    if (!apply) range_flush_x(lo, hi, acc);
}

__global__ void k_cp_resolve(unsigned long long* acc, const double* rng_old, double* rng_new) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (acc[1] == 0ull) {
        rng_new[0] = rng_old[0];
        rng_new[1] = rng_old[1];
    } else {
        rng_new[0] = __longlong_as_double((long long)acc[0]);
        rng_new[1] = __longlong_as_double((long long)acc[1]);
    }
    acc[0] = ~0ull;
    acc[1] = 0ull;
}

__global__ void k_cp_acc_reset(unsigned long long* acc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        acc[0] = ~0ull;
        acc[1] = 0ull;
    }
}

// Modulus-preserving diagonal gate whose phase shift sits on a rounding
// tie: decode, rotate and re-encode the phase of each touched amplitude
// (the range is kept, so the modulus code of a decoded-and-rotated
// amplitude encodes back to itself).
__global__ __launch_bounds__(kBlock) void k_cp_phase(const int8_t* __restrict__ b0, int8_t* __restrict__ b1,
                                                      uint64_t ngroups, Ins ins, CpGate g,
                                                      const double* __restrict__ rng) {
    const Range r{rng[0], rng[1]};
    for (uint64_t gi = (uint64_t)blockIdx.x * kBlock + threadIdx.x; gi < ngroups;
         gi += (uint64_t)gridDim.x * kBlock) {
        const uint64_t i = expand(gi, ins);
        const int c0 = b0[i];
        if (c0 == -128) continue;
        int sel = 0;
        if (g.nsel >= 1) sel = (int)((i >> g.t0) & 1);
        if (g.nsel == 2) sel = 2 * sel + (int)((i >> g.t1) & 1);
        const Cx<double> w = cmul(g.m[sel], decode(c0, b1[i], r));
        b1[i] = (int8_t)encode_phase(w);
    }
}

__global__ __launch_bounds__(kBlock) void k_cp_init(int8_t* __restrict__ b0, int8_t* __restrict__ b1, uint64_t dim,
                                                     int mode, uint64_t basis, double* rng, double uni) {
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < dim; i += (uint64_t)gridDim.x * kBlock) {
        if (mode == JQ_INIT_UNIFORM) {
            b0[i] = -127;
        } else {
            b0[i] = i == basis ? (int8_t)127 : (int8_t)-128;
        }
        b1[i] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        rng[0] = mode == JQ_INIT_UNIFORM ? uni : 0.0;
        rng[1] = mode == JQ_INIT_UNIFORM ? uni : 0.0;
    }
}

__global__ __launch_bounds__(kBlock) void k_cp_decode(const int8_t* __restrict__ b0, const int8_t* __restrict__ b1,
                                                       uint64_t first, uint64_t count, const double* rng,
                                                       double2* __restrict__ dst) {
    const Range r{rng[0], rng[1]};
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (uint64_t)gridDim.x * kBlock) {
        const Cx<double> z = decode(b0[first + i], b1[first + i], r);
        dst[i] = make_double2(z.re, z.im);
    }
}

// Encode a full complex128 state: range pass then encode pass.
__global__ __launch_bounds__(kBlock) void k_cp_range_of(const double2* __restrict__ src, uint64_t dim,
                                                         unsigned long long* acc) {
    double lo = 2.0, hi = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < dim; i += (uint64_t)gridDim.x * kBlock) {
        const double2 v = src[i];
        range_update(modulus(Cx<double>{v.x, v.y}), lo, hi);
    }
    range_flush(lo, hi, acc);
}

__global__ __launch_bounds__(kBlock) void k_cp_encode(const double2* __restrict__ src, uint64_t dim,
                                                       const double* rng, int8_t* __restrict__ b0,
                                                       int8_t* __restrict__ b1) {
    const Range r{rng[0], rng[1]};
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < dim; i += (uint64_t)gridDim.x * kBlock) {
        const double2 v = src[i];
        const Cx<double> z{v.x, v.y};
        const int c0 = encode_mod(modulus(z), r);
        b0[i] = (int8_t)c0;
        b1[i] = (int8_t)(c0 == -128 ? 0 : encode_phase(z));
    }
}

__global__ void k_cp_scale_range(double* rng, double f) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        rng[0] *= f;
        rng[1] *= f;
    }
}

// Reduction loader: decodes through the per-block LDS tables; the modulus
// comes from b0 alone.
struct LoaderCP {
    const int8_t* b0;
    const int8_t* b1;
    const double* rng;
    const DecodeTab* tab;
    // every thread of the block calls this (it ends with a barrier)
    __device__ void prepare() {
        __shared__ DecodeTab t;
        decode_tab_fill(t, Range{rng[0], rng[1]});
        tab = &t;
    }
    __device__ __forceinline__ Cx<double> amp(uint64_t i) const { return decode_tab(*tab, b0[i], b1[i]); }
    __device__ __forceinline__ double modulus2(uint64_t i) const {
        const double m = tab->r[b0[i] + 128];
        return m * m;
    }
    // sum over the 16 amplitudes i..i+15 (i a multiple of 16), in order
    template <int W>
    __device__ __forceinline__ double modulus2_w(uint64_t i) const {
        static_assert(W == 16, "16 codes per access");
        const uint4 x = *reinterpret_cast<const uint4*>(b0 + i);
        const uint32_t w[4] = {x.x, x.y, x.z, x.w};
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const double m = tab->r[(int)(int8_t)(w[u >> 2] >> (8 * (u & 3))) + 128];
            s += m * m;
        }
        return s;
    }
};

// ------------------------------------------------------ chunked forms --
//
// When every fixed index bit of a gate (target, controls) lies at position
// log2(W) or above, W consecutive codes of a plane belong to W consecutive
// groups, so a thread moves them with one 4- or 16-byte access.

template <int W>
struct Codes {
    int8_t v[W];
};

template <int W>
__device__ __forceinline__ Codes<W> ldc(const int8_t* p, uint64_t i) {
    Codes<W> c;
    if constexpr (W == 16) {
        const uint4 x = *reinterpret_cast<const uint4*>(p + i);
        __builtin_memcpy(c.v, &x, 16);
    } else if constexpr (W == 4) {
        const uint32_t x = *reinterpret_cast<const uint32_t*>(p + i);
        __builtin_memcpy(c.v, &x, 4);
    } else {
        c.v[0] = p[i];
    }
    return c;
}

template <int W>
__device__ __forceinline__ void stc(int8_t* p, uint64_t i, const Codes<W>& c) {
    if constexpr (W == 16) {
        uint4 x;
        __builtin_memcpy(&x, c.v, 16);
        *reinterpret_cast<uint4*>(p + i) = x;
    } else if constexpr (W == 4) {
        uint32_t x;
        __builtin_memcpy(&x, c.v, 4);
        *reinterpret_cast<uint32_t*>(p + i) = x;
    } else {
        p[i] = c.v[0];
    }
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_cp_permx_w(int8_t* __restrict__ b0, int8_t* __restrict__ b1,
                                                        uint64_t nchunks, Ins ins, uint64_t tbit) {
    for (uint64_t c = (uint64_t)blockIdx.x * kBlock + threadIdx.x; c < nchunks; c += (uint64_t)gridDim.x * kBlock) {
        const uint64_t i = expand(c * W, ins), j = i | tbit;
        const Codes<W> x0 = ldc<W>(b0, i), x1 = ldc<W>(b1, i), y0 = ldc<W>(b0, j), y1 = ldc<W>(b1, j);
        stc<W>(b0, i, y0);
        stc<W>(b1, i, y1);
        stc<W>(b0, j, x0);
        stc<W>(b1, j, x1);
    }
}

struct Shift {
    double d[4];  // phase of each diagonal entry in code units, 128 arg(d)/pi
};

// Modulus-preserving diagonal gate: the phase code moves by the entry's
// phase in code units, rounded half to even and wrapped to [-128, 128).
// This is the code the decode-multiply-encode step produces, except where
// b1 + shift lies within a few ulps of a half-integer (a rounding tie, where
// either neighbour is a correct rounding).  Zero amplitudes keep code 0.
template <int W>
__global__ __launch_bounds__(kBlock) void k_cp_shift_w(const int8_t* __restrict__ b0, int8_t* __restrict__ b1,
                                                        uint64_t nchunks, Ins ins, int nsel, int s0, int s1,
                                                        Shift sh) {
    for (uint64_t c = (uint64_t)blockIdx.x * kBlock + threadIdx.x; c < nchunks; c += (uint64_t)gridDim.x * kBlock) {
        const uint64_t i = expand(c * W, ins);
        const Codes<W> m = ldc<W>(b0, i);
        Codes<W> p = ldc<W>(b1, i);
#pragma unroll
        for (int u = 0; u < W; ++u) {
            const uint64_t idx = i + u;
            int sel = 0;
            if (nsel >= 1) sel = (int)((idx >> s0) & 1);
            if (nsel == 2) sel = 2 * sel + (int)((idx >> s1) & 1);
            double dv = sh.d[0];
            dv = sel == 1 ? sh.d[1] : dv;
            dv = sel == 2 ? sh.d[2] : dv;
            dv = sel == 3 ? sh.d[3] : dv;
            int t = (int)rint((double)p.v[u] + dv);
            t = ((t + 128) & 255) - 128;
            p.v[u] = m.v[u] == -128 ? (int8_t)0 : (int8_t)t;
        }
        stc<W>(b1, i, p);
    }
}

// W codes of one plane packed into 32-bit words (byte u of the chunk is
// bits 8(u%4).. of word u/4), written with one 4- or 16-byte store.
template <int W>
struct Pack {
    uint32_t w[W >= 4 ? W / 4 : 1] = {};
    __device__ __forceinline__ void set(int u, int code) { w[u >> 2] |= (uint32_t)(uint8_t)code << (8 * (u & 3)); }
};

template <int W>
__device__ __forceinline__ void stp(int8_t* p, uint64_t i, const Pack<W>& c) {
    if constexpr (W == 16) {
        *reinterpret_cast<uint4*>(p + i) = make_uint4(c.w[0], c.w[1], c.w[2], c.w[3]);
    } else if constexpr (W == 4) {
        *reinterpret_cast<uint32_t*>(p + i) = c.w[0];
    } else {
        p[i] = (int8_t)(c.w[0] & 0xff);
    }
}

// Dense single-qubit gate over all pairs (target bit t, W <= 2^t): range
// mode (APPLY = 0) reduces the new moduli, apply mode encodes them with the
// resolved range, as in k_cp_gate.
template <int W, int APPLY>
__global__ __launch_bounds__(kBlock) void k_cp_dense1_w(int8_t* __restrict__ b0, int8_t* __restrict__ b1,
                                                         uint64_t nchunks, Ins ins, uint64_t tbit, CpGate g,
                                                         const double* __restrict__ rng_old,
                                                         const double* __restrict__ rng_new,
                                                         unsigned long long* __restrict__ acc) {
    const Range ro{rng_old[0], rng_old[1]};
    Range rn = ro;
    if (APPLY) rn = Range{rng_new[0], rng_new[1]};
    const EncParams ep = enc_params(rn);
    __shared__ DecodeTab tab;
    decode_tab_fill(tab, ro);
    double lo = 2.0, hi = 0.0;
    for (uint64_t c = (uint64_t)blockIdx.x * kBlock + threadIdx.x; c < nchunks; c += (uint64_t)gridDim.x * kBlock) {
        const uint64_t i = expand(c * W, ins), j = i | tbit;
        const Codes<W> x0 = ldc<W>(b0, i), x1 = ldc<W>(b1, i), y0 = ldc<W>(b0, j), y1 = ldc<W>(b1, j);
        Pack<W> px0, px1, py0, py1;
#pragma unroll
        for (int u = 0; u < W; ++u) {
            const Cx<double> z0 = decode_tab(tab, x0.v[u], x1.v[u]), z1 = decode_tab(tab, y0.v[u], y1.v[u]);
            const bool on = ((i + u) & g.cmask) == g.cmask;
            Cx<double> w0 = cadd(cmul(g.m[0], z0), cmul(g.m[1], z1));
            Cx<double> w1 = cadd(cmul(g.m[2], z0), cmul(g.m[3], z1));
            w0 = csel(on, w0, z0);
            w1 = csel(on, w1, z1);
            if constexpr (!APPLY) {
                range_update_x(modulus2(w0), lo, hi);
                range_update_x(modulus2(w1), lo, hi);
            } else {
                const int c0 = encode_mod_x(modulus2(w0), ep), c1 = encode_mod_x(modulus2(w1), ep);
                px0.set(u, c0);
                px1.set(u, c0 == -128 ? 0 : encode_phase_fast(w0));
                py0.set(u, c1);
                py1.set(u, c1 == -128 ? 0 : encode_phase_fast(w1));
            }
        }
        if constexpr (APPLY) {
            stp<W>(b0, i, px0);
            stp<W>(b1, i, px1);
            stp<W>(b0, j, py0);
            stp<W>(b1, j, py1);
        }
    }
    if constexpr (!APPLY) range_flush_x(lo, hi, acc);
}

// ------------------------------------------------- fused block pass --
//
// Per-block quantisation: the gates of one fused pass run between a single
// decode and a single encode.  A wavefront takes a tile of 2^(6+K)
// amplitudes (lane bits 0..F-1 are index bits 0..F-1, so each plane is read
// in runs of 2^F bytes), decodes it into FP64 registers with the current
// range and applies the pass's ops as the state-vector pass does.  Range
// mode then reduces min/max of the new moduli; apply mode encodes with the
// resolved range and stores both codes.  Waves loop over tiles so that the
// range reduction issues one atomic pair per wave.
template <int K, int F, int APPLY>
__global__ __launch_bounds__(kBlock) void k_cp_fused(int8_t* __restrict__ b0, int8_t* __restrict__ b1, FPass P,
                                                      const FOp* __restrict__ ops, uint64_t ntiles,
                                                      const double* __restrict__ rng_old,
                                                      const double* __restrict__ rng_new,
                                                      unsigned long long* __restrict__ acc) {
    constexpr int S = 1 << K;
    const int lane = threadIdx.x & 63;
    const uint64_t wpb = blockDim.x >> 6;
    const uint64_t wave0 = (uint64_t)blockIdx.x * wpb + (uint64_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * wpb;
    uint64_t lane_off = (uint64_t)(lane & ((1 << F) - 1));
#pragma unroll
    for (int b = F; b < 6; ++b) lane_off |= (uint64_t)((lane >> b) & 1) << P.lane_q[b];
    uint64_t stride[K];
#pragma unroll
    for (int j = 0; j < K; ++j) stride[j] = 1ull << P.reg_q[j];
    const Range ro{rng_old[0], rng_old[1]};
    Range rn = ro;
    if (APPLY) rn = Range{rng_new[0], rng_new[1]};
    const EncParams ep = enc_params(rn);
    __shared__ DecodeTab tab;
    decode_tab_fill(tab, ro);
    double lo = 2.0, hi = 0.0;
    for (uint64_t w = wave0; w < ntiles; w += nwaves) {
        const uint64_t base = tile_base(P, w, lane_off);
        Cx<double> a[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            uint64_t off = 0;
#pragma unroll
            for (int j = 0; j < K; ++j)
                if (s & (1 << j)) off += stride[j];
            a[s] = decode_tab(tab, b0[base + off], b1[base + off]);
        }
        run_ops<double, K>(a, ops, P.n_ops, base, wave_uniform(tile_base(P, w, 0)), lane);
        // recompute the store addresses instead of keeping 2^K of them live
        uint64_t sbase = base;
        asm volatile("" : "+v"(sbase));
#pragma unroll
        for (int s = 0; s < S; ++s) {
            uint64_t off = 0;
#pragma unroll
            for (int j = 0; j < K; ++j)
                if (s & (1 << j)) off += stride[j];
            JQ_SLOT_FENCE();
            const double x = modulus2(a[s]);
            if (!APPLY) {
                range_update_x(x, lo, hi);
            } else {
                const int c0 = encode_mod_x(x, ep);
                b0[sbase + off] = (int8_t)c0;
                b1[sbase + off] = (int8_t)(c0 == -128 ? 0 : encode_phase_fast(a[s]));
            }
        }
    }
    if (!APPLY) range_flush_x(lo, hi, acc);
}

// SHORBOX in the two-byte code: every amplitude of the state has modulus
// 2^(-n_x/2) or 0, so the range is (a, a) and each non-zero code is -127
// with phase code 0 (the planes have been cleared to zero amplitudes).
__global__ __launch_bounds__(kBlock) void k_cp_shorbox(int8_t* __restrict__ b0, int n_x, uint64_t G, uint64_t y,
                                                        double* rng, double a) {
    const uint64_t nx = 1ull << n_x;
    for (uint64_t x = (uint64_t)blockIdx.x * kBlock + threadIdx.x; x < nx; x += (uint64_t)gridDim.x * kBlock) {
        uint64_t r = 1 % G, b = y % G, e = x;
        while (e) {
            if (e & 1) r = r * b % G;
            b = b * b % G;
            e >>= 1;
        }
        b0[x + (r << n_x)] = -127;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        rng[0] = a;
        rng[1] = a;
    }
}

// ------------------------------------------------ fused code pass --
//
// With per-gate quantisation a permutation swaps code pairs and a
// modulus-preserving phase shift adds an integer to the phase code of each
// touched non-zero amplitude (the per-gate kernels above); both are exact
// on the codes, so a run of them executes as one tile pass over both planes
// without decoding, with the codes they would produce one by one.
//
// Tile: register slot bits 0 and 1 are qubits 0 and 1, lane bits qubits
// 2..7, slot bits 2..K-1 qubits the planner picks.  A lane moves four
// consecutive codes of a plane with one 4-byte access (256-byte runs per
// wave instruction).  Two codes share a 32-bit register: register r holds
// slot 2r in bits 0-15 and slot 2r+1 in bits 16-31, each as b0 in the low
// byte and b1 in the high byte of its half.  A phase shift adds to the high
// byte of a half with a 16-bit add, so the sum is taken mod 256 and never
// reaches b0 or the other half; a pending sum travels with its amplitude
// through later permutations.  Zero amplitudes (b0 = -128) get phase code 0
// at the store, as every stored state has on its zero amplitudes.

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// 16-bit add in each half (no carry between the halves)
__device__ __forceinline__ uint32_t add16x2(uint32_t x, uint32_t y) {
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, x) + __builtin_bit_cast(u16x2, y));
}

// the two halves of x exchanged
__device__ __forceinline__ uint32_t swap_halves(uint32_t x) { return (x << 16) | (x >> 16); }

// permutation of slot bit J >= 1: registers r and r | 2^(J-1) exchange
// (whole registers, or only their high halves when slot bit 0 is a control)
template <int P, int J>
__device__ __forceinline__ void hc_perm_reg(uint32_t (&c)[P], uint32_t rc, bool thr_ok) {
    constexpr int B = 1 << (J - 1);
    if constexpr (B < P) {
        const uint32_t rr = rc >> 1;
        if (rc == 0) {
            // no control in the slots: one condition for the whole thread
#pragma unroll
            for (int r = 0; r < P; ++r) {
                if (r & B) continue;
                const uint32_t x = c[r], y = c[r | B];
                c[r] = thr_ok ? y : x;
                c[r | B] = thr_ok ? x : y;
            }
        } else if (!(rc & 1u)) {
#pragma unroll
            for (int r = 0; r < P; ++r) {
                if (r & B) continue;
                const bool ok = thr_ok && ((uint32_t)r & rr) == rr;
                const uint32_t x = c[r], y = c[r | B];
                c[r] = ok ? y : x;
                c[r | B] = ok ? x : y;
            }
        } else {
            const uint32_t hi = thr_ok ? 0xffff0000u : 0u;
#pragma unroll
            for (int r = 0; r < P; ++r) {
                if (r & B) continue;
                const uint32_t msk = ((uint32_t)r & rr) == rr ? hi : 0u;
                const uint32_t x = c[r], y = c[r | B];
                c[r] = (y & msk) | (x & ~msk);
                c[r | B] = (x & msk) | (y & ~msk);
            }
        }
    }
}

// permutation of slot bit 0: the halves of each register exchange
template <int P>
__device__ __forceinline__ void hc_perm_half(uint32_t (&c)[P], uint32_t rc, bool thr_ok) {
    const uint32_t rr = rc >> 1;
    if (rr == 0) {
#pragma unroll
        for (int r = 0; r < P; ++r) c[r] = thr_ok ? swap_halves(c[r]) : c[r];
        return;
    }
#pragma unroll
    for (int r = 0; r < P; ++r) {
        const bool ok = thr_ok && ((uint32_t)r & rr) == rr;
        c[r] = ok ? swap_halves(c[r]) : c[r];
    }
}

// Each case ends in its own empty asm statement so that the compiler cannot
// merge the cases into one body with a run-time register index (which would
// move the register tile to scratch memory).
template <int P>
__device__ __forceinline__ void hc_perm_reg_dispatch(uint32_t (&c)[P], int j, uint32_t rc, bool thr_ok) {
    switch (j) {
        case 0: hc_perm_half<P>(c, rc, thr_ok); asm volatile("; code slot 0"); break;
        case 1: hc_perm_reg<P, 1>(c, rc, thr_ok); asm volatile("; code slot 1"); break;
        case 2: hc_perm_reg<P, 2>(c, rc, thr_ok); asm volatile("; code slot 2"); break;
        case 3: hc_perm_reg<P, 3>(c, rc, thr_ok); asm volatile("; code slot 3"); break;
        case 4: hc_perm_reg<P, 4>(c, rc, thr_ok); asm volatile("; code slot 4"); break;
        case 5: hc_perm_reg<P, 5>(c, rc, thr_ok); asm volatile("; code slot 5"); break;
        case 6: hc_perm_reg<P, 6>(c, rc, thr_ok); asm volatile("; code slot 6"); break;
        default: break;
    }
}

// permutation of lane bit b: codes move between lanes 2^b apart (whole
// registers, or only the high halves when slot bit 0 is a control)
template <int P>
__device__ __forceinline__ void hc_perm_lane(uint32_t (&c)[P], int b, uint32_t rc, bool thr_ok) {
    const int mask = 1 << b;
    const uint32_t rr = rc >> 1;
    if (rc == 0) {
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const uint32_t partner = (uint32_t)__shfl_xor((int)c[r], mask, 64);
            c[r] = thr_ok ? partner : c[r];
            // a few exchanges in flight at a time, not one result register per slot
            if ((r & 7) == 7) JQ_SLOT_FENCE();
        }
        return;
    }
    const uint32_t keep = (rc & 1u) ? 0x0000ffffu : 0u;
#pragma unroll
    for (int r = 0; r < P; ++r) {
        const uint32_t partner = (uint32_t)__shfl_xor((int)c[r], mask, 64);
        const bool ok = thr_ok && ((uint32_t)r & rr) == rr;
        c[r] = ok ? (partner & ~keep) | (c[r] & keep) : c[r];
        if ((r & 7) == 7) JQ_SLOT_FENCE();
    }
}

// registers whose bit J-1 is set get y added (a selector in slot J >= 1)
template <int P, int J>
__device__ __forceinline__ void hc_add_bit(uint32_t (&c)[P], uint32_t y) {
    constexpr int B = 1 << (J - 1);
    if constexpr (B < P) {
#pragma unroll
        for (int r = 0; r < P; ++r)
            if (r & B) c[r] = add16x2(c[r], y);
    }
}

// Slot s gets e (phase-code units in bits 8..15) where (s & m) == m.
template <int P>
__device__ __forceinline__ void hc_add_mask(uint32_t (&c)[P], uint32_t m, uint32_t e) {
    const uint32_t both = e | (e << 16), hi = e << 16;
    // the halves to add to: both, or only the high one when slot bit 0 is
    // in the mask; the registers by the mask's other bits
    const uint32_t y = (m & 1u) ? hi : both;
    const uint32_t rm = m >> 1;
    if (rm == 0) {
#pragma unroll
        for (int r = 0; r < P; ++r) c[r] = add16x2(c[r], y);
        return;
    }
    switch (rm) {
        case 1u: hc_add_bit<P, 1>(c, y); asm volatile("; add slot 1"); return;
        case 2u: hc_add_bit<P, 2>(c, y); asm volatile("; add slot 2"); return;
        case 4u: hc_add_bit<P, 3>(c, y); asm volatile("; add slot 3"); return;
        case 8u: hc_add_bit<P, 4>(c, y); asm volatile("; add slot 4"); return;
        case 16u: hc_add_bit<P, 5>(c, y); asm volatile("; add slot 5"); return;
        case 32u: hc_add_bit<P, 6>(c, y); asm volatile("; add slot 6"); return;
        default: break;
    }
#pragma unroll
    for (int r = 0; r < P; ++r) {
        c[r] = add16x2(c[r], ((uint32_t)r & rm) == rm ? y : 0u);
        if ((r & 7) == 7) JQ_SLOT_FENCE();
    }
}

// A shift arrives as up to four masked adds of one value per thread (its
// selector and control bits outside the slots decide the value, those in
// the slots the mask).  A term that reaches every slot of a thread goes
// into the thread's pending sum acc instead (added to all its slots before
// the next cross-lane exchange and at the store): register permutations
// leave a value common to all slots of the thread where it is, and adds
// commute.
template <int P>
__device__ __forceinline__ void hc_shift(uint32_t (&c)[P], uint32_t& acc, const FOp* op, uint64_t base) {
    // the op's fields are wave-uniform: read them into scalar registers
    // before any per-thread choice
    const int nt = __builtin_amdgcn_readfirstlane(op->cs_n);
    for (int t = 0; t < nt; ++t) {
        const uint64_t tm = op->cs_thr[t];
        const uint32_t m = (uint32_t)__builtin_amdgcn_readfirstlane((int)op->cs_reg[t]);
        const uint32_t add = (uint32_t)__builtin_amdgcn_readfirstlane((int)op->cs_add[t]);
        const uint32_t e = (base & tm) == tm ? add : 0u;
        if (m == 0)
            acc += e;
        else
            hc_add_mask<P>(c, m, e);
    }
}

template <int P>
__device__ __forceinline__ void hc_flush(uint32_t (&c)[P], uint32_t& acc) {
    const uint32_t y = (acc & 0xff00u) * 0x10001u;
#pragma unroll
    for (int r = 0; r < P; ++r) c[r] = add16x2(c[r], y);
    acc = 0;
}

// Waves loop over the tiles (a launch holds at most 2^32 threads).
template <int K>
__global__ __launch_bounds__(kBlock) void k_cp_codes(int8_t* __restrict__ b0, int8_t* __restrict__ b1, FPass P,
                                                      const FOp* __restrict__ ops, uint64_t ntiles) {
    constexpr int NP = 1 << (K - 1);  // registers, two codes each
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t wpb = blockDim.x >> 6;
    const uint64_t wave0 = (uint64_t)blockIdx.x * wpb + (uint64_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * wpb;
    // a lane's codes start at byte 4 lane of the tile's (wave-uniform) base,
    // and the slots' offsets are uniform too, so every access is a scalar
    // pointer plus the lane's 32-bit byte offset
    const uint32_t lane_b = lane << 2;
    uint64_t stride[K];
#pragma unroll
    for (int j = 0; j < K; ++j) stride[j] = 1ull << P.reg_q[j];
    for (uint64_t w = wave0; w < ntiles; w += nwaves) {
    const uint64_t ubase = wave_uniform(tile_base(P, w, 0));
    const uint64_t base = ubase | (uint64_t)lane_b;
    uint32_t c[NP];
#pragma unroll
    for (int sh = 0; sh < (1 << K); sh += 4) {
        uint64_t off = ubase;
#pragma unroll
        for (int j = 2; j < K; ++j)
            if (sh & (1 << j)) off += stride[j];
        // every code is read and written once per pass: non-temporal (measured
        // 14.60 -> 13.98 ms per pass at N=34, 102.0 -> 100.8 ms at N=37)
        const uint32_t x0 = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(b0 + off + lane_b));
        const uint32_t x1 = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(b1 + off + lane_b));
        // bytes (b0, b1) of slots sh, sh+1 and of sh+2, sh+3
        c[sh / 2] = __builtin_amdgcn_perm(x1, x0, 0x05010400u);
        c[sh / 2 + 1] = __builtin_amdgcn_perm(x1, x0, 0x07030602u);
    }
    uint32_t acc = 0;
    bool pending = false;  // wave-uniform: some term went into acc
    for (int k = 0; k < P.n_ops; ++k) {
        const FOp* op = ops + k;
        const bool thr_ok = (base & op->thr_ctrl) == op->thr_ctrl;
        switch (op->kind) {
            case F_PERM_REG: hc_perm_reg_dispatch<NP>(c, op->slot, op->reg_ctrl, thr_ok); break;
            case F_PERM_LANE:
                if (pending) hc_flush<NP>(c, acc);
                pending = false;
                hc_perm_lane<NP>(c, op->slot, op->reg_ctrl, thr_ok);
                break;
            case F_CSHIFT:
                hc_shift<NP>(c, acc, op, base);
                pending = true;
                break;
            default: break;
        }
    }
    if (pending) hc_flush<NP>(c, acc);
    // the store addresses are recomputed from a fresh copy of the base,
    // not kept live in registers across the ops
    uint64_t sbase = ubase;
    asm volatile("" : "+s"(sbase));
#pragma unroll
    for (int sh = 0; sh < (1 << K); sh += 4) {
        uint64_t off = sbase;
#pragma unroll
        for (int j = 2; j < K; ++j)
            if (sh & (1 << j)) off += stride[j];
        const uint32_t lo = c[sh / 2], hi = c[sh / 2 + 1];
        const uint32_t y0 = __builtin_amdgcn_perm(hi, lo, 0x06040200u);
        uint32_t y1 = __builtin_amdgcn_perm(hi, lo, 0x07050301u);
        // bytes of y0 equal to 0x80 (zero amplitudes): exact per-byte test
        const uint32_t t = y0 ^ 0x80808080u;
        const uint32_t z = ~(((t & 0x7f7f7f7fu) + 0x7f7f7f7fu) | t) & 0x80808080u;
        y1 &= ~(z | (z - (z >> 7)));
        __builtin_nontemporal_store(y0, reinterpret_cast<uint32_t*>(b0 + off + lane_b));
        __builtin_nontemporal_store(y1, reinterpret_cast<uint32_t*>(b1 + off + lane_b));
    }
    }
}

// ------------------------------------------------------------ launchers --

namespace {

std::once_flag g_lut_once[64];

void ensure_lut() {
    int dev = 0;
    JQ_HIP(hipGetDevice(&dev));
    std::call_once(g_lut_once[dev & 63], [] {
        double c[256], s[256];
        for (int k = -128; k < 128; ++k) {
            const double th = (kPiD * (double)k) / 128.0;
            c[k + 128] = std::cos(th);
            s[k + 128] = std::sin(th);
        }
        JQ_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_cos), c, sizeof(c)));
        JQ_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_sin), s, sizeof(s)));
        // least x with sqrt(x) >= 1 - kOneTol (sqrt correctly rounded)
        const double T = 1.0 - kOneTol;
        double x = T * T;
        while (std::sqrt(x) >= T) x = std::nextafter(x, 0.0);
        while (std::sqrt(x) < T) x = std::nextafter(x, 2.0);
        JQ_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_x_one), &x, sizeof(x)));
    });
}

unsigned persistent_blocks(uint64_t items) {
    uint64_t b = (items + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    return (unsigned)(b < 16384 ? b : 16384);
}

// widest chunk (16, 4 or 1 codes) whose index bits hold no fixed bit and
// that fits in the ng groups
int chunk_width(uint64_t fixed_bits, uint64_t ng) {
    const int low = fixed_bits ? __builtin_ctzll(fixed_bits) : 64;
    int w = low >= 4 ? 16 : low >= 2 ? 4 : 1;
    while ((uint64_t)w > ng) w /= 4;
    return w < 1 ? 1 : w;
}

CpGate to_cp(const GateOp& op) {
    CpGate g{};
    g.kind = op.kind;
    g.nsel = op.nsel;
    g.t0 = op.t0 < 0 ? 0 : op.t0;
    g.t1 = op.t1 < 0 ? 0 : op.t1;
    g.cmask = op.cmask;
    for (int i = 0; i < 16; ++i) g.m[i] = Cx<double>{op.m[i].re, op.m[i].im};
    return g;
}

}  // namespace

void cp_init(const CompactBufs& b, int n, int mode, uint64_t basis, hipStream_t st) {
    ensure_lut();
    const uint64_t dim = 1ull << n;
    const double uni = uniform_amplitude(n);
    hipLaunchKernelGGL(k_cp_init, dim3(persistent_blocks(dim)), dim3(kBlock), 0, st, b.codes, b.codes + dim, dim, mode,
                       basis, b.range, uni);
    hipLaunchKernelGGL(k_cp_acc_reset, dim3(1), dim3(64), 0, st, (unsigned long long*)b.acc);
    JQ_HIP(hipGetLastError());
}

void cp_shorbox(const CompactBufs& b, int n, int n_x, uint64_t G, uint64_t y, hipStream_t st) {
    cp_init(b, n, JQ_INIT_BASIS, ~0ull, st);  // all codes -128 (zero), range (0, 0)
    const uint64_t nx = 1ull << n_x;
    hipLaunchKernelGGL(k_cp_shorbox, dim3(persistent_blocks(nx)), dim3(kBlock), 0, st, b.codes, n_x, G, y, b.range,
                       uniform_amplitude(n_x));
    JQ_HIP(hipGetLastError());
}

void cp_apply_op(const CompactBufs& b, int n, const GateOp& op, hipStream_t st) {
    ensure_lut();
    const uint64_t dim = 1ull << n;
    int8_t* b0 = b.codes;
    int8_t* b1 = b.codes + dim;
    unsigned long long* acc = (unsigned long long*)b.acc;
    if (op.kind == OP_PERMX) {
        const uint64_t tb = 1ull << op.t0;
        const uint64_t fixed = op.cmask | tb;
        const uint64_t ng = 1ull << (n - 1 - __builtin_popcountll(op.cmask));
        const Ins ins = make_ins(fixed, op.cmask);
        const int w = chunk_width(fixed, ng);
        if (w == 16)
            hipLaunchKernelGGL(k_cp_permx_w<16>, dim3(persistent_blocks(ng / 16)), dim3(kBlock), 0, st, b0, b1,
                               ng / 16, ins, tb);
        else if (w == 4)
            hipLaunchKernelGGL(k_cp_permx_w<4>, dim3(persistent_blocks(ng / 4)), dim3(kBlock), 0, st, b0, b1, ng / 4,
                               ins, tb);
        else
            hipLaunchKernelGGL(k_cp_permx_w<1>, dim3(persistent_blocks(ng)), dim3(kBlock), 0, st, b0, b1, ng, ins, tb);
        JQ_HIP(hipGetLastError());
        return;
    }
    if (op.kind == OP_DIAG && op.keeps_modulus) {
        const uint64_t ng = 1ull << (n - __builtin_popcountll(op.cmask));
        const Ins ins = make_ins(op.cmask, op.cmask);
        Shift sh{};
        if (!phase_code_shifts(op, sh.d)) {
            // the shift puts every code on a rounding tie: decode, rotate and
            // re-encode each amplitude so the tie is broken by its own value
            hipLaunchKernelGGL(k_cp_phase, dim3(persistent_blocks(ng)), dim3(kBlock), 0, st, b0, b1, ng, ins,
                               to_cp(op), (const double*)b.range);
            JQ_HIP(hipGetLastError());
            return;
        }
        const int w = chunk_width(op.cmask, ng);
        const int s0 = op.t0 < 0 ? 0 : op.t0, s1 = op.t1 < 0 ? 0 : op.t1;
        if (w == 16)
            hipLaunchKernelGGL(k_cp_shift_w<16>, dim3(persistent_blocks(ng / 16)), dim3(kBlock), 0, st, b0, b1,
                               ng / 16, ins, op.nsel, s0, s1, sh);
        else if (w == 4)
            hipLaunchKernelGGL(k_cp_shift_w<4>, dim3(persistent_blocks(ng / 4)), dim3(kBlock), 0, st, b0, b1, ng / 4,
                               ins, op.nsel, s0, s1, sh);
        else
            hipLaunchKernelGGL(k_cp_shift_w<1>, dim3(persistent_blocks(ng)), dim3(kBlock), 0, st, b0, b1, ng, ins,
                               op.nsel, s0, s1, sh);
        JQ_HIP(hipGetLastError());
        return;
    }
    const CpGate g = to_cp(op);
    uint64_t ng = 0, hb = 0, lb = 0;
    Ins ins{};
    auto launch = [&](int apply) {
        const double* rn = b.range_next;
        const int w = op.kind == OP_DENSE1 ? chunk_width(lb, ng) : 1;
        switch (op.kind) {
            case OP_DENSE1:
                if (apply) {
                    if (w == 16)
                        hipLaunchKernelGGL((k_cp_dense1_w<16, 1>), dim3(persistent_blocks(ng / 16)), dim3(kBlock), 0,
                                           st, b0, b1, ng / 16, ins, lb, g, (const double*)b.range, rn, acc);
                    else if (w == 4)
                        hipLaunchKernelGGL((k_cp_dense1_w<4, 1>), dim3(persistent_blocks(ng / 4)), dim3(kBlock), 0, st,
                                           b0, b1, ng / 4, ins, lb, g, (const double*)b.range, rn, acc);
                    else
                        hipLaunchKernelGGL((k_cp_dense1_w<1, 1>), dim3(persistent_blocks(ng)), dim3(kBlock), 0, st, b0,
                                           b1, ng, ins, lb, g, (const double*)b.range, rn, acc);
                } else {
                    if (w == 16)
                        hipLaunchKernelGGL((k_cp_dense1_w<16, 0>), dim3(persistent_blocks(ng / 16)), dim3(kBlock), 0,
                                           st, b0, b1, ng / 16, ins, lb, g, (const double*)b.range, rn, acc);
                    else if (w == 4)
                        hipLaunchKernelGGL((k_cp_dense1_w<4, 0>), dim3(persistent_blocks(ng / 4)), dim3(kBlock), 0, st,
                                           b0, b1, ng / 4, ins, lb, g, (const double*)b.range, rn, acc);
                    else
                        hipLaunchKernelGGL((k_cp_dense1_w<1, 0>), dim3(persistent_blocks(ng)), dim3(kBlock), 0, st, b0,
                                           b1, ng, ins, lb, g, (const double*)b.range, rn, acc);
                }
                break;
            case OP_DENSE2:
                hipLaunchKernelGGL(k_cp_gate<OP_DENSE2>, dim3(persistent_blocks(ng)), dim3(kBlock), 0, st, b0, b1, ng,
                                   ins, hb, lb, g, (const double*)b.range, rn, acc, apply);
                break;
            default:
                hipLaunchKernelGGL(k_cp_gate<OP_DIAG>, dim3(persistent_blocks(ng)), dim3(kBlock), 0, st, b0, b1, ng,
                                   ins, hb, lb, g, (const double*)b.range, rn, acc, apply);
                break;
        }
        JQ_HIP(hipGetLastError());
    };
    if (op.kind == OP_DENSE1) {
        lb = 1ull << op.t0;
        ng = dim >> 1;
        ins = make_ins(lb, 0);
    } else if (op.kind == OP_DENSE2) {
        hb = 1ull << op.t0;
        lb = 1ull << op.t1;
        ng = dim >> 2;
        ins = make_ins(hb | lb, 0);
    } else {
        ng = dim;
        ins = make_ins(0, 0);
    }
    if (op.keeps_modulus) {
        // modulus-preserving dense gate (e.g. a permutation matrix given as DENSE): range kept
        hipLaunchKernelGGL(k_cp_resolve, dim3(1), dim3(64), 0, st, acc, (const double*)b.range, b.range_next);
        JQ_HIP(hipGetLastError());
        launch(1);
    } else {
        launch(0);
        hipLaunchKernelGGL(k_cp_resolve, dim3(1), dim3(64), 0, st, acc, (const double*)b.range, b.range_next);
        JQ_HIP(hipGetLastError());
        launch(1);
    }
    JQ_HIP(hipMemcpyAsync(b.range, b.range_next, 2 * sizeof(double), hipMemcpyDeviceToDevice, st));
}

namespace {

template <int K, int F>
void launch_cp_fused(const CompactBufs& b, int n, const FPass& pass, bool keeps, hipStream_t st) {
    const uint64_t dim = 1ull << n;
    const uint64_t ntiles = 1ull << (n - 6 - K);
    const unsigned wpb = (unsigned)(ntiles < 4 ? ntiles : 4);
    const uint64_t blocks_needed = ntiles / wpb;
    // enough waves to fill the chip several times over; each loops over tiles
    const unsigned blocks = (unsigned)(blocks_needed < 4096 ? blocks_needed : 4096);
    int8_t* b0 = b.codes;
    int8_t* b1 = b.codes + dim;
    unsigned long long* acc = (unsigned long long*)b.acc;
    if (!keeps) {
        hipLaunchKernelGGL((k_cp_fused<K, F, 0>), dim3(blocks), dim3(64 * wpb), 0, st, b0, b1, pass, pass.ops, ntiles,
                           (const double*)b.range, (const double*)b.range_next, acc);
        JQ_HIP(hipGetLastError());
    }
    // keeps: acc still holds its reset value, so resolve copies the old range
    hipLaunchKernelGGL(k_cp_resolve, dim3(1), dim3(64), 0, st, acc, (const double*)b.range, b.range_next);
    hipLaunchKernelGGL((k_cp_fused<K, F, 1>), dim3(blocks), dim3(64 * wpb), 0, st, b0, b1, pass, pass.ops, ntiles,
                       (const double*)b.range, (const double*)b.range_next, acc);
    JQ_HIP(hipGetLastError());
    JQ_HIP(hipMemcpyAsync(b.range, b.range_next, 2 * sizeof(double), hipMemcpyDeviceToDevice, st));
}

}  // namespace

namespace {

template <int K>
void launch_cp_codes(const CompactBufs& b, int n, const FPass& pass, hipStream_t st) {
    const uint64_t dim = 1ull << n;
    const uint64_t ntiles = 1ull << (n - 6 - K);
    const unsigned wpb = (unsigned)(ntiles < 4 ? ntiles : 4);
    const uint64_t need = ntiles / wpb;
    // up to 2^20 blocks of 4 waves; larger states loop over their tiles
    const unsigned blocks = (unsigned)(need < (1ull << 20) ? need : (1ull << 20));
    hipLaunchKernelGGL((k_cp_codes<K>), dim3(blocks), dim3(64 * wpb), 0, st, b.codes, b.codes + dim, pass,
                       pass.ops, ntiles);
    JQ_HIP(hipGetLastError());
}

}  // namespace

void cp_apply_codes(const CompactBufs& b, int n, const FPass& pass, int k_reg, int fixed_reg_bits, hipStream_t st) {
    if (n < 6 + k_reg) fail(JQ_EINVAL, "compact code pass: state smaller than a tile");
    if (fixed_reg_bits == kCpCodeRegBits) {
        // the kernel addresses slots 0, 1 as qubits 0, 1 and lane bit b as
        // qubit 2 + b
        bool ok = pass.reg_q[0] == 0 && pass.reg_q[1] == 1;
        for (int q = 0; q < 6; ++q) ok = ok && pass.lane_q[q] == 2 + q;
        if (!ok) fail(JQ_EDEVICE, "compact code pass: tile layout does not match");
        switch (k_reg) {
            case 2: launch_cp_codes<2>(b, n, pass, st); break;
            case 3: launch_cp_codes<3>(b, n, pass, st); break;
            case 4: launch_cp_codes<4>(b, n, pass, st); break;
            case 5: launch_cp_codes<5>(b, n, pass, st); break;
            case 6: launch_cp_codes<6>(b, n, pass, st); break;
            case 7: launch_cp_codes<7>(b, n, pass, st); break;
            default: fail(JQ_EINVAL, "compact code pass: register bits must be 2..7");
        }
        return;
    }
    fail(JQ_EINVAL, "compact code pass: unsupported layout");
}

void cp_apply_block(const CompactBufs& b, int n, const FPass& pass, int k_reg, int fixed_lane_bits, bool keeps,
                    hipStream_t st) {
    ensure_lut();
    if (n < 6 + k_reg) fail(JQ_EINVAL, "compact fused pass: state smaller than a tile");
    if (fixed_lane_bits != kCpFixedLaneBits) fail(JQ_EINVAL, "compact fused pass: unsupported lane layout");
    check_table_tag(pass, dg_table_tag<double>());
    switch (k_reg) {
        case 2: launch_cp_fused<2, kCpFixedLaneBits>(b, n, pass, keeps, st); break;
        case 3: launch_cp_fused<3, kCpFixedLaneBits>(b, n, pass, keeps, st); break;
        case 4: launch_cp_fused<4, kCpFixedLaneBits>(b, n, pass, keeps, st); break;
        default: fail(JQ_EINVAL, "compact fused pass: register bits must be 2..4");
    }
}

void cp_probabilities(const CompactBufs& b, int n, const int* qubits, int nq, double* out, double* partial, size_t cap,
                      hipStream_t st) {
    const uint64_t dim = 1ull << n;
    ensure_lut();
    launch_probs<LoaderCP, 16>(LoaderCP{b.codes, b.codes + dim, b.range, {}}, n, qubits, nq, out, partial, cap, st);
}

void cp_sample(const CompactBufs& b, int n, const double* u, uint64_t count, uint64_t* out, double* scratch,
               hipStream_t st) {
    ensure_lut();
    const uint64_t dim = 1ull << n;
    launch_sample(LoaderCP{b.codes, b.codes + dim, b.range, {}}, n, u, count, out, scratch, st);
}

void cp_expectations(const CompactBufs& b, int n, double* out, double* partial, size_t cap, hipStream_t st) {
    ensure_lut();
    const uint64_t dim = 1ull << n;
    launch_expect(LoaderCP{b.codes, b.codes + dim, b.range, {}}, n, out, partial, cap, st);
}

void cp_scale_range(const CompactBufs& b, double f, hipStream_t st) {
    hipLaunchKernelGGL(k_cp_scale_range, dim3(1), dim3(64), 0, st, b.range, f);
    JQ_HIP(hipGetLastError());
}

void cp_to_c128(const CompactBufs& b, int n, uint64_t first, uint64_t count, double* dst, hipStream_t st) {
    ensure_lut();
    const uint64_t dim = 1ull << n;
    hipLaunchKernelGGL(k_cp_decode, dim3(persistent_blocks(count)), dim3(kBlock), 0, st, b.codes, b.codes + dim, first,
                       count, (const double*)b.range, (double2*)dst);
    JQ_HIP(hipGetLastError());
}

void cp_encode_from_c128(const CompactBufs& b, int n, const double* src, hipStream_t st) {
    const uint64_t dim = 1ull << n;
    unsigned long long* acc = (unsigned long long*)b.acc;
    hipLaunchKernelGGL(k_cp_acc_reset, dim3(1), dim3(64), 0, st, acc);
    hipLaunchKernelGGL(k_cp_range_of, dim3(persistent_blocks(dim)), dim3(kBlock), 0, st, (const double2*)src, dim, acc);
    hipLaunchKernelGGL(k_cp_resolve, dim3(1), dim3(64), 0, st, acc, (const double*)b.range, b.range);
    hipLaunchKernelGGL(k_cp_encode, dim3(persistent_blocks(dim)), dim3(kBlock), 0, st, (const double2*)src, dim,
                       (const double*)b.range, b.codes, b.codes + dim);
    JQ_HIP(hipGetLastError());
}

}  // namespace jq

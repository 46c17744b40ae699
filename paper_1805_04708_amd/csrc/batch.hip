// Batched small circuits in one persistent launch.
//
// Many independent circuits (each N <= 20) run as one batch: a grid sized to
// fill the GPU pulls circuit indices from a device work counter, largest
// states first, and a workgroup owns one circuit at a time.
//
// Block mode (fusion depth KB = 1..3): a circuit is cut into blocks of
// consecutive gates whose targets fall in at most KB qubits.  For each block
// every thread takes groups of 2^KB amplitudes (all values of the block's
// qubits for one value of the others), applies all the block's gates in
// registers, and writes them back; one barrier per block.  Diagonal gates
// and controls are tested on each amplitude's full index.  States of at most
// 64 KiB live in LDS for the whole circuit (two workgroups per CU); larger
// ones are updated in place in their slot of the global arena, where they
// stay L2/MALL resident.
//
// Tile mode (depth 4, states of at least one tile): the circuit runs as the
// register/lane tile passes of the state-vector planner (many gates per
// pass, reordered where they commute) on its arena slot; the workgroup's
// waves loop over the state's tiles, one barrier per pass.  Tile-mode
// circuits run in their own kernel, without LDS, on a second stream forked
// from the batch's stream, concurrently with the block-mode kernel.
//
// The depth is tuned per (encoding, N) on first use in the process, then the
// launch policy (which kernel starts first, and the block kernel's LDS
// request) per encoding.
#include <algorithm>
#include <map>
#include <mutex>

#include "fused_ops.hpp"

namespace jq {

enum BOpKind : int32_t { B_DENSE = 0, B_PERM = 1, B_DIAG = 2, B_DENSE2 = 3 };

struct BOp {
    int32_t kind;
    int32_t slot;     // register slot of the target (B_DENSE2: the MSB target)
    int32_t slot2;    // B_DENSE2: the LSB target's slot
    int32_t nsel;     // B_DIAG selectors
    uint32_t cmask;   // full-index bits that must be 1
    int32_t s0, s1;   // B_DIAG selector qubits
    int32_t pad;
    double m[32];     // B_DENSE 2x2 / B_DENSE2 4x4 / B_DIAG d0..d3 (complex)
};

struct BBlock {
    int32_t k;        // qubits in the block (1..3)
    int32_t q[3];
    int32_t first_op;
    int32_t n_ops;
};

struct BCirc {
    int32_t n;
    int32_t first_block;
    int32_t n_blocks;
    int32_t n_passes;    // tile mode: passes (0: block mode)
    int32_t first_pass;
    int32_t pad;
    uint64_t state_off;  // amplitude offset in the arena
};

// fusion depth value that selects tile mode
constexpr int kTileDepth = 4;

// tile layout per precision, as for single large states: fixed lane bits F
// (128-byte lines) and register bits K
template <typename R>
struct TileShape {
    static constexpr int K = sizeof(R) == 8 ? 4 : 5;
    static constexpr int F = sizeof(R) == 8 ? 3 : 4;
};

constexpr int kBatchThreads = 256;
constexpr int kLdsBytes = 64 * 1024;

template <typename R, int KB>
__device__ __forceinline__ void block_dense(Cx<R> (&a)[1 << KB], int j, const BOp* op, uint32_t base,
                                            const int (&q)[3]) {
    const Cx<R> m0{(R)op->m[0], (R)op->m[1]}, m1{(R)op->m[2], (R)op->m[3]};
    const Cx<R> m2{(R)op->m[4], (R)op->m[5]}, m3{(R)op->m[6], (R)op->m[7]};
    const uint32_t cm = op->cmask;
#pragma unroll
    for (int s = 0; s < (1 << KB); ++s) {
        if ((s >> j) & 1) continue;
        uint32_t idx = base;
#pragma unroll
        for (int i = 0; i < KB; ++i)
            if ((s >> i) & 1) idx |= 1u << q[i];
        const bool ok = (idx & cm) == cm;
        const int t = s | (1 << j);
        const Cx<R> x = a[s], y = a[t];
        const Cx<R> nx = mac2(m0, x, m1, y), ny = mac2(m2, x, m3, y);
        a[s] = csel(ok, nx, x);
        a[t] = csel(ok, ny, y);
    }
}

template <typename R, int KB>
__device__ __forceinline__ void block_perm(Cx<R> (&a)[1 << KB], int j, const BOp* op, uint32_t base,
                                           const int (&q)[3]) {
    const uint32_t cm = op->cmask;
#pragma unroll
    for (int s = 0; s < (1 << KB); ++s) {
        if ((s >> j) & 1) continue;
        uint32_t idx = base;
#pragma unroll
        for (int i = 0; i < KB; ++i)
            if ((s >> i) & 1) idx |= 1u << q[i];
        const bool ok = (idx & cm) == cm;
        const int t = s | (1 << j);
        const Cx<R> x = a[s], y = a[t];
        a[s] = csel(ok, y, x);
        a[t] = csel(ok, x, y);
    }
}

template <typename R, int KB>
__device__ __forceinline__ void block_diag(Cx<R> (&a)[1 << KB], const BOp* op, uint32_t base, const int (&q)[3]) {
    const uint32_t cm = op->cmask;
    Cx<R> d[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) d[i] = Cx<R>{(R)op->m[2 * i], (R)op->m[2 * i + 1]};
#pragma unroll
    for (int s = 0; s < (1 << KB); ++s) {
        uint32_t idx = base;
#pragma unroll
        for (int i = 0; i < KB; ++i)
            if ((s >> i) & 1) idx |= 1u << q[i];
        int sel = 0;
        if (op->nsel >= 1) sel = (idx >> op->s0) & 1;
        if (op->nsel == 2) sel = 2 * sel + ((idx >> op->s1) & 1);
        Cx<R> f = d[0];
        f = csel(sel == 1, d[1], f);
        f = csel(sel == 2, d[2], f);
        f = csel(sel == 3, d[3], f);
        const bool ok = (idx & cm) == cm;
        a[s] = csel(ok, cmulf(f, a[s]), a[s]);
    }
}

// Two-qubit dense op on register slots JH (matrix MSB) and JL, both known at
// compile time so that the register tile is never indexed at run time.
template <typename R, int KB, int JH, int JL>
__device__ __forceinline__ void block_dense2_t(Cx<R> (&a)[1 << KB], const BOp* op, uint32_t base,
                                               const int (&q)[3]) {
    if constexpr (KB >= 2 && JH < KB && JL < KB && JH != JL) {
        const uint32_t cm = op->cmask;
#pragma unroll
        for (int s = 0; s < (1 << KB); ++s) {
            if (((s >> JH) & 1) || ((s >> JL) & 1)) continue;
            uint32_t idx = base;
#pragma unroll
            for (int i = 0; i < KB; ++i)
                if ((s >> i) & 1) idx |= 1u << q[i];
            const bool ok = (idx & cm) == cm;
            constexpr int h = 1 << JH, l = 1 << JL;
            Cx<R> x[4] = {a[s], a[s | l], a[s | h], a[s | h | l]};
            Cx<R> y[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                Cx<R> acc = cmulf(Cx<R>{(R)op->m[8 * r], (R)op->m[8 * r + 1]}, x[0]);
#pragma unroll
                for (int c = 1; c < 4; ++c)
                    acc = cadd(acc, cmulf(Cx<R>{(R)op->m[8 * r + 2 * c], (R)op->m[8 * r + 2 * c + 1]}, x[c]));
                y[r] = acc;
            }
            a[s] = csel(ok, y[0], x[0]);
            a[s | l] = csel(ok, y[1], x[1]);
            a[s | h] = csel(ok, y[2], x[2]);
            a[s | h | l] = csel(ok, y[3], x[3]);
        }
    }
}

template <typename R, int KB>
__device__ __forceinline__ void block_dense2(Cx<R> (&a)[1 << KB], const BOp* op, uint32_t base, const int (&q)[3]) {
    // one empty asm statement per case, as in run_block's slot switch
    switch (op->slot * 4 + op->slot2) {
        case 1: block_dense2_t<R, KB, 0, 1>(a, op, base, q); asm volatile("; batch pair 01"); break;
        case 2: block_dense2_t<R, KB, 0, 2>(a, op, base, q); asm volatile("; batch pair 02"); break;
        case 4: block_dense2_t<R, KB, 1, 0>(a, op, base, q); asm volatile("; batch pair 10"); break;
        case 6: block_dense2_t<R, KB, 1, 2>(a, op, base, q); asm volatile("; batch pair 12"); break;
        case 8: block_dense2_t<R, KB, 2, 0>(a, op, base, q); asm volatile("; batch pair 20"); break;
        case 9: block_dense2_t<R, KB, 2, 1>(a, op, base, q); asm volatile("; batch pair 21"); break;
        default: break;
    }
}

// One block over the whole state S (LDS or global) of dimension 2^n.
template <typename R, int KB>
__device__ void run_block(typename Vec<R>::T* S, int n, const BBlock& blk, const BOp* ops) {
    int q[3] = {blk.q[0], blk.q[1], blk.q[2]};
    // sorted copy for the zero-bit insertion
    int qs[3] = {q[0], q[1], q[2]};
    for (int i = 0; i < KB; ++i)
        for (int k = i + 1; k < KB; ++k)
            if (qs[k] < qs[i]) {
                const int t = qs[i];
                qs[i] = qs[k];
                qs[k] = t;
            }
    const uint32_t groups = 1u << (n - KB);
    for (uint32_t g = threadIdx.x; g < groups; g += blockDim.x) {
        uint32_t base = g;
#pragma unroll
        for (int i = 0; i < KB; ++i) {
            const int p = qs[i];
            base = ((base >> p) << (p + 1)) | (base & ((1u << p) - 1));
        }
        Cx<R> a[1 << KB];
#pragma unroll
        for (int s = 0; s < (1 << KB); ++s) {
            uint32_t idx = base;
#pragma unroll
            for (int i = 0; i < KB; ++i)
                if ((s >> i) & 1) idx |= 1u << q[i];
            a[s] = ld<R>(S, idx);
        }
        for (int o = 0; o < blk.n_ops; ++o) {
            const BOp* op = ops + blk.first_op + o;
            switch (op->kind) {
                case B_DENSE:
                case B_PERM: {
                    const int j = op->slot;
// Each case ends in its own empty asm statement so that the compiler cannot
// merge the cases into one body with a run-time slot (which would move the
// register tile to scratch memory).
#define JQ_BCASE(J)                                                                        \
    case J:                                                                                \
        if constexpr (J < KB) {                                                            \
            if (op->kind == B_DENSE) block_dense<R, KB>(a, J, op, base, q);                \
            else block_perm<R, KB>(a, J, op, base, q);                                     \
        }                                                                                  \
        asm volatile("; batch slot " #J);                                                  \
        break;
                    switch (j) {
                        JQ_BCASE(0)
                        JQ_BCASE(1)
                        JQ_BCASE(2)
                        default:
                            break;
                    }
#undef JQ_BCASE
                    break;
                }
                case B_DIAG:
                    block_diag<R, KB>(a, op, base, q);
                    break;
                case B_DENSE2:
                    block_dense2<R, KB>(a, op, base, q);
                    break;
                default:
                    break;
            }
        }
#pragma unroll
        for (int s = 0; s < (1 << KB); ++s) {
            uint32_t idx = base;
#pragma unroll
            for (int i = 0; i < KB; ++i)
                if ((s >> i) & 1) idx |= 1u << q[i];
            st<R>(S, idx, a[s]);
        }
    }
}

// The passes of one circuit over its state psi (2^n amplitudes, in the
// arena): each wave takes tiles wave, wave + 4, ...; the barrier after each
// pass makes its stores visible to the next pass's loads (one workgroup, one
// compute unit).  In batch plans a pass's ops field holds the index of its
// first op in fops (a kernel argument, so the ops are read with scalar
// loads).
//
// The state starts as |0...0>, and a pass moves amplitude only along its
// tile's qubits (every op is linear, and its selectors and controls outside
// the tile only choose among matrices): after passes 0..p-1 the state is
// zero at every index with a bit set outside the union of their tile
// qubits (the support).  A pass therefore runs only its active tiles, those
// whose outer bits lie in the support (any other tile is zero before and
// after it), enumerated directly and spread over the waves.  Memory holds
// the state only inside the support: the arena is never cleared.  The
// first pass's one active tile, tile 0 (index 0 in lane 0, slot 0), starts
// from |0...0> in registers; a later pass reads only the amplitudes inside
// the support and takes the others as zero.  Its active tiles cover every
// index inside the new support, so the invariant holds after it.  At the
// end, the indices outside the final support (qubits no pass held) are
// written as zeros.
template <typename R>
__device__ void run_tiles(typename Vec<R>::T* psi, int n, const FPass* __restrict__ passes, int n_passes,
                          const FOp* __restrict__ fops) {
    constexpr int K = TileShape<R>::K, F = TileShape<R>::F, S = 1 << K;
    const int lane = threadIdx.x & 63;
    const uint64_t wave = (uint64_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t nw = blockDim.x >> 6;
    const uint64_t ntiles = 1ull << (n - 6 - K);
    uint64_t support = 0;  // qubits of the tiles of the passes so far
    for (int p = 0; p < n_passes; ++p) {
        const FPass& P = passes[p];
        uint64_t lane_off = (uint64_t)(lane & ((1 << F) - 1));
#pragma unroll
        for (int b = F; b < 6; ++b) lane_off |= (uint64_t)((lane >> b) & 1) << P.lane_q[b];
        uint64_t stride[K];
#pragma unroll
        for (int j = 0; j < K; ++j) stride[j] = 1ull << P.reg_q[j];
        const FOp* ops = fops + reinterpret_cast<uintptr_t>(P.ops);
        const int n_ops = P.n_ops;
        uint64_t tmask = 0;
        for (int i = 0; i < P.n_tile; ++i) tmask |= 1ull << P.tile_sorted[i];
        // bit k of a tile number is the k-th lowest qubit outside the tile;
        // act: the bits whose qubit is in the support
        uint64_t act = 0;
        for (int q = 0, k = 0; q < n; ++q) {
            if ((tmask >> q) & 1) continue;
            if ((support >> q) & 1) act |= 1ull << k;
            ++k;
        }
        const uint64_t n_visit = 1ull << __builtin_popcountll(act);
        for (uint64_t j = wave; j < n_visit; j += nw) {
            // the j-th active tile: j's bits deposited at the set bits of act
            uint64_t t = 0, jj = j;
            for (uint64_t m = act; m; m &= m - 1, jj >>= 1)
                if (jj & 1) t |= m & (~m + 1);
            uint64_t base = tile_base(P, t, lane_off);
            Cx<R> a[S];
            if (p == 0) {
#pragma unroll
                for (int s = 0; s < S; ++s) a[s] = Cx<R>{(R)(s == 0 && lane == 0 ? 1 : 0), (R)0};
            } else {
                const uint64_t outside = ~support;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    uint64_t off = 0;
#pragma unroll
                    for (int j = 0; j < K; ++j)
                        if (s & (1 << j)) off += stride[j];
                    const uint64_t i = base + off;
                    a[s] = Cx<R>{(R)0, (R)0};
                    if (!(i & outside)) a[s] = ld<R>(psi, i);
                }
            }
            run_ops<R, K>(a, ops, n_ops, base, wave_uniform(tile_base(P, t, 0)), lane);
            // recompute the store addresses instead of keeping 2^K of them live
            asm volatile("" : "+v"(base));
#pragma unroll
            for (int s = 0; s < S; ++s) {
                uint64_t off = 0;
#pragma unroll
                for (int j = 0; j < K; ++j)
                    if (s & (1 << j)) off += stride[j];
                st<R>(psi, base + off, a[s]);
            }
        }
        support |= tmask;
        __syncthreads();
    }
    const uint64_t outside = ~support & ((1ull << n) - 1);
    if (outside) {
        for (uint64_t i = threadIdx.x; i < (1ull << n); i += blockDim.x)
            if (i & outside) st<R>(psi, i, Cx<R>{(R)0, (R)0});
        __syncthreads();
    }
}

template <typename R>
__global__ __launch_bounds__(kBatchThreads) void k_batch(typename Vec<R>::T* __restrict__ arena,
                                                          const BCirc* __restrict__ circs,
                                                          const int32_t* __restrict__ order, uint32_t count,
                                                          const BBlock* __restrict__ blocks,
                                                          const BOp* __restrict__ ops, uint32_t* counter,
                                                          int lds_max_n) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    typename Vec<R>::T* lds = reinterpret_cast<typename Vec<R>::T*>(lds_raw);
    __shared__ uint32_t next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1u);
        __syncthreads();
        // the same value in every lane: keep it (and what it indexes) scalar
        const uint32_t w = (uint32_t)__builtin_amdgcn_readfirstlane((int)next);
        __syncthreads();
        if (w >= count) break;
        const BCirc c = circs[order[w]];
        const int n = c.n;
        const uint32_t dim = 1u << n;
        typename Vec<R>::T* S = n <= lds_max_n ? lds : arena + c.state_off;
        for (uint32_t i = threadIdx.x; i < dim; i += blockDim.x) {
            typename Vec<R>::T v;
            v.x = (R)(i == 0 ? 1 : 0);
            v.y = (R)0;
            S[i] = v;
        }
        __syncthreads();
        for (int b = 0; b < c.n_blocks; ++b) {
            const BBlock blk = blocks[c.first_block + b];
            switch (blk.k) {
                case 1: run_block<R, 1>(S, n, blk, ops); break;
                case 2: run_block<R, 2>(S, n, blk, ops); break;
                default: run_block<R, 3>(S, n, blk, ops); break;
            }
            __syncthreads();
        }
        if (n <= lds_max_n) {
            for (uint32_t i = threadIdx.x; i < dim; i += blockDim.x) arena[c.state_off + i] = S[i];
            __syncthreads();
        }
    }
}

// Tile-mode circuits (states in the arena): the same work counter scheme,
// no LDS, so more workgroups fit per compute unit than in the block kernel.
// Held to 128 VGPRs (4 waves per SIMD; the complex128 kernel spills 68
// bytes, which costs less than running 3 waves: measured 0.97 vs 1.02 ms
// per 4096-circuit launch).
template <typename R>
__global__ __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_batch_tiles(typename Vec<R>::T* __restrict__ arena,
                                                                const BCirc* __restrict__ circs,
                                                                const int32_t* __restrict__ order, uint32_t count,
                                                                const FPass* __restrict__ passes,
                                                                const FOp* __restrict__ fops, uint32_t* counter) {
    __shared__ uint32_t next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1u);
        __syncthreads();
        // the same value in every lane: keep it (and what it indexes) scalar
        const uint32_t w = (uint32_t)__builtin_amdgcn_readfirstlane((int)next);
        __syncthreads();
        if (w >= count) break;
        const BCirc c = circs[order[w]];
        const uint32_t dim = 1u << c.n;
        typename Vec<R>::T* S = arena + c.state_off;
        if (c.n_passes == 0) {
            // no gates: the state is |0...0>
            for (uint32_t i = threadIdx.x; i < dim; i += blockDim.x) {
                typename Vec<R>::T v;
                v.x = (R)(i == 0 ? 1 : 0);
                v.y = (R)0;
                S[i] = v;
            }
            __syncthreads();
            continue;
        }
        run_tiles<R>(S, c.n, passes + c.first_pass, c.n_passes, fops);
    }
}

__global__ void k_batch_reset(uint32_t* counter) {
    if (threadIdx.x < 2 && blockIdx.x == 0) counter[threadIdx.x] = 0u;
}

// ------------------------------------------------------------- host ------

namespace {

BOp to_bop(const GateOp& op, const int* q, int k) {
    BOp b{};
    b.cmask = (uint32_t)op.cmask;
    auto slot_of = [&](int t) {
        for (int i = 0; i < k; ++i)
            if (q[i] == t) return i;
        fail(JQ_EDEVICE, "batch planner: target outside its block");
    };
    switch (op.kind) {
        case OP_DENSE1:
            b.kind = B_DENSE;
            b.slot = slot_of(op.t0);
            for (int i = 0; i < 4; ++i) {
                b.m[2 * i] = op.m[i].re;
                b.m[2 * i + 1] = op.m[i].im;
            }
            break;
        case OP_PERMX:
            b.kind = B_PERM;
            b.slot = slot_of(op.t0);
            break;
        case OP_DENSE2:
            b.kind = B_DENSE2;
            b.slot = slot_of(op.t0);
            b.slot2 = slot_of(op.t1);
            for (int i = 0; i < 16; ++i) {
                b.m[2 * i] = op.m[i].re;
                b.m[2 * i + 1] = op.m[i].im;
            }
            break;
        default:
            b.kind = B_DIAG;
            b.nsel = op.nsel;
            b.s0 = op.t0 < 0 ? 0 : op.t0;
            b.s1 = op.t1 < 0 ? 0 : op.t1;
            for (int i = 0; i < 4; ++i) {
                b.m[2 * i] = op.m[i].re;
                b.m[2 * i + 1] = op.m[i].im;
            }
    }
    return b;
}

// Cut a circuit into blocks of at most kb target qubits (two-qubit dense
// gates need both targets in one block; kb = 1 gives them a block of 2).
void plan_blocks(const std::vector<GateOp>& ops, int n, int kb, std::vector<BBlock>& blocks,
                 std::vector<BOp>& bops) {
    size_t i = 0;
    while (i < ops.size()) {
        int q[3] = {-1, -1, -1};
        int k = 0;
        const size_t start = i;
        auto has = [&](int t) {
            for (int j = 0; j < k; ++j)
                if (q[j] == t) return true;
            return false;
        };
        for (; i < ops.size(); ++i) {
            const GateOp& op = ops[i];
            int need[2] = {-1, -1};
            int nn = 0;
            if (op.kind == OP_DENSE1 || op.kind == OP_PERMX) need[nn++] = op.t0;
            if (op.kind == OP_DENSE2) {
                need[nn++] = op.t0;
                need[nn++] = op.t1;
            }
            int add = 0;
            for (int j = 0; j < nn; ++j) add += !has(need[j]);
            const int cap = std::max(kb, nn);
            if (k + add > cap) break;
            for (int j = 0; j < nn; ++j)
                if (!has(need[j])) q[k++] = need[j];
        }
        if (k == 0) {
            // only diagonal gates: give them the lowest qubit as the block
            q[k++] = 0;
        }
        // widen to a fixed size of at most 3 with free qubits (cheap, and keeps
        // the number of kernel variants small)
        const int kk = std::min(std::max(k, kb), std::min(3, n));
        for (int t = 0; k < kk && t < n; ++t)
            if (!has(t)) q[k++] = t;
        BBlock blk{};
        blk.k = k;
        for (int j = 0; j < 3; ++j) blk.q[j] = j < k ? q[j] : 0;
        blk.first_op = (int32_t)bops.size();
        for (size_t g = start; g < i; ++g) bops.push_back(to_bop(ops[g], q, k));
        blk.n_ops = (int32_t)(i - start);
        blocks.push_back(blk);
    }
    (void)n;
}

std::mutex g_tune_mu;
std::map<std::pair<int, int>, int> g_tuned_kb;  // (enc, n) -> kb
std::map<int, int> g_tuned_policy;              // enc -> launch policy

constexpr int kPolicyBlockFirst = 1;
constexpr int kPolicyFitLds = 2;

}  // namespace

}  // namespace jq

struct jq_batch {
    int enc = JQ_C128;
    size_t count = 0;
    std::vector<int> n;
    std::vector<uint64_t> offs;
    uint64_t arena_amps = 0;
    void* arena = nullptr;
    void* circs = nullptr;
    void* order = nullptr;       // block-mode circuits, largest state first
    void* order_tile = nullptr;  // tile-mode circuits, largest state first
    uint32_t count_blk = 0, count_tile = 0;
    hipStream_t stream2 = nullptr;  // tile kernel, forked from stream
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int cus = 0, per_cu_blk = 1, per_cu_tile = 1;
    void* blocks = nullptr;
    void* ops = nullptr;
    void* passes = nullptr;  // tile mode: FPass per pass, ops pointing into fops
    void* fops = nullptr;
    uint32_t* counter = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int lds_max_n = 0;
    size_t lds_bytes = 0;      // the block kernel's LDS when the policy does not size it
    size_t lds_fit_bytes = 0;  // the largest LDS-resident block-mode state
    int per_cu_blk_fit = 1;    // occupancy of the block kernel with lds_fit_bytes
    // launch policy (tuned): kPolicyBlockFirst launches the block kernel
    // before the tile kernel; kPolicyFitLds gives it only lds_fit_bytes
    int policy = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<std::vector<jq::GateOp>> ops_host;
    std::vector<int> kb;  // fusion depth used per circuit
    // tile plans, made once per circuit on first use (0 = not made yet,
    // 1 = made, -1 = the circuit cannot run in tile mode)
    std::vector<int> tile_state;
    std::vector<std::vector<jq::FPass>> tile_passes;  // ops field: index into tile_fops[i]
    std::vector<std::vector<jq::FOp>> tile_fops;
};

namespace jq {

namespace {

void free_batch(jq_batch* b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->stream2) (void)hipStreamSynchronize(b->stream2);
    for (void* p : {b->arena, b->circs, b->order, b->order_tile, b->blocks, b->ops, b->passes, b->fops,
                    (void*)b->counter})
        if (p) (void)hipFree(p);
    for (hipEvent_t e : {b->ev0, b->ev1, b->ev_fork, b->ev_join})
        if (e) (void)hipEventDestroy(e);
    if (b->stream2) (void)hipStreamDestroy(b->stream2);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

// Tile mode applies to states that hold a whole tile (they then live in
// the arena, not in LDS).
bool tile_capable(const jq_batch* b, int n) {
    const int K = b->enc == JQ_C128 ? TileShape<double>::K : TileShape<float>::K;
    return n >= 6 + K;
}

// The tile passes of one circuit, appended to passes/fops (a pass's ops
// field holds the index of its first op in fops); false if some gate cannot
// run in a pass (a two-qubit dense gate), in which case the circuit uses
// blocks.  The plan is made on first use and kept.
bool plan_tiles(jq_batch* b, size_t i, std::vector<FPass>& passes, std::vector<FOp>& fops) {
    if (b->tile_state[i] == 0) {
        PlanConfig cfg;
        cfg.n = b->n[i];
        cfg.fixed_lane_bits = b->enc == JQ_C128 ? TileShape<double>::F : TileShape<float>::F;
        cfg.k_reg = b->enc == JQ_C128 ? TileShape<double>::K : TileShape<float>::K;
        cfg.max_ops = 48;
        cfg.always_pass = true;
        cfg.table_elem = b->enc == JQ_C64 ? 4 : 8;
        Plan plan = make_plan(b->ops_host[i], cfg);
        bool ok = true;
        for (const Step& st : plan.steps) ok = ok && st.fused;
        b->tile_state[i] = ok ? 1 : -1;
        if (ok) {
            for (const Step& st : plan.steps) {
                FPass p = st.pass;
                check_table_tag(p, b->enc == JQ_C128 ? dg_table_tag<double>() : dg_table_tag<float>());
                p.ops = reinterpret_cast<const FOp*>((uintptr_t)st.first_fop);
                b->tile_passes[i].push_back(p);
            }
            b->tile_fops[i] = std::move(plan.fops);
        }
    }
    if (b->tile_state[i] < 0) return false;
    const uintptr_t base = fops.size();
    for (FPass p : b->tile_passes[i]) {
        p.ops = reinterpret_cast<const FOp*>(base + reinterpret_cast<uintptr_t>(p.ops));
        passes.push_back(p);
    }
    fops.insert(fops.end(), b->tile_fops[i].begin(), b->tile_fops[i].end());
    return true;
}

// Lay out plans for the given per-circuit depths and upload them.
void upload_plans(jq_batch* b) {
    std::vector<BCirc> circs(b->count);
    std::vector<BBlock> blocks;
    std::vector<BOp> bops;
    std::vector<FPass> passes;
    std::vector<FOp> fops;
    for (size_t i = 0; i < b->count; ++i) {
        BCirc& c = circs[i];
        c = BCirc{};
        c.n = b->n[i];
        c.state_off = b->offs[i];
        c.first_block = (int32_t)blocks.size();
        c.first_pass = (int32_t)passes.size();
        if (b->kb[i] == kTileDepth && tile_capable(b, b->n[i]) && plan_tiles(b, i, passes, fops)) {
            c.n_passes = (int32_t)(passes.size() - c.first_pass);
            c.n_blocks = 0;
            continue;
        }
        plan_blocks(b->ops_host[i], b->n[i], std::min(b->kb[i], 3), blocks, bops);
        c.n_blocks = (int32_t)(blocks.size() - c.first_block);
    }
    if (bops.empty()) bops.push_back(BOp{});
    if (blocks.empty()) blocks.push_back(BBlock{});
    if (fops.empty()) fops.push_back(FOp{});
    if (passes.empty()) passes.push_back(FPass{});
    // one work list per kernel, largest states first (the long jobs start early)
    std::vector<int32_t> ob, ot;
    for (size_t i = 0; i < b->count; ++i) (circs[i].n_passes > 0 ? ot : ob).push_back((int32_t)i);
    auto larger = [&](int32_t x, int32_t y) { return b->n[x] > b->n[y]; };
    std::stable_sort(ob.begin(), ob.end(), larger);
    std::stable_sort(ot.begin(), ot.end(), larger);
    b->count_blk = (uint32_t)ob.size();
    b->count_tile = (uint32_t)ot.size();
    {
        int mx = 0;
        for (int32_t i : ob) mx = std::max(mx, std::min(b->n[i], b->lds_max_n));
        b->lds_fit_bytes = (size_t)bytes_per_amp(b->enc) << mx;
        const void* kfn = b->enc == JQ_C128 ? (const void*)k_batch<double> : (const void*)k_batch<float>;
        JQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b->per_cu_blk_fit, kfn, kBatchThreads,
                                                            b->lds_fit_bytes));
        b->per_cu_blk_fit = std::max(1, b->per_cu_blk_fit);
    }
    if (ob.empty()) ob.push_back(0);
    if (ot.empty()) ot.push_back(0);
    for (void* p : {b->circs, b->blocks, b->ops, b->passes, b->fops, b->order, b->order_tile})
        if (p) JQ_HIP(hipFree(p));
    b->circs = b->blocks = b->ops = b->passes = b->fops = b->order = b->order_tile = nullptr;
    JQ_HIP(hipMalloc(&b->order, ob.size() * sizeof(int32_t)));
    JQ_HIP(hipMalloc(&b->order_tile, ot.size() * sizeof(int32_t)));
    JQ_HIP(hipMemcpy(b->order, ob.data(), ob.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    JQ_HIP(hipMemcpy(b->order_tile, ot.data(), ot.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    JQ_HIP(hipMalloc(&b->circs, circs.size() * sizeof(BCirc)));
    JQ_HIP(hipMalloc(&b->blocks, blocks.size() * sizeof(BBlock)));
    JQ_HIP(hipMalloc(&b->ops, bops.size() * sizeof(BOp)));
    JQ_HIP(hipMalloc(&b->fops, fops.size() * sizeof(FOp)));
    JQ_HIP(hipMalloc(&b->passes, passes.size() * sizeof(FPass)));
    JQ_HIP(hipMemcpy(b->circs, circs.data(), circs.size() * sizeof(BCirc), hipMemcpyHostToDevice));
    JQ_HIP(hipMemcpy(b->blocks, blocks.data(), blocks.size() * sizeof(BBlock), hipMemcpyHostToDevice));
    JQ_HIP(hipMemcpy(b->ops, bops.data(), bops.size() * sizeof(BOp), hipMemcpyHostToDevice));
    JQ_HIP(hipMemcpy(b->fops, fops.data(), fops.size() * sizeof(FOp), hipMemcpyHostToDevice));
    JQ_HIP(hipMemcpy(b->passes, passes.data(), passes.size() * sizeof(FPass), hipMemcpyHostToDevice));
}

// The two kernels are persistent and run concurrently, each pulling its own
// work list; the one launched first takes the compute units first, and the
// block kernel's LDS request bounds how many of its workgroups share a unit
// with the tile kernel's (both choices are tuned: see autotune).
void launch(jq_batch* b) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, b->stream, b->counter);
    JQ_HIP(hipGetLastError());
    auto launch_tiles = [&] {
        JQ_HIP(hipStreamWaitEvent(b->stream2, b->ev_fork, 0));
        const unsigned grid = (unsigned)std::max(1, std::min<int>((int)b->count_tile, b->cus * b->per_cu_tile));
        if (b->enc == JQ_C128)
            hipLaunchKernelGGL(k_batch_tiles<double>, dim3(grid), dim3(kBatchThreads), 0, b->stream2,
                               (double2*)b->arena, (const BCirc*)b->circs, (const int32_t*)b->order_tile,
                               b->count_tile, (const FPass*)b->passes, (const FOp*)b->fops, b->counter + 1);
        else
            hipLaunchKernelGGL(k_batch_tiles<float>, dim3(grid), dim3(kBatchThreads), 0, b->stream2,
                               (float2*)b->arena, (const BCirc*)b->circs, (const int32_t*)b->order_tile,
                               b->count_tile, (const FPass*)b->passes, (const FOp*)b->fops, b->counter + 1);
        JQ_HIP(hipGetLastError());
        JQ_HIP(hipEventRecord(b->ev_join, b->stream2));
    };
    // the tile kernel's stream forks from here, before the block kernel, so
    // that neither kernel waits for the other
    if (b->count_tile) JQ_HIP(hipEventRecord(b->ev_fork, b->stream));
    const bool block_first = (b->policy & kPolicyBlockFirst) != 0;
    if (b->count_tile && !block_first) launch_tiles();
    if (b->count_blk) {
        const bool fit = (b->policy & kPolicyFitLds) != 0;
        const size_t lds = fit ? b->lds_fit_bytes : b->lds_bytes;
        const int per_cu = fit ? b->per_cu_blk_fit : b->per_cu_blk;
        const unsigned grid = (unsigned)std::max(1, std::min<int>((int)b->count_blk, b->cus * per_cu));
        if (b->enc == JQ_C128)
            hipLaunchKernelGGL(k_batch<double>, dim3(grid), dim3(kBatchThreads), lds, b->stream,
                               (double2*)b->arena, (const BCirc*)b->circs, (const int32_t*)b->order,
                               b->count_blk, (const BBlock*)b->blocks, (const BOp*)b->ops, b->counter,
                               b->lds_max_n);
        else
            hipLaunchKernelGGL(k_batch<float>, dim3(grid), dim3(kBatchThreads), lds, b->stream,
                               (float2*)b->arena, (const BCirc*)b->circs, (const int32_t*)b->order,
                               b->count_blk, (const BBlock*)b->blocks, (const BOp*)b->ops, b->counter,
                               b->lds_max_n);
        JQ_HIP(hipGetLastError());
    }
    if (b->count_tile && block_first) launch_tiles();
    if (b->count_tile) JQ_HIP(hipStreamWaitEvent(b->stream, b->ev_join, 0));
}

float timed_launch(jq_batch* b) {
    JQ_HIP(hipEventRecord(b->ev0, b->stream));
    launch(b);
    JQ_HIP(hipEventRecord(b->ev1, b->stream));
    JQ_HIP(hipEventSynchronize(b->ev1));
    float ms = 0.f;
    JQ_HIP(hipEventElapsedTime(&ms, b->ev0, b->ev1));
    return ms;
}

// A tuning trial: the best of three launches after a warm-up launch (one
// launch alone is too noisy to compare modes that differ by 10%).
float trial_ms(jq_batch* b) {
    timed_launch(b);
    float best = timed_launch(b);
    for (int r = 0; r < 2; ++r) best = std::min(best, timed_launch(b));
    return best;
}

void tune_depths(jq_batch* b);

// The launch policy per encoding: on first use in the process, each of the
// four (block kernel first or not, its LDS sized to its states or not) is
// timed on the batch with its tuned depths, and the fastest kept.
void tune_policy(jq_batch* b) {
    auto it = g_tuned_policy.find(b->enc);
    if (it != g_tuned_policy.end()) {
        b->policy = it->second;
        return;
    }
    upload_plans(b);
    float best_ms = 0;
    int best = 0;
    for (int pol = 0; pol < 4; ++pol) {
        b->policy = pol;
        const float ms = trial_ms(b);
        if (pol == 0 || ms < best_ms) {
            best_ms = ms;
            best = pol;
        }
    }
    b->policy = best;
    g_tuned_policy[b->enc] = best;
}

void autotune(jq_batch* b, const jq_exec_opts* opts) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (opts && opts->fusion >= 1) {
        // depth 4 and up: tile mode where it applies (blocks of 3 elsewhere);
        // the launch policy as tuned in this process, if it was
        for (size_t i = 0; i < b->count; ++i)
            b->kb[i] = opts->fusion >= kTileDepth ? kTileDepth : std::min(opts->fusion, std::min(3, b->n[i]));
        auto it = g_tuned_policy.find(b->enc);
        b->policy = it != g_tuned_policy.end() ? it->second : 0;
        return;
    }
    tune_depths(b);
    tune_policy(b);
}

// Fusion depth per (encoding, N): the first batch that meets an untuned N
// times every depth on its circuits of that N (all depths give the same
// state up to rounding) and keeps the fastest for the rest of the process,
// so a circuit runs the same code in every batch of this process.  The
// caller holds g_tune_mu.
void tune_depths(jq_batch* b) {
    std::map<int, std::vector<size_t>> by_n;
    for (size_t i = 0; i < b->count; ++i) by_n[b->n[i]].push_back(i);
    std::vector<int> untuned;
    for (auto& kv : by_n) {
        auto it = g_tuned_kb.find({b->enc, kv.first});
        if (it != g_tuned_kb.end())
            for (size_t i : kv.second) b->kb[i] = it->second;
        else
            untuned.push_back(kv.first);
    }
    if (untuned.empty()) return;
    // time each depth on the whole batch with the untuned sizes at that depth
    const int maxk = 3;
    float best_ms = 0;
    std::map<int, int> best;
    for (int n : untuned) best[n] = std::min(2, n);
    for (int k = 1; k <= maxk; ++k) {
        for (int n : untuned)
            for (size_t i : by_n[n]) b->kb[i] = std::min(k, n);
        upload_plans(b);
        const float ms = trial_ms(b);
        if (k == 1 || ms < best_ms) {
            best_ms = ms;
            for (int n : untuned) best[n] = std::min(k, n);
        }
    }
    // then tile mode, one size at a time from the largest down, kept where
    // the whole batch gets faster
    for (int n : untuned)
        for (size_t i : by_n[n]) b->kb[i] = best[n];
    for (auto it = untuned.rbegin(); it != untuned.rend(); ++it) {
        const int n = *it;
        if (!tile_capable(b, n)) continue;
        for (size_t i : by_n[n]) b->kb[i] = kTileDepth;
        upload_plans(b);
        const float ms = trial_ms(b);
        if (ms < best_ms) {
            best_ms = ms;
            best[n] = kTileDepth;
        } else {
            for (size_t i : by_n[n]) b->kb[i] = best[n];
        }
    }
    for (int n : untuned) {
        g_tuned_kb[{b->enc, n}] = best[n];
        for (size_t i : by_n[n]) b->kb[i] = best[n];
    }
}

}  // namespace

}  // namespace jq

using namespace jq;

extern "C" {

int jq_batch_create(const jq_circuit* cs, size_t count, jq_encoding enc, const jq_exec_opts* opts, void* stream,
                    jq_batch** out) {
    jq_batch* b = nullptr;
    try {
        set_last_error("");
        if (!out) fail(JQ_EINVAL, "jq_batch_create: null output");
        *out = nullptr;
        if (count == 0 || !cs) fail(JQ_EINVAL, "jq_batch_create: empty batch");
        if (count > (1u << 30)) fail(JQ_EINVAL, "jq_batch_create: too many circuits");
        if (enc != JQ_C128 && enc != JQ_C64) fail(JQ_EINVAL, "jq_batch_create: encoding must be c128 or c64");
        b = new jq_batch();
        b->enc = enc;
        b->count = count;
        b->n.resize(count);
        b->offs.resize(count);
        b->ops_host.resize(count);
        b->kb.assign(count, 2);
        b->tile_state.assign(count, 0);
        b->tile_passes.resize(count);
        b->tile_fops.resize(count);
        uint64_t off = 0;
        for (size_t i = 0; i < count; ++i) {
            const int n = cs[i].n_qubits;
            if (n < 1 || n > 20) fail(JQ_EINVAL, "jq_batch_create: circuit " + std::to_string(i) + " needs 1 <= N <= 20");
            if (cs[i].n_gates && !cs[i].gates) fail(JQ_EINVAL, "jq_batch_create: null gates");
            b->n[i] = n;
            b->offs[i] = off;
            off += 1ull << n;
            for (uint64_t g = 0; g < cs[i].n_gates; ++g) {
                if (cs[i].gates[g].nq == 0) continue;
                try {
                    b->ops_host[i].push_back(canonicalize(cs[i].gates[g], n));
                } catch (const Error& e) {
                    fail(e.code, "circuit " + std::to_string(i) + " gate " + std::to_string(g) + ": " + e.what());
                }
            }
        }
        b->arena_amps = off;
        const int bpa = bytes_per_amp(enc);
        size_t free_b = 0, total_b = 0;
        JQ_HIP(hipMemGetInfo(&free_b, &total_b));
        if (off * bpa > free_b) fail(JQ_ENOMEM, "jq_batch_create: arena does not fit in device memory");
        JQ_HIP(hipMalloc(&b->arena, off * bpa));
        JQ_HIP(hipMalloc(&b->counter, 2 * sizeof(uint32_t)));  // block kernel, tile kernel
        // LDS-resident states up to 64 KiB
        int lds_n = 0;
        while (lds_n < 20 && ((size_t)bpa << (lds_n + 1)) <= (size_t)kLdsBytes) ++lds_n;
        b->lds_max_n = lds_n;
        b->lds_bytes = (size_t)bpa << lds_n;
        int dev = 0;
        JQ_HIP(hipGetDevice(&dev));
        JQ_HIP(hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev));
        const void* kfn = enc == JQ_C128 ? (const void*)k_batch<double> : (const void*)k_batch<float>;
        const void* kft = enc == JQ_C128 ? (const void*)k_batch_tiles<double> : (const void*)k_batch_tiles<float>;
        JQ_HIP(hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds_bytes));
        JQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b->per_cu_blk, kfn, kBatchThreads, b->lds_bytes));
        JQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b->per_cu_tile, kft, kBatchThreads, 0));
        b->per_cu_blk = std::max(1, b->per_cu_blk);
        b->per_cu_tile = std::max(1, b->per_cu_tile);
        if (stream) {
            b->stream = (hipStream_t)stream;
        } else {
            JQ_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
            b->own_stream = true;
        }
        JQ_HIP(hipStreamCreateWithFlags(&b->stream2, hipStreamNonBlocking));
        JQ_HIP(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
        JQ_HIP(hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming));
        JQ_HIP(hipEventCreate(&b->ev0));
        JQ_HIP(hipEventCreate(&b->ev1));
        autotune(b, opts);
        upload_plans(b);
        *out = b;
        return JQ_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        free_batch(b);
        return e.code;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        free_batch(b);
        return JQ_EDEVICE;
    }
}

int jq_batch_run(jq_batch* b, double* elapsed_ms) {
    try {
        set_last_error("");
        if (!b) fail(JQ_EINVAL, "null batch");
        if (elapsed_ms) {
            *elapsed_ms = timed_launch(b);
        } else {
            launch(b);
        }
        return JQ_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    }
}

int jq_batch_read(jq_batch* b, size_t index, uint64_t first, uint64_t count, double* out) {
    try {
        set_last_error("");
        if (!b) fail(JQ_EINVAL, "null batch");
        if (index >= b->count) fail(JQ_EINVAL, "jq_batch_read: index out of range");
        const uint64_t dim = 1ull << b->n[index];
        if (first > dim || count > dim - first) fail(JQ_EINVAL, "jq_batch_read: range out of bounds");
        if (count && !out) fail(JQ_EINVAL, "jq_batch_read: null output");
        const uint64_t at = b->offs[index] + first;
        if (b->enc == JQ_C128) {
            JQ_HIP(hipMemcpyAsync(out, (const double2*)b->arena + at, count * 16, hipMemcpyDeviceToHost, b->stream));
        } else {
            double* tmp = nullptr;
            JQ_HIP(hipMalloc(&tmp, std::max<uint64_t>(count, 1) * 16));
            sv_to_c128(JQ_C64, b->arena, at, count, tmp, b->stream);
            JQ_HIP(hipMemcpyAsync(out, tmp, count * 16, hipMemcpyDeviceToHost, b->stream));
            JQ_HIP(hipStreamSynchronize(b->stream));
            JQ_HIP(hipFree(tmp));
        }
        JQ_HIP(hipStreamSynchronize(b->stream));
        return JQ_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    }
}

int jq_batch_destroy(jq_batch* b) {
    free_batch(b);
    return JQ_OK;
}

}  // extern "C"

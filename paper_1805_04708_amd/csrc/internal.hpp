// Internal types of the jq library: error plumbing, canonical gate ops, the
// fused-pass plan, and the launcher entry points of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/jq.h"

namespace jq {

// ---------------------------------------------------------------- errors --

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);
[[noreturn]] void fail(int code, const std::string& msg);
void hip_check(hipError_t e, const char* what);

#define JQ_HIP(call) ::jq::hip_check((call), #call)

// ------------------------------------------------------- canonical gate --

// A gate reduced to one of four device operations (the planner's input).
//  DENSE1: 2x2 matrix m[0..3] on target t0.
//  DENSE2: 4x4 matrix m[0..15] on (t0, t1), t0 the MSB of the matrix index.
//  DIAG:   multiply by d[sel] where sel is built from the bits of the
//          nsel selector qubits (t0 the MSB when nsel == 2); nsel == 0
//          multiplies the whole controlled subset by d[0].
//  PERMX:  exchange the amplitude pairs that differ in bit t0.
// Every op acts only where all bits of cmask are 1.
enum OpKind : int32_t { OP_DENSE1 = 0, OP_DENSE2 = 1, OP_DIAG = 2, OP_PERMX = 3 };

struct cd {
    double re, im;
};

struct GateOp {
    int32_t kind = OP_DENSE1;
    int32_t t0 = -1, t1 = -1;
    int32_t nsel = 0;
    uint64_t cmask = 0;
    cd m[16] = {};
    // unimodular diagonal or permutation: leaves every modulus unchanged
    bool keeps_modulus = false;
    uint64_t support() const {
        uint64_t s = cmask;
        if (t0 >= 0) s |= 1ull << t0;
        if (t1 >= 0) s |= 1ull << t1;
        return s;
    }
    // number of amplitudes the op reads and writes
    uint64_t touched(int n) const {
        int fixed = __builtin_popcountll(cmask);
        return 1ull << (n - fixed);
    }
};

// Lower a jq_gate (ABI form) to a canonical op, validating it against n.
GateOp canonicalize(const jq_gate& g, int n);

// Phase-code shifts of a modulus-preserving diagonal op on the two-byte code:
// d[i] = 128 arg(m[i]) / pi in code units.  False when a shift lies within
// 1e-6 of a half-integer (a rounding tie, which the amplitude's own value
// must decide); then the op is applied by decoding, rotating and encoding.
bool phase_code_shifts(const GateOp& op, double d[4]);

// Lower a named App. A instruction into a jq_gate (throws Error).
int gate_named(const char* name, const int* qubits, int nq, const double* params, int np, jq_gate* out);

// ------------------------------------------------------- fused passes --

// Lane bits of a wavefront: bits 0..F-1 of the lane id are index bits
// 0..F-1 (F = 3 for 16-byte amplitudes, so eight lanes cover one 128-byte
// line); lane bits F..5 map to arbitrary qubits.  A thread holds 2^K
// amplitudes, register slot bit j being qubit reg_q[j].
enum FOpKind : int32_t {
    F_DENSE_REG = 0,    // 2x2 on a register slot
    F_CDENSE_REG = 1,   // controlled 2x2 on a register slot
    F_DENSE_LANE = 2,   // 2x2 on a lane bit
    F_CDENSE_LANE = 3,  // controlled 2x2 on a lane bit
    F_PERM_REG = 4,     // X (controlled or not) on a register slot
    F_PERM_LANE = 5,    // X (controlled or not) on a lane bit
    F_PHASE = 6,        // multiply the controlled subset by d0
    F_NEG = 7,          // negate the controlled subset (d0 = -1)
    F_DIAG = 8,         // diagonal with one or two selector bits
    F_MDENSE_REG = 9,   // 2x2 on a register slot chosen by 1-2 selector bits
    F_MDENSE_LANE = 10, // 2x2 on a lane bit chosen by 1-2 selector bits
    F_CSHIFT = 11,      // two-byte code: add the integer m[v] to the phase code (v = selector value),
                        // run as the masked-add terms cs_*
    F_DGROUP = 12,      // product of uncontrolled one-qubit diagonals: n_od on lane bits and
                        // index bits outside the tile, and those on register slots as their
                        // product per slot s, a table whose element type slot names
                        // (kDgTableF64: double pairs at m[2s], m[2s+1], at most 16 slots;
                        // kDgTableF32: float pairs over m's bytes, at most 32; 0: no table)
};

// F_DGROUP register tables: the tag in FOp::slot and the slots each holds
constexpr int kDgTableF64 = 1;
constexpr int kDgTableF32 = 2;
constexpr int kDgSlotsF64 = 16;
constexpr int kDgSlotsF32 = 32;
// the tag of the tables a kernel computing in R reads
template <typename R>
constexpr int dg_table_tag() { return sizeof(R) == 4 ? kDgTableF32 : kDgTableF64; }


constexpr int kMaxOdiag = 8;  // components of one F_DGROUP op

struct FOp {
    int32_t kind;
    int32_t slot;        // register slot bit or lane bit of the target
    uint32_t reg_ctrl;   // register slots whose bit must be 1
    int32_t has_ctrl;    // any control at all
    uint64_t thr_ctrl;   // index bits outside the register slots that must be 1
    int32_t sel_reg[2];  // diag selector / dense multiplexer bit as register slot, or -1
    int32_t sel_glob[2]; // the same as a thread index bit (lane/outer), or -1
    int32_t nsel;        // diag: selector bits; dense: multiplexer bits (0..2)
    int32_t sel_lane;    // bit i: sel_glob[i] is a lane bit of the tile (else an
                         // outer bit, the same in every lane of a wave)
    // dense: matrix v (v = multiplexer value, first selector the MSB) at
    // m[8v .. 8v+7] as m00 m01 m10 m11; diag: d0..d3
    double m[32];
    // code-domain phase shift as cs_n masked adds: slot s of a thread gets
    // cs_add[t] (phase-code units in bits 8..15) where (s & cs_reg[t]) ==
    // cs_reg[t] and the thread's index has every bit of cs_thr[t] set
    int32_t cs_n;
    uint32_t cs_reg[4];
    uint32_t cs_add[4];
    uint64_t cs_thr[4];
    // F_DGROUP: component c acts on lane bit (od_where[c] = 1) or index bit
    // (od_where[c] = 2) od_idx[c], with values d0, d1 at od_m[4c .. 4c+3]
    int32_t n_od;
    int32_t od_where[kMaxOdiag];
    int32_t od_idx[kMaxOdiag];
    double od_m[4 * kMaxOdiag];
};

// the fused kernels read FOp::m with 16-byte vector loads per lane
static_assert(offsetof(FOp, m) % 16 == 0 && sizeof(FOp) % 16 == 0, "FOp::m must stay 16-byte aligned in an array");

constexpr int kMaxTileBits = 16;

struct FPass {
    int32_t reg_q[8];
    int32_t lane_q[6];
    int32_t n_tile;
    int32_t tile_sorted[kMaxTileBits];
    int32_t n_ops;
    int32_t table_tag;   // the tag of the pass's F_DGROUP register tables (0: none)
    uint32_t kinds;      // bit k: the pass holds an op of kind k (0: not recorded, any kind)
    const FOp* ops;      // device pointer
};

// Host check before a fused pass runs in a kernel computing in R: its
// register tables must be in R's element type (throws JQ_EINVAL).
void check_table_tag(const FPass& p, int tag_of_kernel);

// One step of an execution plan: a single op through a per-gate kernel, or
// a fused pass over [first_fop, first_fop + n_fops) of the plan's FOp list.
struct Step {
    bool fused = false;
    GateOp op;              // single
    FPass pass{};           // fused (ops pointer patched after upload)
    size_t first_fop = 0;
    int k_reg = 0;          // register bits of the fused kernel
    size_t n_gates = 0;     // source gates covered
    std::vector<int> gates; // their indices in the op list, in the order applied
};

struct PlanConfig {
    int n = 0;
    int fixed_lane_bits = 3;  // F
    int k_reg = 5;            // K
    int max_ops = 48;
    bool fuse = true;
    bool absorb = true;  // fold diagonal gates into neighbouring dense gates
    // two-byte code with per-gate quantisation: only permutations and
    // modulus-preserving phase shifts (exact on the codes) fuse, and no gate
    // moves past one that does not
    bool code_domain = false;
    // R register slots fixed to qubits 0..R-1; the F fixed lane bits are
    // then qubits R..R+F-1 (R = 0: lane bit b is qubit b)
    int fixed_reg_bits = 0;
    // every run of fusable gates becomes a pass, however few bytes single
    // gates would move (states that stay in the caches)
    bool always_pass = false;
    // rounds of the tile-slot search (0: first come, first served)
    int search_rounds = 0;
    // time of a pass's streaming in units of one op's arithmetic (weighs
    // fewer passes against more ops in the search)
    double pass_ops = 18.0;
    // bytes of the fused kernel's real type: 8 (double pairs in per-slot
    // diagonal tables, up to 16 slots) or 4 (complex64: float pairs, up to
    // 32); make_plan rejects other values
    int table_elem = 8;
    // widest register width at which the fused kernel compiled for every op
    // kind keeps 4 waves per SIMD (0: no limit); make_plan narrows a wider
    // k_reg to it unless every gate lowers to the reduced kind set, or the
    // caller asked for the width (k_explicit)
    int k_general_max = 0;
    bool k_explicit = false;
};

struct Plan {
    std::vector<Step> steps;
    std::vector<FOp> fops;
};

// Called after each step is appended (plan.steps.back(); a fused step's
// ops are at the end of plan.fops), so a caller can launch steps while the
// rest is still being planned.
using StepSink = std::function<void(Plan&)>;
Plan make_plan(const std::vector<GateOp>& ops, const PlanConfig& cfg, const StepSink& on_step = {});

// ------------------------------------------------------------ kernels --

enum Enc : int32_t { ENC_C128 = JQ_C128, ENC_C64 = JQ_C64, ENC_COMPACT = JQ_COMPACT };

// 2^(-N/2), correctly rounded: exact for even N, sqrt(1/2) * 2^(-(N-1)/2) for odd N
inline double uniform_amplitude(int n) {
    return (n % 2 == 0) ? std::ldexp(1.0, -n / 2) : std::ldexp(std::sqrt(0.5), -(n - 1) / 2);
}

inline int bytes_per_amp(int enc) { return enc == JQ_C128 ? 16 : enc == JQ_C64 ? 8 : 2; }

// state-vector (c128 / c64) launchers; psi is the device buffer
void sv_init(int enc, void* psi, int n, int mode, uint64_t basis, hipStream_t st);
// one op by its per-gate kernel; wide_mask: dense and X targets whose bit is
// set take four pairs per thread (the others one)
void sv_apply_op(int enc, void* psi, int n, const GateOp& op, uint64_t wide_mask, hipStream_t st);
// SHORBOX (App. A): 2^(-n_x/2) sum_x |x>|y^x mod G>, x on the n_x low qubits
void sv_shorbox(int enc, void* psi, int n, int n_x, uint64_t G, uint64_t y, hipStream_t st);
void sv_apply_fused(int enc, void* psi, int n, const FPass& pass, int k_reg, int fixed_lane_bits,
                    hipStream_t st);
// FP64 marginal distribution; out_dev receives 2^nq doubles (device)
void sv_probabilities(int enc, const void* psi, int n, const int* qubits, int nq, double* out_dev,
                      double* partial_dev, size_t partial_cap, hipStream_t st);
size_t probabilities_partial_count(int n, int nq);
void sv_expectations(int enc, const void* psi, int n, double* out_dev /* 3*n */, double* partial_dev,
                     size_t partial_cap, hipStream_t st);
void sv_scale(int enc, void* psi, int n, double factor, hipStream_t st);
// Sampling hierarchy: 16 amplitudes per thread, 4096 per block, 4096 blocks
// per super-block.
constexpr int kSampleLeaf = 16;
constexpr int kSampleBlockBits = 12;
constexpr int kSampleSuperBits = 12;

// Scratch of the sampler: nblocks (block sums) + nblocks (block prefixes) +
// nsuper (super-block sums) + nsuper + 1 (super-block prefixes) doubles.
inline size_t sample_scratch_doubles(int n) {
    const uint64_t nblocks = n > kSampleBlockBits ? 1ull << (n - kSampleBlockBits) : 1;
    const uint64_t nsuper = (nblocks + (1ull << kSampleSuperBits) - 1) >> kSampleSuperBits;
    return 2 * nblocks + 2 * nsuper + 1;
}

// basis states drawn from |a|^2 for the draws u (device arrays; scratch holds
// sample_scratch_doubles(n) doubles)
void sv_sample(int enc, const void* psi, int n, const double* u, uint64_t count, uint64_t* out, double* scratch,
               hipStream_t st);
// convert [first, first+count) to complex128 into dst (device)
void sv_to_c128(int enc, const void* psi, uint64_t first, uint64_t count, double* dst, hipStream_t st);
void sv_from_c128(int enc, void* psi, uint64_t first, uint64_t count, const double* src, hipStream_t st);

// two-byte code launchers (planes b0 = codes, b1 = codes + 2^n)
struct CompactBufs {
    int8_t* codes;     // b0 plane then b1 plane
    double* range;     // [2]: current (r0, r1)
    double* range_next;// [2]: resolved range of the gate in flight
    uint64_t* acc;     // [2]: min / max of |z| as ordered bit patterns
};
void cp_init(const CompactBufs& b, int n, int mode, uint64_t basis, hipStream_t st);
void cp_apply_op(const CompactBufs& b, int n, const GateOp& op, hipStream_t st);
void cp_shorbox(const CompactBufs& b, int n, int n_x, uint64_t G, uint64_t y, hipStream_t st);
// lane bits of the compact fused pass fixed to index bits 0..F-1 (each
// code plane is read in runs of 2^F bytes)
constexpr int kCpFixedLaneBits = 6;
// a fused pass of code-domain ops (permutations, integer phase-code shifts)
// on both code planes, no decoding; qubits 0 and 1 in register slots 0 and
// 1 (fixed_reg_bits = kCpCodeRegBits), lane bits qubits 2..7
constexpr int kCpCodeRegBits = 2;
void cp_apply_codes(const CompactBufs& b, int n, const FPass& pass, int k_reg, int fixed_reg_bits, hipStream_t st);
// one fused pass quantised once: decode, the pass's ops in FP64, range
// (unless every gate of the block keeps all moduli), encode
void cp_apply_block(const CompactBufs& b, int n, const FPass& pass, int k_reg, int fixed_lane_bits,
                    bool keeps_modulus, hipStream_t st);
void cp_probabilities(const CompactBufs& b, int n, const int* qubits, int nq, double* out_dev,
                      double* partial_dev, size_t partial_cap, hipStream_t st);
void cp_expectations(const CompactBufs& b, int n, double* out_dev, double* partial_dev, size_t cap,
                     hipStream_t st);
void cp_scale_range(const CompactBufs& b, double factor, hipStream_t st);
void cp_sample(const CompactBufs& b, int n, const double* u, uint64_t count, uint64_t* out, double* scratch,
               hipStream_t st);
void cp_to_c128(const CompactBufs& b, int n, uint64_t first, uint64_t count, double* dst,
                hipStream_t st);
void cp_encode_from_c128(const CompactBufs& b, int n, const double* src, hipStream_t st);

// ---------------------------------------------------- runtime helpers --

// Create a state whose work runs on `stream`.  async_alloc: its device
// memory comes from the stream-ordered allocator (hipMallocAsync) and is
// returned with hipFreeAsync, so creating and destroying states never waits
// for other streams (used by the request loop).
jq_state* state_create(int n, int enc, hipStream_t stream, bool async_alloc);

// Apply canonical ops to a state (planner + kernels), asynchronously.
void state_apply(jq_state* s, const std::vector<GateOp>& ops, const jq_exec_opts* opts);

// The planner's configuration for an N-qubit state of encoding enc under
// the caller's options (validated; NULL or fusion 0: the tuned values).
PlanConfig plan_config(int n, int enc, const jq_exec_opts* opts);
// The configuration with a given register width and pass weight (tuning).
PlanConfig plan_config_tuned(int n, int enc, int k_reg, double pass_ops);
// Apply canonical ops under an explicit planner configuration.
void state_apply_config(jq_state* s, const std::vector<GateOp>& ops, const PlanConfig& cfg);

// Tuning of the single-state path (tuning.cpp): the values for an N-qubit
// state of encoding enc on the current device, and the built-in defaults.
jq_tuning tuned_for(int n, int enc);
jq_tuning default_tuning(int enc);
// Enqueue the FP64 squared norm into pinned host memory (no synchronisation).
void state_norm_async(jq_state* s, double* pinned_out);

}  // namespace jq

// --------------------------------------------------------------- state --

struct jq_state {
    int n = 0;
    int enc = JQ_C128;
    void* buf = nullptr;         // amplitudes or code planes
    uint64_t bytes = 0;
    double* aux = nullptr;       // device scratch: ranges, accumulators, reduction partials
    size_t aux_doubles = 0;
    void* (*alloc)(size_t, void*) = nullptr;
    void (*release)(void*, void*) = nullptr;
    void* alloc_ctx = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool async_alloc = false;
    int device = 0;
    // per-launch timing
    bool profiling = false;
    struct Rec {
        int cls;
        double bytes;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> event_pool;
    struct Acc {
        uint64_t launches = 0;
        double ms = 0, bytes = 0;
    };
    std::vector<Acc> acc;
    // fused-op list: with stream-ordered allocation, a device copy of the
    // last plan; without, a ring of plan_dev_bytes in device memory and in
    // pinned staging, filled from ring_head on, with the copies still to run
    void* plan_dev = nullptr;
    void* plan_host = nullptr;
    size_t plan_dev_bytes = 0;
    struct RingUse {
        size_t off, n;  // FOp slots
        hipEvent_t ev;  // recorded after the copy out of them
    };
    size_t ring_head = 0;
    std::deque<RingUse> ring_busy;
    std::vector<hipEvent_t> ring_ev_free;
};

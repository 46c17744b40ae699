// The C ABI of include/jq.h: state objects, validation, planning and
// dispatch to the HIP kernels, FP64 reductions, transfers and timing.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "internal.hpp"

namespace jq {

namespace {
thread_local std::string g_last_error;

struct AllocHooks {
    void* (*alloc)(size_t, void*) = nullptr;
    void (*release)(void*, void*) = nullptr;
    void* ctx = nullptr;
};
AllocHooks g_hooks;
std::mutex g_hooks_mu;
}  // namespace

void set_last_error(const std::string& msg) { g_last_error = msg; }

void fail(int code, const std::string& msg) { throw Error(code, msg); }

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(e == hipErrorOutOfMemory ? JQ_ENOMEM : JQ_EDEVICE,
                    std::string(what) + ": " + hipGetErrorString(e));
    }
}

template <class F>
int guarded(F&& f) {
    try {
        g_last_error.clear();
        f();
        return JQ_OK;
    } catch (const Error& e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return JQ_ENOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return JQ_EDEVICE;
    }
}

// ------------------------------------------------------ kernel timing --

enum KClass {
    K_DENSE1, K_DENSE2, K_DIAG, K_PERMX, K_FUSED, K_CP_GATE, K_CP_PERM, K_CP_PHASE, K_REDUCE, K_CP_FUSED,
    K_CP_CODES, K_NCLASS
};
const char* kClassName[K_NCLASS] = {"dense1", "dense2", "diag", "permx", "fused", "compact_gate",
                                    "compact_perm", "compact_phase", "reduce", "compact_fused", "compact_codes"};

struct Timed {
    jq_state* s;
    int cls;
    double bytes;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(jq_state* st, int c, double by) : s(st), cls(c), bytes(by) {
        if (!s->profiling) return;
        a = take();
        b = take();
        JQ_HIP(hipEventRecord(a, s->stream));
    }
    ~Timed() {
        if (!s->profiling) return;
        if (hipEventRecord(b, s->stream) == hipSuccess) s->recs.push_back({cls, bytes, a, b});
    }
    hipEvent_t take() {
        if (s->event_pool.empty()) {
            hipEvent_t e;
            JQ_HIP(hipEventCreate(&e));
            return e;
        }
        hipEvent_t e = s->event_pool.back();
        s->event_pool.pop_back();
        return e;
    }
};

void drain_profile(jq_state* s) {
    if (s->recs.empty()) return;
    JQ_HIP(hipStreamSynchronize(s->stream));
    if (s->acc.size() < K_NCLASS) s->acc.resize(K_NCLASS);
    for (auto& r : s->recs) {
        float ms = 0.f;
        JQ_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        s->acc[r.cls].launches++;
        s->acc[r.cls].ms += ms;
        s->acc[r.cls].bytes += r.bytes;
        s->event_pool.push_back(r.a);
        s->event_pool.push_back(r.b);
    }
    s->recs.clear();
}

// ------------------------------------------------------ debug switches --

// Read once per process from the environment:
//  JQ_LAUNCH_BLOCKING=1  wait for every kernel and check it before the call
//                        returns (a device fault then names its step);
//  JQ_FORCE_KERNEL=per_gate | fused
//                        every circuit runs one kernel per gate, or every run
//                        of fusable gates as a fused pass (results the same up
//                        to rounding);
//  JQ_ROCTX=1            roctx ranges around each call and each step, for
//                        rocprofv3 --marker-trace;
//  JQ_FUSED_OPS=all      every complex128 / complex64 fused pass runs the op
//                        loop compiled for every op kind, also where the
//                        reduced loop would do (the same amplitudes, bit for
//                        bit: both instances share the ops' code).
struct DebugFlags {
    bool launch_blocking = false;
    int force = 0;  // 0: none, 1: per gate, 2: fused
    bool roctx = false;
    bool fused_all_kinds = false;
};

const DebugFlags& debug_flags() {
    static const DebugFlags f = [] {
        DebugFlags d;
        auto on = [](const char* v) { return v && v[0] && std::strcmp(v, "0") != 0; };
        d.launch_blocking = on(std::getenv("JQ_LAUNCH_BLOCKING"));
        d.roctx = on(std::getenv("JQ_ROCTX"));
        if (const char* k = std::getenv("JQ_FORCE_KERNEL")) {
            if (!std::strcmp(k, "per_gate")) d.force = 1;
            else if (!std::strcmp(k, "fused")) d.force = 2;
        }
        if (const char* k = std::getenv("JQ_FUSED_OPS")) d.fused_all_kinds = !std::strcmp(k, "all");
        return d;
    }();
    return f;
}

// A roctx range for the lifetime of the object (only with JQ_ROCTX set).
struct Range {
    bool on;
    template <class F>
    explicit Range(F&& label) : on(debug_flags().roctx) {
        if (on) roctxRangePushA(label().c_str());
    }
    ~Range() {
        if (on) roctxRangePop();
    }
};

// With JQ_LAUNCH_BLOCKING: wait for the stream and report a failed step.
void blocking_check(jq_state* s, const char* what) {
    if (!debug_flags().launch_blocking) return;
    const hipError_t e = hipStreamSynchronize(s->stream);
    const hipError_t l = hipGetLastError();
    if (e != hipSuccess || l != hipSuccess)
        fail(JQ_EDEVICE, std::string(what) + ": " + hipGetErrorString(e != hipSuccess ? e : l));
}

// ---------------------------------------------------------- helpers --

CompactBufs compact_bufs(jq_state* s) {
    CompactBufs b;
    b.codes = (int8_t*)s->buf;
    b.range = s->aux;
    b.range_next = s->aux + 2;
    b.acc = (uint64_t*)(s->aux + 4);
    return b;
}

constexpr size_t kAuxHead = 8;  // doubles reserved at the start of aux

double* partials(jq_state* s, size_t need) {
    if (kAuxHead + need > s->aux_doubles) {
        JQ_HIP(hipStreamSynchronize(s->stream));
        double* na = nullptr;
        const size_t cnt = kAuxHead + need;
        JQ_HIP(hipMalloc(&na, cnt * sizeof(double)));
        JQ_HIP(hipMemcpy(na, s->aux, kAuxHead * sizeof(double), hipMemcpyDeviceToDevice));
        JQ_HIP(hipFree(s->aux));
        s->aux = na;
        s->aux_doubles = cnt;
    }
    return s->aux + kAuxHead;
}

void check_state(const jq_state* s) {
    if (!s) fail(JQ_EINVAL, "null state");
}

// Validate and lower a gate list (identity gates dropped).
std::vector<GateOp> lower_circuit(const jq_state* s, const jq_gate* gates, size_t count, const char* who) {
    if (count && !gates) fail(JQ_EINVAL, std::string(who) + ": null gates");
    std::vector<GateOp> ops;
    ops.reserve(count);
    for (size_t i = 0; i < count; ++i) {
        if (gates[i].nq == 0) continue;  // identity
        try {
            ops.push_back(canonicalize(gates[i], s->n));
        } catch (const Error& e) {
            fail(e.code, "gate " + std::to_string(i) + ": " + e.what());
        }
    }
    return ops;
}

double op_bytes(const GateOp& op, int n, int enc) {
    const double bpa = bytes_per_amp(enc);
    const double touched = std::ldexp((double)op.touched(n), 0);
    double amps = touched;
    if (op.kind == OP_DIAG) amps = touched;  // each touched amplitude read and written once
    if (enc == JQ_COMPACT) {
        if (op.kind == OP_PERMX) return 2.0 * amps * 2.0;
        if (op.kind == OP_DIAG && op.keeps_modulus) return amps * 1.0 + 2.0 * amps * 1.0;
        const double full = std::ldexp(1.0, n);
        return op.keeps_modulus ? 2.0 * full * 2.0 : 3.0 * full * 2.0;
    }
    return 2.0 * amps * bpa;
}

int kclass(const GateOp& op, int enc) {
    if (enc == JQ_COMPACT) {
        if (op.kind == OP_PERMX) return K_CP_PERM;
        if (op.kind == OP_DIAG && op.keeps_modulus) return K_CP_PHASE;
        return K_CP_GATE;
    }
    switch (op.kind) {
        case OP_DENSE1: return K_DENSE1;
        case OP_DENSE2: return K_DENSE2;
        case OP_DIAG: return K_DIAG;
        default: return K_PERMX;
    }
}

void run_single(jq_state* s, const GateOp& op) {
    Range r([&] {
        return std::string(kClassName[kclass(op, s->enc)]) + " t0=" + std::to_string(op.t0) +
               " t1=" + std::to_string(op.t1);
    });
    {
        Timed t(s, kclass(op, s->enc), op_bytes(op, s->n, s->enc));
        if (s->enc == JQ_COMPACT) cp_apply_op(compact_bufs(s), s->n, op, s->stream);
        else sv_apply_op(s->enc, s->buf, s->n, op, tuned_for(s->n, s->enc).wide_mask, s->stream);
    }
    blocking_check(s, "per-gate kernel");
}

// Kernel layout per encoding: fixed lane bits F (128-byte lines for the
// state vector; 64-byte runs of each code plane) and register bits K.
// Compact states fuse only in per-block quantisation mode.
PlanConfig plan_config(int n, int enc, const jq_exec_opts* opts) {
    PlanConfig c;
    c.n = n;
    const bool compact = enc == JQ_COMPACT;
    c.fixed_lane_bits = compact ? kCpFixedLaneBits : enc == JQ_C64 ? 4 : 3;
    const int k_max = compact ? 4 : enc == JQ_C64 ? 6 : 5;
    c.max_ops = 48;
    c.fuse = true;
    // register width and a pass's streaming time over one op's arithmetic:
    // tuned per device, encoding and N, else the defaults measured at N = 30
    // (4.3 ms against 0.23 ms per op for complex128, 1.25 ms against 0.20 ms
    // for complex64: half the bytes, as many instructions per op); the
    // two-byte code's decoding passes are taken as complex128's
    const jq_tuning tune = compact ? default_tuning(JQ_C128) : tuned_for(n, enc);
    c.k_reg = compact ? 4 : tune.k_reg;
    c.k_general_max = compact ? 0 : enc == JQ_C64 ? 5 : 4;
    c.pass_ops = tune.pass_ops;
    c.table_elem = enc == JQ_C64 ? 4 : 8;
    // the tile-slot search costs about 0.1 ms of host time per pass: worth
    // it once a pass streams 2 GiB or more
    c.search_rounds = std::ldexp((double)bytes_per_amp(enc), n) >= std::ldexp(1.0, 30) ? 2 : 0;
    if (tune.search == JQ_SEARCH_ON) c.search_rounds = 2;
    else if (tune.search == JQ_SEARCH_OFF) c.search_rounds = 0;
    // two-byte code, per-gate quantisation (the default): code-domain passes
    c.code_domain = compact;
    if (opts) {
        if (opts->compact_mode != JQ_COMPACT_PER_GATE && opts->compact_mode != JQ_COMPACT_PER_BLOCK)
            fail(JQ_EINVAL, "jq_exec_opts: bad compact_mode");
        if (compact && opts->compact_mode == JQ_COMPACT_PER_BLOCK) c.code_domain = false;
        if (opts->fusion == 1) c.fuse = false;
        else if (opts->fusion >= 2) c.k_reg = std::min(opts->fusion, c.code_domain ? 7 : k_max), c.k_explicit = true;
        if (opts->max_ops > 0) c.max_ops = std::min(opts->max_ops, 256);
        if (opts->search == JQ_SEARCH_ON) c.search_rounds = 2;
        else if (opts->search == JQ_SEARCH_OFF) c.search_rounds = 0;
        else if (opts->search != JQ_SEARCH_AUTO) fail(JQ_EINVAL, "jq_exec_opts: bad search");
        for (int r : opts->reserved)
            if (r != 0) fail(JQ_EINVAL, "jq_exec_opts: reserved fields must be zero");
    }
    if (c.code_domain) {
        c.absorb = false;
        c.fixed_reg_bits = kCpCodeRegBits;
        // code passes: 0.83 ms per pass against 0.0054 ms per op
        c.pass_ops = 150.0;
        if (!(opts && opts->fusion >= 2)) c.k_reg = 7;
    }
    if (debug_flags().force == 1) c.fuse = false;
    else if (debug_flags().force == 2) c.always_pass = true;
    while (c.fuse && c.k_reg > 2 && c.n < 6 + c.k_reg) c.k_reg--;
    return c;
}

PlanConfig plan_config_tuned(int n, int enc, int k_reg, double pass_ops) {
    PlanConfig c = plan_config(n, enc, nullptr);
    c.k_reg = k_reg;
    c.pass_ops = pass_ops;
    // the size rule for the large-state steps, whatever is tuned now
    c.search_rounds = std::ldexp((double)bytes_per_amp(enc), n) >= std::ldexp(1.0, 30) ? 2 : 0;
    while (c.fuse && c.k_reg > 2 && c.n < 6 + c.k_reg) c.k_reg--;
    return c;
}

// Copy the fused-op list of a state with stream-ordered allocation to the
// device (its buffer is reused in stream order, after every kernel that read
// the previous plan).
void upload_fops(jq_state* s, const std::vector<FOp>& fops) {
    const size_t bytes = fops.size() * sizeof(FOp);
    if (bytes == 0) return;
    if (bytes > s->plan_dev_bytes) {
        if (s->plan_dev) JQ_HIP(hipFreeAsync(s->plan_dev, s->stream));
        s->plan_dev = nullptr;
        JQ_HIP(hipMallocAsync(&s->plan_dev, bytes, s->stream));
        s->plan_dev_bytes = bytes;
    }
    // pageable source: the runtime stages it before the call returns
    JQ_HIP(hipMemcpyAsync(s->plan_dev, fops.data(), bytes, hipMemcpyHostToDevice, s->stream));
}

// Copy n fused ops into the ring and return their device address.  A copy
// runs in stream order, after every kernel that read the slots before, so
// only the pinned staging needs a wait: slots whose earlier copy has not yet
// run are not written until it has.
const FOp* ring_put(jq_state* s, const FOp* src, size_t n) {
    const size_t cap = s->plan_dev_bytes / sizeof(FOp);
    if (n > cap) {
        JQ_HIP(hipStreamSynchronize(s->stream));
        for (auto& u : s->ring_busy) s->ring_ev_free.push_back(u.ev);
        s->ring_busy.clear();
        if (s->plan_dev) JQ_HIP(hipFree(s->plan_dev));
        if (s->plan_host) JQ_HIP(hipHostFree(s->plan_host));
        s->plan_dev = nullptr;
        s->plan_host = nullptr;
        s->plan_dev_bytes = 0;
        const size_t bytes = std::max<size_t>(1024, 4 * n) * sizeof(FOp);
        JQ_HIP(hipMalloc(&s->plan_dev, bytes));
        JQ_HIP(hipHostMalloc(&s->plan_host, bytes, hipHostMallocDefault));
        s->plan_dev_bytes = bytes;
        s->ring_head = 0;
        return ring_put(s, src, n);
    }
    size_t off = s->ring_head;
    if (off + n > cap) off = 0;
    // the newest pending copy out of [off, off + n); the older ones have
    // run once it has
    size_t last = 0;
    for (size_t i = 0; i < s->ring_busy.size(); ++i) {
        const auto& u = s->ring_busy[i];
        if (u.off < off + n && off < u.off + u.n) last = i + 1;
    }
    if (last) JQ_HIP(hipEventSynchronize(s->ring_busy[last - 1].ev));
    for (size_t i = 0; i < last; ++i) {
        s->ring_ev_free.push_back(s->ring_busy.front().ev);
        s->ring_busy.pop_front();
    }
    FOp* host = static_cast<FOp*>(s->plan_host) + off;
    FOp* dev = static_cast<FOp*>(s->plan_dev) + off;
    std::memcpy(host, src, n * sizeof(FOp));
    JQ_HIP(hipMemcpyAsync(dev, host, n * sizeof(FOp), hipMemcpyHostToDevice, s->stream));
    hipEvent_t ev;
    if (s->ring_ev_free.empty()) {
        JQ_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    } else {
        ev = s->ring_ev_free.back();
        s->ring_ev_free.pop_back();
    }
    JQ_HIP(hipEventRecord(ev, s->stream));
    s->ring_busy.push_back({off, n, ev});
    s->ring_head = off + n;
    return dev;
}

void run_step(jq_state* s, const std::vector<GateOp>& ops, const PlanConfig& cfg, const Step& step,
              const FOp* dev_ops) {
    if (!step.fused) {
        run_single(s, step.op);
        return;
    }
    const double sweep = std::ldexp(1.0, s->n) * bytes_per_amp(s->enc);
    FPass p = step.pass;
    p.ops = dev_ops;
    Range r([&] {
        std::string q;
        for (int j = 0; j < step.k_reg; ++j) q += (j ? "," : "") + std::to_string(p.reg_q[j]);
        return "fused pass: " + std::to_string(p.n_ops) + " ops, " + std::to_string(step.n_gates) +
               " gates, register qubits " + q;
    });
    if (s->enc == JQ_COMPACT && cfg.code_domain) {
        {
            Timed t(s, K_CP_CODES, 2.0 * sweep);
            cp_apply_codes(compact_bufs(s), s->n, p, step.k_reg, cfg.fixed_reg_bits, s->stream);
        }
        blocking_check(s, "two-byte code pass");
        return;
    }
    if (s->enc == JQ_COMPACT) {
        bool keeps = true;
        for (int g : step.gates) keeps = keeps && ops[g].keeps_modulus;
        {
            Timed t(s, K_CP_FUSED, (keeps ? 2.0 : 3.0) * sweep);
            cp_apply_block(compact_bufs(s), s->n, p, step.k_reg, cfg.fixed_lane_bits, keeps, s->stream);
        }
        blocking_check(s, "two-byte fused block");
        return;
    }
    {
        Timed t(s, K_FUSED, 2.0 * sweep);
        if (debug_flags().fused_all_kinds) p.kinds = 0;  // kinds not recorded: the general loop
        sv_apply_fused(s->enc, s->buf, s->n, p, step.k_reg, cfg.fixed_lane_bits, s->stream);
    }
    blocking_check(s, "fused pass");
}

void apply_ops(jq_state* s, const std::vector<GateOp>& ops, const PlanConfig& cfg) {
    if (s->async_alloc) {
        // served states: plan, upload, launch
        Plan plan = make_plan(ops, cfg);
        upload_fops(s, plan.fops);
        const FOp* dev = (const FOp*)s->plan_dev;
        for (const auto& step : plan.steps) run_step(s, ops, cfg, step, dev + step.first_fop);
        return;
    }
    // Launch steps while the rest is planned: the first fused pass as soon
    // as it is planned, then every few passes, so the device is busy while
    // the host plans.
    size_t launched = 0, uploaded = 0, flushes = 0;
    auto flush = [&](Plan& plan) {
        const size_t n = plan.fops.size() - uploaded;
        const FOp* dev = n ? ring_put(s, plan.fops.data() + uploaded, n) : nullptr;
        for (; launched < plan.steps.size(); ++launched) {
            const Step& st = plan.steps[launched];
            run_step(s, ops, cfg, st, st.fused ? dev + (st.first_fop - uploaded) : nullptr);
        }
        uploaded = plan.fops.size();
        ++flushes;
    };
    Plan plan = make_plan(ops, cfg, [&](Plan& pl) {
        size_t waiting = 0;
        for (size_t i = launched; i < pl.steps.size(); ++i) waiting += pl.steps[i].fused;
        if (waiting >= (flushes ? 4u : 1u) || !pl.steps.back().fused) flush(pl);
    });
    if (launched < plan.steps.size()) flush(plan);
}

// ------------------------------------------ allocation-free circuits --

// Fused-op workspace of jq_apply_circuit_noalloc: one fixed array per GPU,
// held until the process ends.  In host code its name is only a stand-in;
// the device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[JQ_NOALLOC_WORKSPACE_BYTES];

// the header states the size of a fused op and how many the workspace holds
static_assert(sizeof(FOp) == 704, "jq.h documents 704-byte fused ops");

constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
void* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];

// The workspace's address on device dev, which must be the current device.
FOp* noalloc_workspace(int dev) {
    if (dev < 0 || dev >= kMaxDevices) fail(JQ_EDEVICE, "jq_apply_circuit_noalloc: device index out of range");
    std::call_once(g_scratch_once[dev], [dev] {
        void* p = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = p;
    });
    if (g_scratch_err[dev] != hipSuccess || !g_scratch_ptr[dev])
        fail(JQ_EDEVICE, std::string("jq_apply_circuit_noalloc: hipGetSymbolAddress: ") +
                             hipGetErrorString(g_scratch_err[dev]));
    return static_cast<FOp*>(g_scratch_ptr[dev]);
}

// The whole plan first, then one copy of its fused ops into the workspace
// and the launches; per-launch timing is skipped (it would create events).
void apply_ops_noalloc(jq_state* s, const std::vector<GateOp>& ops, const PlanConfig& cfg) {
    int dev = -1;
    JQ_HIP(hipGetDevice(&dev));
    if (dev != s->device) fail(JQ_EINVAL, "jq_apply_circuit_noalloc: the state's device must be current");
    FOp* ws = noalloc_workspace(dev);
    const Plan plan = make_plan(ops, cfg);
    const size_t bytes = plan.fops.size() * sizeof(FOp);
    if (bytes > JQ_NOALLOC_WORKSPACE_BYTES)
        fail(JQ_EINVAL, "jq_apply_circuit_noalloc: the plan has " + std::to_string(plan.fops.size()) +
                            " fused ops (" + std::to_string(bytes) + " bytes), the workspace holds " +
                            std::to_string(JQ_NOALLOC_WORKSPACE_BYTES / sizeof(FOp)));
    // pageable source: the runtime stages it before the call returns
    if (bytes) JQ_HIP(hipMemcpyAsync(ws, plan.fops.data(), bytes, hipMemcpyHostToDevice, s->stream));
    const bool prof = s->profiling;
    s->profiling = false;
    try {
        for (const auto& step : plan.steps) run_step(s, ops, cfg, step, step.fused ? ws + step.first_fop : nullptr);
    } catch (...) {
        s->profiling = prof;
        throw;
    }
    s->profiling = prof;
}

void do_probabilities(jq_state* s, const int* qubits, int nq, double* out_host) {
    if (nq < 0 || nq > s->n || nq > 30) fail(JQ_EINVAL, "jq_probabilities: bad qubit count");
    if (nq > 0 && !qubits) fail(JQ_EINVAL, "jq_probabilities: null qubits");
    if (!out_host) fail(JQ_EINVAL, "jq_probabilities: null output");
    uint64_t seen = 0;
    for (int m = 0; m < nq; ++m) {
        if (qubits[m] < 0 || qubits[m] >= s->n) fail(JQ_EINVAL, "jq_probabilities: qubit out of range");
        if (seen & (1ull << qubits[m])) fail(JQ_EINVAL, "jq_probabilities: repeated qubit");
        seen |= 1ull << qubits[m];
    }
    const size_t nbins = 1ull << nq;
    const size_t cap = std::max<size_t>(16384, 2 * nbins);
    double* scratch = partials(s, nbins + cap);
    double* out_dev = scratch;
    double* part = scratch + nbins;
    {
        Timed t(s, K_REDUCE, std::ldexp(1.0, s->n) * (s->enc == JQ_COMPACT ? 1 : bytes_per_amp(s->enc)));
        if (s->enc == JQ_COMPACT) cp_probabilities(compact_bufs(s), s->n, qubits, nq, out_dev, part, cap, s->stream);
        else sv_probabilities(s->enc, s->buf, s->n, qubits, nq, out_dev, part, cap, s->stream);
    }
    JQ_HIP(hipMemcpyAsync(out_host, out_dev, nbins * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    JQ_HIP(hipStreamSynchronize(s->stream));
}

jq_state* state_create(int n, int enc, hipStream_t stream, bool async_alloc) {
    if (n < 1 || n > JQ_MAX_QUBITS) fail(JQ_EINVAL, "jq_state_create: N must be in [1, 63]");
    if (enc != JQ_C128 && enc != JQ_C64 && enc != JQ_COMPACT) fail(JQ_EINVAL, "jq_state_create: bad encoding");
    const int bpa = bytes_per_amp(enc);
    if (n > 61) fail(JQ_ENOMEM, "jq_state_create: 2^N amplitudes cannot be addressed");
    const uint64_t bytes = (uint64_t)bpa << n;
    size_t free_b = 0, total_b = 0;
    JQ_HIP(hipMemGetInfo(&free_b, &total_b));
    if (bytes > free_b)
        fail(JQ_ENOMEM, "jq_state_create: state needs " + std::to_string(bytes) + " bytes, " +
                            std::to_string(free_b) + " free");
    auto s = new jq_state();
    s->n = n;
    s->enc = enc;
    s->bytes = bytes;
    s->async_alloc = async_alloc;
    JQ_HIP(hipGetDevice(&s->device));
    if (!async_alloc) {
        std::lock_guard<std::mutex> lk(g_hooks_mu);
        s->alloc = g_hooks.alloc;
        s->release = g_hooks.release;
        s->alloc_ctx = g_hooks.ctx;
    }
    try {
        if (stream) {
            s->stream = stream;
        } else {
            JQ_HIP(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
            s->own_stream = true;
        }
        s->aux_doubles = kAuxHead + 16384 + 64;
        if (async_alloc) {
            JQ_HIP(hipMallocAsync(&s->buf, bytes, s->stream));
            JQ_HIP(hipMallocAsync((void**)&s->aux, s->aux_doubles * sizeof(double), s->stream));
        } else {
            if (s->alloc) {
                s->buf = s->alloc(bytes, s->alloc_ctx);
                if (!s->buf) fail(JQ_ENOMEM, "jq_state_create: allocator returned null");
            } else {
                JQ_HIP(hipMalloc(&s->buf, bytes));
            }
            JQ_HIP(hipMalloc(&s->aux, s->aux_doubles * sizeof(double)));
        }
        if (enc == JQ_COMPACT) cp_init(compact_bufs(s), n, JQ_INIT_ZERO, 0, s->stream);
        else sv_init(enc, s->buf, n, JQ_INIT_ZERO, 0, s->stream);
    } catch (...) {
        if (s->async_alloc) {
            if (s->buf) (void)hipFreeAsync(s->buf, s->stream);
            if (s->aux) (void)hipFreeAsync(s->aux, s->stream);
        } else {
            if (s->buf) {
                if (s->release) s->release(s->buf, s->alloc_ctx);
                else (void)hipFree(s->buf);
            }
            if (s->aux) (void)hipFree(s->aux);
        }
        if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
        delete s;
        throw;
    }
    return s;
}

void state_apply(jq_state* s, const std::vector<GateOp>& ops, const jq_exec_opts* opts) {
    apply_ops(s, ops, plan_config(s->n, s->enc, opts));
}

void state_apply_config(jq_state* s, const std::vector<GateOp>& ops, const PlanConfig& cfg) {
    apply_ops(s, ops, cfg);
}

void state_norm_async(jq_state* s, double* pinned_out) {
    const size_t cap = 16384;
    double* scratch = partials(s, 1 + cap);
    if (s->enc == JQ_COMPACT) cp_probabilities(compact_bufs(s), s->n, nullptr, 0, scratch, scratch + 1, cap, s->stream);
    else sv_probabilities(s->enc, s->buf, s->n, nullptr, 0, scratch, scratch + 1, cap, s->stream);
    JQ_HIP(hipMemcpyAsync(pinned_out, scratch, sizeof(double), hipMemcpyDeviceToHost, s->stream));
}


// f |v><v| on qubit q as a diagonal op (entry v = f, the other entry 0)
GateOp projector(int n, int q, int v, double f) {
    jq_gate g;
    std::memset(&g, 0, sizeof(g));
    g.kind = JQ_DIAGONAL;
    g.nq = 1;
    g.qubits[0] = q;
    g.m[2 * v] = f;
    return canonicalize(g, n);
}

void check_qubit(const jq_state* s, int q, const char* who) {
    if (q < 0 || q >= s->n) fail(JQ_EINVAL, std::string(who) + ": qubit out of range");
}

// Host-only planning of a circuit for the schedule and step reports:
// validates, lowers, and plans; src[k] is the input index of op k.
Plan plan_host(const char* who, int n_qubits, int enc, const jq_gate* gates, size_t count,
               const jq_exec_opts* opts, std::vector<int32_t>* src_out) {
    const std::string w(who);
    if (n_qubits < 1 || n_qubits > JQ_MAX_QUBITS) fail(JQ_EINVAL, w + ": N must be in [1, 63]");
    if (enc != JQ_C128 && enc != JQ_C64 && enc != JQ_COMPACT) fail(JQ_EINVAL, w + ": bad encoding");
    if (count && !gates) fail(JQ_EINVAL, w + ": null gates");
    std::vector<GateOp> ops;
    std::vector<int32_t> src;
    for (size_t i = 0; i < count; ++i) {
        if (gates[i].nq == 0) continue;  // identity
        try {
            ops.push_back(canonicalize(gates[i], n_qubits));
        } catch (const Error& e) {
            fail(e.code, "gate " + std::to_string(i) + ": " + e.what());
        }
        src.push_back((int32_t)i);
    }
    if (src_out) *src_out = std::move(src);
    return make_plan(ops, plan_config(n_qubits, enc, opts));
}

}  // namespace jq

using namespace jq;

// ================================================================ ABI ==

extern "C" {

const char* jq_last_error(void) { return jq::g_last_error.c_str(); }

const char* jq_version(void) { return "jq 0.1 (gfx950)"; }

int jq_set_allocator(void* (*alloc)(size_t, void*), void (*release)(void*, void*), void* ctx) {
    return guarded([&] {
        if ((alloc == nullptr) != (release == nullptr)) fail(JQ_EINVAL, "jq_set_allocator: give both or neither");
        std::lock_guard<std::mutex> lk(g_hooks_mu);
        g_hooks.alloc = alloc;
        g_hooks.release = release;
        g_hooks.ctx = ctx;
    });
}

int jq_state_create(int n, jq_encoding enc, jq_state** out) {
    return guarded([&] {
        if (!out) fail(JQ_EINVAL, "jq_state_create: null output");
        *out = nullptr;
        *out = state_create(n, enc, nullptr, false);
    });
}

int jq_state_destroy(jq_state* s) {
    return guarded([&] {
        check_state(s);
        if (s->async_alloc) {
            // stream-ordered: memory returns to the pool after the queued work
            for (auto& r : s->recs) {
                (void)hipEventDestroy(r.a);
                (void)hipEventDestroy(r.b);
            }
            for (auto ev : s->event_pool) (void)hipEventDestroy(ev);
            if (s->buf) (void)hipFreeAsync(s->buf, s->stream);
            if (s->aux) (void)hipFreeAsync(s->aux, s->stream);
            if (s->plan_dev) (void)hipFreeAsync(s->plan_dev, s->stream);
            delete s;
            return;
        }
        hipError_t e = hipStreamSynchronize(s->stream);
        for (auto& r : s->recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto ev : s->event_pool) (void)hipEventDestroy(ev);
        if (s->buf) {
            if (s->release) s->release(s->buf, s->alloc_ctx);
            else (void)hipFree(s->buf);
        }
        if (s->aux) (void)hipFree(s->aux);
        if (s->plan_dev) (void)hipFree(s->plan_dev);
        if (s->plan_host) (void)hipHostFree(s->plan_host);
        for (auto& u : s->ring_busy) (void)hipEventDestroy(u.ev);
        for (auto ev : s->ring_ev_free) (void)hipEventDestroy(ev);
        if (s->own_stream) (void)hipStreamDestroy(s->stream);
        delete s;
        hip_check(e, "jq_state_destroy: pending work failed");
    });
}

int jq_state_init(jq_state* s, jq_init mode, uint64_t basis) {
    return guarded([&] {
        check_state(s);
        if (mode != JQ_INIT_ZERO && mode != JQ_INIT_UNIFORM && mode != JQ_INIT_BASIS)
            fail(JQ_EINVAL, "jq_state_init: bad mode");
        if (mode == JQ_INIT_BASIS && basis >= (1ull << s->n)) fail(JQ_EINVAL, "jq_state_init: basis out of range");
        const uint64_t b = mode == JQ_INIT_BASIS ? basis : 0;
        if (s->enc == JQ_COMPACT) cp_init(compact_bufs(s), s->n, mode == JQ_INIT_UNIFORM ? 1 : 2, b, s->stream);
        else sv_init(s->enc, s->buf, s->n, mode == JQ_INIT_UNIFORM ? JQ_INIT_UNIFORM : JQ_INIT_BASIS, b, s->stream);
    });
}

int jq_shorbox(jq_state* s, int n_x, uint64_t G, uint64_t y) {
    return guarded([&] {
        check_state(s);
        if (n_x < 1 || n_x >= s->n || n_x > 40) fail(JQ_EINVAL, "jq_shorbox: need 1 <= n_x < N and n_x <= 40");
        if (G < 2 || G >= (1ull << 32)) fail(JQ_EINVAL, "jq_shorbox: need 2 <= G < 2^32");
        if (s->n - n_x < 64 && G > (1ull << (s->n - n_x)))
            fail(JQ_EINVAL, "jq_shorbox: the f-register cannot hold values up to G - 1");
        if (y <= 1 || y >= G) fail(JQ_EINVAL, "jq_shorbox: need 1 < y < G");
        if (s->enc == JQ_COMPACT) cp_shorbox(compact_bufs(s), s->n, n_x, G, y, s->stream);
        else sv_shorbox(s->enc, s->buf, s->n, n_x, G, y, s->stream);
    });
}

int jq_state_info(const jq_state* s, int* n, int* enc, uint64_t* bytes) {
    return guarded([&] {
        check_state(s);
        if (n) *n = s->n;
        if (enc) *enc = s->enc;
        if (bytes) *bytes = s->bytes;
    });
}

int jq_state_device_ptr(const jq_state* s, void** ptr) {
    return guarded([&] {
        check_state(s);
        if (!ptr) fail(JQ_EINVAL, "null output");
        *ptr = s->buf;
    });
}

int jq_set_stream(jq_state* s, void* stream) {
    return guarded([&] {
        check_state(s);
        hipStream_t ns = (hipStream_t)stream;
        if (ns == s->stream) return;
        // order the new stream after the work already queued on the old one
        hipEvent_t ev;
        JQ_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        JQ_HIP(hipEventRecord(ev, s->stream));
        if (!ns) {
            if (!s->own_stream) {
                JQ_HIP(hipStreamCreateWithFlags(&ns, hipStreamNonBlocking));
                s->own_stream = true;
            } else {
                (void)hipEventDestroy(ev);
                return;
            }
        } else if (s->own_stream) {
            JQ_HIP(hipStreamWaitEvent(ns, ev, 0));
            JQ_HIP(hipStreamSynchronize(s->stream));
            JQ_HIP(hipStreamDestroy(s->stream));
            s->own_stream = false;
        }
        JQ_HIP(hipStreamWaitEvent(ns, ev, 0));
        JQ_HIP(hipEventDestroy(ev));
        s->stream = ns;
    });
}

int jq_synchronize(jq_state* s) {
    return guarded([&] {
        check_state(s);
        JQ_HIP(hipStreamSynchronize(s->stream));
    });
}

int jq_gate_named(const char* name, const int* qubits, int nq, const double* params, int np, jq_gate* out) {
    return guarded([&] { gate_named(name, qubits, nq, params, np, out); });
}

int jq_gates_named(size_t count, const char* const* names, const int* nq, const int* qubits, const int* np,
                   const double* params, const int* nc, const int* controls, jq_gate* out) {
    return guarded([&] {
        if (count > 0 && (!names || !nq || !np || !out)) fail(JQ_EINVAL, "jq_gates_named: null argument");
        size_t qo = 0, po = 0, co = 0;
        for (size_t i = 0; i < count; ++i) {
            const std::string at = "jq_gates_named: instruction " + std::to_string(i) + ": ";
            const int k = nc ? nc[i] : 0;
            if (nq[i] < 0 || np[i] < 0 || k < 0) fail(JQ_EINVAL, at + "negative count");
            if ((nq[i] > 0 && !qubits) || (np[i] > 0 && !params) || (k > 0 && !controls))
                fail(JQ_EINVAL, at + "null argument");
            try {
                gate_named(names[i], nq[i] ? qubits + qo : nullptr, nq[i], np[i] ? params + po : nullptr, np[i],
                           &out[i]);
            } catch (const Error& e) {
                fail(e.code, at + e.what());
            }
            if (out[i].nc + k > JQ_MAX_CONTROLS) fail(JQ_EINVAL, at + "too many controls");
            for (int c = 0; c < k; ++c) out[i].controls[out[i].nc++] = controls[co + c];
            qo += (size_t)nq[i];
            po += (size_t)np[i];
            co += (size_t)k;
        }
    });
}

int jq_apply_gate(jq_state* s, int kind, const int* qubits, int nq, const int* controls, int nc,
                  const double* matrix) {
    return guarded([&] {
        check_state(s);
        if (nq < 1 || nq > 2 || !qubits) fail(JQ_EINVAL, "jq_apply_gate: need 1 or 2 qubits");
        if (nc < 0 || nc > JQ_MAX_CONTROLS || (nc > 0 && !controls)) fail(JQ_EINVAL, "jq_apply_gate: bad controls");
        jq_gate g;
        std::memset(&g, 0, sizeof(g));
        g.kind = kind;
        g.nq = nq;
        g.nc = nc;
        for (int i = 0; i < nq; ++i) g.qubits[i] = qubits[i];
        for (int i = 0; i < nc; ++i) g.controls[i] = controls[i];
        if (kind == JQ_DENSE || kind == JQ_DIAGONAL) {
            if (!matrix) fail(JQ_EINVAL, "jq_apply_gate: null matrix");
            const int entries = kind == JQ_DENSE ? (1 << nq) * (1 << nq) : (1 << nq);
            for (int i = 0; i < 2 * entries; ++i) g.m[i] = matrix[i];
        }
        run_single(s, canonicalize(g, s->n));
    });
}

int jq_apply_circuit(jq_state* s, const jq_gate* gates, size_t count, const jq_exec_opts* opts) {
    return guarded([&] {
        check_state(s);
        Range r([&] {
            return "jq_apply_circuit n=" + std::to_string(s->n) + " gates=" + std::to_string(count);
        });
        const std::vector<GateOp> ops = lower_circuit(s, gates, count, "jq_apply_circuit");
        apply_ops(s, ops, plan_config(s->n, s->enc, opts));  // options validated before any work
    });
}

int jq_apply_circuit_noalloc(jq_state* s, const jq_gate* gates, size_t count, const jq_exec_opts* opts) {
    return guarded([&] {
        check_state(s);
        const std::vector<GateOp> ops = lower_circuit(s, gates, count, "jq_apply_circuit_noalloc");
        apply_ops_noalloc(s, ops, plan_config(s->n, s->enc, opts));
    });
}

int jq_apply_circuit_noisy(jq_state* s, const jq_gate* gates, size_t count, double px, double py, double pz,
                           const double* u, const jq_exec_opts* opts) {
    return guarded([&] {
        check_state(s);
        if (count && (!gates || !u)) fail(JQ_EINVAL, "jq_apply_circuit_noisy: null array");
        if (!(px >= 0.0 && py >= 0.0 && pz >= 0.0 && px + py + pz <= 1.0 + 1e-12))
            fail(JQ_EINVAL, "jq_apply_circuit_noisy: need p_x, p_y, p_z >= 0 with sum <= 1");
        const int n = s->n;
        // the channel's Pauli gates (App. A matrices), lowered once per qubit
        std::vector<GateOp> pauli[3];
        const char* names[3] = {"X", "Y", "Z"};
        for (int k = 0; k < 3; ++k)
            for (int q = 0; q < n; ++q) {
                jq_gate g;
                gate_named(names[k], &q, 1, nullptr, 0, &g);
                pauli[k].push_back(canonicalize(g, n));
            }
        std::vector<GateOp> ops;
        ops.reserve(count * 2);
        for (size_t i = 0; i < count; ++i) {
            if (gates[i].nq != 0) {
                try {
                    ops.push_back(canonicalize(gates[i], n));
                } catch (const Error& e) {
                    fail(e.code, "gate " + std::to_string(i) + ": " + e.what());
                }
            }
            for (int q = 0; q < n; ++q) {
                const double x = u[i * (size_t)n + q];
                if (!(x >= 0.0 && x < 1.0)) fail(JQ_EINVAL, "jq_apply_circuit_noisy: draws must lie in [0, 1)");
                if (x < px) ops.push_back(pauli[0][q]);
                else if (x < px + py) ops.push_back(pauli[1][q]);
                else if (x < px + py + pz) ops.push_back(pauli[2][q]);
            }
        }
        apply_ops(s, ops, plan_config(s->n, s->enc, opts));
    });
}

int jq_sample(jq_state* s, const double* u, size_t count, uint64_t* out) {
    return guarded([&] {
        check_state(s);
        if (count && (!u || !out)) fail(JQ_EINVAL, "jq_sample: null array");
        if (s->n > 43) fail(JQ_EUNSUPPORTED, "jq_sample: more than 2^43 amplitudes");
        for (size_t k = 0; k < count; ++k)
            if (!(u[k] >= 0.0 && u[k] < 1.0)) fail(JQ_EINVAL, "jq_sample: draws must lie in [0, 1)");
        if (count == 0) return;
        // zero state check from the FP64 norm (the sampler needs a positive total)
        double nrm = 0.0;
        {
            const int none = 0;
            double p[1];
            do_probabilities(s, &none, 0, p);
            nrm = p[0];
        }
        if (!(nrm > 0.0)) fail(JQ_EZERO, "jq_sample: zero state");
        const size_t work = sample_scratch_doubles(s->n);
        const size_t batch = std::min<size_t>(count, 1u << 20);  // draws per round trip
        double* scratch = partials(s, work + 2 * batch);
        double* u_dev = scratch + work;
        uint64_t* out_dev = reinterpret_cast<uint64_t*>(u_dev + batch);
        for (size_t first = 0; first < count; first += batch) {
            const size_t c = std::min(batch, count - first);
            JQ_HIP(hipMemcpyAsync(u_dev, u + first, c * sizeof(double), hipMemcpyHostToDevice, s->stream));
            {
                Timed t(s, K_REDUCE, std::ldexp(1.0, s->n) * (s->enc == JQ_COMPACT ? 1 : bytes_per_amp(s->enc)));
                if (s->enc == JQ_COMPACT) cp_sample(compact_bufs(s), s->n, u_dev, c, out_dev, scratch, s->stream);
                else sv_sample(s->enc, s->buf, s->n, u_dev, c, out_dev, scratch, s->stream);
            }
            JQ_HIP(hipMemcpyAsync(out + first, out_dev, c * sizeof(uint64_t), hipMemcpyDeviceToHost, s->stream));
            JQ_HIP(hipStreamSynchronize(s->stream));
        }
    });
}

int jq_project(jq_state* s, int qubit, int value, double* p_out) {
    return guarded([&] {
        check_state(s);
        check_qubit(s, qubit, "jq_project");
        if (value != 0 && value != 1) fail(JQ_EINVAL, "jq_project: value must be 0 or 1");
        double p[2];
        do_probabilities(s, &qubit, 1, p);
        if (p_out) *p_out = p[value];
        if (!(p[value] > 0.0)) fail(JQ_EZERO, "jq_project: the projection leaves no amplitude");
        run_single(s, projector(s->n, qubit, value, 1.0 / std::sqrt(p[value])));
    });
}

int jq_measure(jq_state* s, int qubit, double u, int* outcome, double* p1_out) {
    return guarded([&] {
        check_state(s);
        check_qubit(s, qubit, "jq_measure");
        if (!(u >= 0.0 && u < 1.0)) fail(JQ_EINVAL, "jq_measure: u must lie in [0, 1)");
        if (!outcome) fail(JQ_EINVAL, "jq_measure: null outcome");
        double p[2];
        do_probabilities(s, &qubit, 1, p);
        const double tot = p[0] + p[1];
        if (!(tot > 0.0)) fail(JQ_EZERO, "jq_measure: zero state");
        const int o = u >= p[0] / tot ? 1 : 0;
        *outcome = o;
        if (p1_out) *p1_out = p[1] / tot;
        run_single(s, projector(s->n, qubit, o, 1.0 / std::sqrt(p[o])));
    });
}

int jq_plan_steps(int n_qubits, int enc, const jq_gate* gates, size_t count, const jq_exec_opts* opts,
                  jq_plan_step* out, size_t max, size_t* n_steps) {
    return guarded([&] {
        if (!n_steps) fail(JQ_EINVAL, "jq_plan_steps: null n_steps");
        if (max && !out) fail(JQ_EINVAL, "jq_plan_steps: null output");
        const Plan plan = plan_host("jq_plan_steps", n_qubits, enc, gates, count, opts, nullptr);
        for (size_t k = 0; k < plan.steps.size() && k < max; ++k) {
            const Step& st = plan.steps[k];
            jq_plan_step& o = out[k];
            std::memset(&o, 0, sizeof(o));
            o.fused = st.fused ? 1 : 0;
            o.n_gates = (int32_t)st.gates.size();
            for (int j = 0; j < 8; ++j) o.reg_q[j] = -1;
            for (int b = 0; b < 6; ++b) o.lane_q[b] = -1;
            if (!st.fused) continue;
            o.k_reg = st.k_reg;
            for (int j = 0; j < st.k_reg && j < 8; ++j) o.reg_q[j] = st.pass.reg_q[j];
            for (int b = 0; b < 6; ++b) o.lane_q[b] = st.pass.lane_q[b];
            o.n_ops = st.pass.n_ops;
            o.table_tag = st.pass.table_tag;
            for (int i = 0; i < st.pass.n_ops; ++i) {
                const FOp& f = plan.fops[st.first_fop + i];
                if (f.kind == F_DGROUP && f.slot != 0) ++o.n_tables;
            }
        }
        *n_steps = plan.steps.size();
    });
}

int jq_plan_schedule(int n_qubits, int enc, const jq_gate* gates, size_t count, const jq_exec_opts* opts,
                     int32_t* order, int32_t* block_len, int32_t* block_fused, size_t* n_blocks) {
    return guarded([&] {
        if (!n_blocks) fail(JQ_EINVAL, "jq_plan_schedule: null n_blocks");
        if (count && (!gates || !order || !block_len)) fail(JQ_EINVAL, "jq_plan_schedule: null array");
        std::vector<int32_t> src;
        const Plan plan = plan_host("jq_plan_schedule", n_qubits, enc, gates, count, opts, &src);
        size_t k = 0, b = 0;
        for (const auto& step : plan.steps) {
            for (int g : step.gates) order[k++] = src[g];
            block_len[b] = (int32_t)step.gates.size();
            if (block_fused) block_fused[b] = step.fused ? 1 : 0;
            ++b;
        }
        *n_blocks = b;
    });
}

int jq_norm(jq_state* s, double* out) {
    return guarded([&] {
        check_state(s);
        if (!out) fail(JQ_EINVAL, "jq_norm: null output");
        do_probabilities(s, nullptr, 0, out);
    });
}

int jq_probabilities(jq_state* s, const int* qubits, int nq, double* out) {
    return guarded([&] {
        check_state(s);
        do_probabilities(s, qubits, nq, out);
    });
}

int jq_expectations(jq_state* s, double* qx, double* qy, double* qz) {
    return guarded([&] {
        check_state(s);
        const int n = s->n;
        const size_t cap = 8192;
        double* scratch = partials(s, 3 * (size_t)n + cap);
        {
            Timed t(s, K_REDUCE, (double)n * std::ldexp(1.0, n) * bytes_per_amp(s->enc));
            if (s->enc == JQ_COMPACT) cp_expectations(compact_bufs(s), n, scratch, scratch + 3 * n, cap, s->stream);
            else sv_expectations(s->enc, s->buf, n, scratch, scratch + 3 * n, cap, s->stream);
        }
        std::vector<double> h(3 * (size_t)n);
        JQ_HIP(hipMemcpyAsync(h.data(), scratch, h.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        JQ_HIP(hipStreamSynchronize(s->stream));
        for (int q = 0; q < n; ++q) {
            if (qx) qx[q] = h[q];
            if (qy) qy[q] = h[n + q];
            if (qz) qz[q] = h[2 * n + q];
        }
    });
}

int jq_renormalize(jq_state* s) {
    return guarded([&] {
        check_state(s);
        double nrm = 0.0;
        do_probabilities(s, nullptr, 0, &nrm);
        if (!(nrm > 0.0)) fail(JQ_EZERO, "jq_renormalize: zero norm");
        const double f = 1.0 / std::sqrt(nrm);
        if (s->enc == JQ_COMPACT) cp_scale_range(compact_bufs(s), f, s->stream);
        else sv_scale(s->enc, s->buf, s->n, f, s->stream);
    });
}

int jq_read_amplitudes(jq_state* s, uint64_t first, uint64_t count, double* out) {
    return guarded([&] {
        check_state(s);
        const uint64_t dim = 1ull << s->n;
        if (first > dim || count > dim - first) fail(JQ_EINVAL, "jq_read_amplitudes: range out of bounds");
        if (count && !out) fail(JQ_EINVAL, "jq_read_amplitudes: null output");
        if (s->enc == JQ_C128) {
            JQ_HIP(hipMemcpyAsync(out, (const double*)s->buf + 2 * first, count * 16, hipMemcpyDeviceToHost, s->stream));
            JQ_HIP(hipStreamSynchronize(s->stream));
            return;
        }
        const uint64_t chunk = 1ull << 22;
        double* tmp = nullptr;
        JQ_HIP(hipMalloc(&tmp, std::min(chunk, std::max<uint64_t>(count, 1)) * 16));
        try {
            for (uint64_t done = 0; done < count; done += chunk) {
                const uint64_t c = std::min(chunk, count - done);
                if (s->enc == JQ_COMPACT) cp_to_c128(compact_bufs(s), s->n, first + done, c, tmp, s->stream);
                else sv_to_c128(s->enc, s->buf, first + done, c, tmp, s->stream);
                JQ_HIP(hipMemcpyAsync(out + 2 * done, tmp, c * 16, hipMemcpyDeviceToHost, s->stream));
                JQ_HIP(hipStreamSynchronize(s->stream));
            }
        } catch (...) {
            (void)hipFree(tmp);
            throw;
        }
        JQ_HIP(hipFree(tmp));
    });
}

int jq_write_amplitudes(jq_state* s, uint64_t first, uint64_t count, const double* in) {
    return guarded([&] {
        check_state(s);
        const uint64_t dim = 1ull << s->n;
        if (first > dim || count > dim - first) fail(JQ_EINVAL, "jq_write_amplitudes: range out of bounds");
        if (count && !in) fail(JQ_EINVAL, "jq_write_amplitudes: null input");
        for (uint64_t i = 0; i < 2 * count; ++i)
            if (!std::isfinite(in[i])) fail(JQ_EINVAL, "jq_write_amplitudes: non-finite value");
        if (s->enc == JQ_C128) {
            JQ_HIP(hipMemcpyAsync((double*)s->buf + 2 * first, in, count * 16, hipMemcpyHostToDevice, s->stream));
            JQ_HIP(hipStreamSynchronize(s->stream));
            return;
        }
        if (s->enc == JQ_COMPACT && (first != 0 || count != dim))
            fail(JQ_EINVAL, "jq_write_amplitudes: the two-byte code takes only a full write");
        double* tmp = nullptr;
        JQ_HIP(hipMalloc(&tmp, std::max<uint64_t>(count, 1) * 16));
        try {
            JQ_HIP(hipMemcpyAsync(tmp, in, count * 16, hipMemcpyHostToDevice, s->stream));
            if (s->enc == JQ_COMPACT) cp_encode_from_c128(compact_bufs(s), s->n, tmp, s->stream);
            else sv_from_c128(s->enc, s->buf, first, count, tmp, s->stream);
            JQ_HIP(hipStreamSynchronize(s->stream));
        } catch (...) {
            (void)hipFree(tmp);
            throw;
        }
        JQ_HIP(hipFree(tmp));
    });
}

int jq_read_codes(jq_state* s, uint64_t first, uint64_t count, int8_t* b0, int8_t* b1, double* range) {
    return guarded([&] {
        check_state(s);
        if (s->enc != JQ_COMPACT) fail(JQ_EINVAL, "jq_read_codes: state is not in the two-byte code");
        const uint64_t dim = 1ull << s->n;
        if (first > dim || count > dim - first) fail(JQ_EINVAL, "jq_read_codes: range out of bounds");
        const int8_t* codes = (const int8_t*)s->buf;
        if (b0) JQ_HIP(hipMemcpyAsync(b0, codes + first, count, hipMemcpyDeviceToHost, s->stream));
        if (b1) JQ_HIP(hipMemcpyAsync(b1, codes + dim + first, count, hipMemcpyDeviceToHost, s->stream));
        if (range) JQ_HIP(hipMemcpyAsync(range, s->aux, 2 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        JQ_HIP(hipStreamSynchronize(s->stream));
    });
}

int jq_write_codes(jq_state* s, const int8_t* b0, const int8_t* b1, const double* range) {
    return guarded([&] {
        check_state(s);
        if (s->enc != JQ_COMPACT) fail(JQ_EINVAL, "jq_write_codes: state is not in the two-byte code");
        if (!b0 || !b1 || !range) fail(JQ_EINVAL, "jq_write_codes: null argument");
        if (!(range[0] >= 0.0 && range[1] >= range[0] && std::isfinite(range[1])))
            fail(JQ_EINVAL, "jq_write_codes: need 0 <= r0 <= r1");
        const uint64_t dim = 1ull << s->n;
        for (uint64_t i = 0; i < dim; ++i)
            if (b0[i] == -128 && b1[i] != 0) fail(JQ_EINVAL, "jq_write_codes: zero amplitude with a phase code");
        int8_t* codes = (int8_t*)s->buf;
        JQ_HIP(hipMemcpyAsync(codes, b0, dim, hipMemcpyHostToDevice, s->stream));
        JQ_HIP(hipMemcpyAsync(codes + dim, b1, dim, hipMemcpyHostToDevice, s->stream));
        JQ_HIP(hipMemcpyAsync(s->aux, range, 2 * sizeof(double), hipMemcpyHostToDevice, s->stream));
        JQ_HIP(hipStreamSynchronize(s->stream));
    });
}

int jq_profile_enable(jq_state* s, int on) {
    return guarded([&] {
        check_state(s);
        if (on) {
            drain_profile(s);
            s->acc.assign(K_NCLASS, jq_state::Acc{});
        } else {
            drain_profile(s);
        }
        s->profiling = on != 0;
    });
}

int jq_profile_read(jq_state* s, jq_kernel_stat* out, int max, int* count) {
    return guarded([&] {
        check_state(s);
        drain_profile(s);
        if (s->acc.size() < K_NCLASS) s->acc.resize(K_NCLASS);
        int c = 0;
        for (int k = 0; k < K_NCLASS; ++k) {
            if (s->acc[k].launches == 0) continue;
            if (out && c < max) {
                std::memset(&out[c], 0, sizeof(jq_kernel_stat));
                std::snprintf(out[c].name, sizeof(out[c].name), "%s", kClassName[k]);
                out[c].launches = s->acc[k].launches;
                out[c].total_ms = s->acc[k].ms;
                out[c].bytes = s->acc[k].bytes;
            }
            ++c;
        }
        if (count) *count = c;
    });
}

}  // extern "C"

// Request loop for circuits of mixed size (continuous batching).
//
// Clients submit circuits from any thread.  A scheduler thread admits
// requests in arrival order whenever the request's state (2^N * bytes per
// amplitude) fits in the remaining HBM budget; a request that does not fit
// lets later, smaller ones pass unless it has waited longer than the
// bypass limit.  An admitted request gets its own state on one of S
// streams (least work in flight first), its gates are planned and launched
// asynchronously, and an event marks its completion, so requests that
// arrive while others run overlap with them on the device.  The state of a
// finished request stays resident, counted against the budget, until the
// client releases it.  The kernels and plans a request runs depend only on
// its circuit, N and encoding, so its result is the same alone and in any
// mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace jq {
namespace {

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point t0, Clock::time_point t1) {
    return std::chrono::duration<double, std::milli>(t1 - t0).count();
}

struct Request {
    uint64_t ticket = 0;
    int n = 0;
    uint64_t bytes = 0;
    std::vector<GateOp> ops;
    Clock::time_point submitted, admitted;
    jq_state* state = nullptr;
    int stream = -1;
    hipEvent_t done = nullptr;
    double* norm = nullptr;  // pinned
    int status = JQ_OK;
};

}  // namespace
}  // namespace jq

struct jq_server {
    uint64_t budget = 0;
    int enc = JQ_C128;
    int queue_cap = 0;
    std::vector<hipStream_t> streams;
    std::vector<int> in_flight_per_stream;
    int device = 0;

    std::mutex mu;
    std::condition_variable cv_sched, cv_done, cv_space;
    bool stop = false;
    std::deque<jq::Request*> queue;
    std::vector<jq::Request*> running;
    std::deque<jq_result> done;
    std::map<uint64_t, jq::Request*> resident;
    uint64_t resident_bytes = 0, peak_bytes = 0;
    uint64_t next_ticket = 1, submitted = 0, completed = 0, rejected = 0;
    std::vector<double> latencies;
    jq::Clock::time_point first_submit, last_done;
    bool any_submit = false;
    double bypass_ms = 50.0;
    std::thread sched;
    // pinned host slots for the FP64 norms (freeing pinned memory per request
    // would synchronise the device)
    double* norms = nullptr;
    std::vector<int> free_norms;
};

namespace jq {
namespace {

void finish(jq_server* sv, Request* r, int status) {
    // called with sv->mu held
    const auto now = Clock::now();
    jq_result res{};
    res.ticket = r->ticket;
    res.status = status;
    res.n_qubits = r->n;
    res.norm = r->norm ? *r->norm : 0.0;
    res.latency_ms = ms_since(r->submitted, now);
    res.queue_ms = ms_since(r->submitted, r->admitted);
    res.state = status == JQ_OK ? r->state : nullptr;
    if (status == JQ_OK) {
        sv->completed++;
        sv->latencies.push_back(res.latency_ms);
        sv->last_done = now;
        sv->resident[r->ticket] = r;
    } else {
        sv->rejected++;
    }
    sv->done.push_back(res);
    sv->cv_done.notify_all();
}

void release_request(jq_server* sv, Request* r) {
    // called with sv->mu held (bytes) — the HIP calls are safe from any thread
    if (r->state) jq_state_destroy(r->state);
    if (r->done) (void)hipEventDestroy(r->done);
    if (r->norm) sv->free_norms.push_back((int)(r->norm - sv->norms));
    sv->resident_bytes -= r->bytes;
    delete r;
}

bool launch(jq_server* sv, Request* r) {
    // outside the lock: allocate, plan and enqueue the request's work
    try {
        jq_state* st = state_create(r->n, sv->enc, sv->streams[r->stream], true);
        r->state = st;
        state_apply(st, r->ops, nullptr);
        *r->norm = 0.0;
        state_norm_async(st, r->norm);
        JQ_HIP(hipEventCreateWithFlags(&r->done, hipEventDisableTiming));
        JQ_HIP(hipEventRecord(r->done, sv->streams[r->stream]));
        return true;
    } catch (const Error& e) {
        r->status = e.code;
        set_last_error(e.what());
        return false;
    }
}

void scheduler(jq_server* sv) {
    JQ_HIP(hipSetDevice(sv->device));
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        // completions
        for (size_t i = 0; i < sv->running.size();) {
            Request* r = sv->running[i];
            const hipError_t q = hipEventQuery(r->done);
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            sv->in_flight_per_stream[r->stream]--;
            sv->running.erase(sv->running.begin() + i);
            finish(sv, r, q == hipSuccess ? JQ_OK : JQ_EDEVICE);
            sv->cv_space.notify_all();
        }
        // admissions, in arrival order with bounded bypass
        bool admitted_any = false;
        const auto now = Clock::now();
        bool head_blocked_long = false;
        for (auto it = sv->queue.begin(); it != sv->queue.end();) {
            Request* r = *it;
            if (sv->resident_bytes + r->bytes > sv->budget) {
                if (it == sv->queue.begin() && ms_since(r->submitted, now) > sv->bypass_ms) head_blocked_long = true;
                if (head_blocked_long) break;
                ++it;
                continue;
            }
            it = sv->queue.erase(it);
            sv->cv_space.notify_all();
            int best = 0;
            for (int s = 1; s < (int)sv->streams.size(); ++s)
                if (sv->in_flight_per_stream[s] < sv->in_flight_per_stream[best]) best = s;
            if (sv->free_norms.empty()) {
                // every slot is held by a resident result: wait for releases
                sv->queue.push_front(r);
                break;
            }
            r->norm = sv->norms + sv->free_norms.back();
            sv->free_norms.pop_back();
            r->stream = best;
            r->admitted = Clock::now();
            sv->resident_bytes += r->bytes;
            sv->peak_bytes = std::max(sv->peak_bytes, sv->resident_bytes);
            sv->in_flight_per_stream[best]++;
            lk.unlock();
            const bool ok = launch(sv, r);
            lk.lock();
            if (ok) {
                sv->running.push_back(r);
            } else {
                sv->in_flight_per_stream[best]--;
                finish(sv, r, r->status);
                sv->resident_bytes -= r->bytes;
                if (r->state) jq_state_destroy(r->state);
                r->state = nullptr;
                if (r->norm) sv->free_norms.push_back((int)(r->norm - sv->norms));
                if (r->done) (void)hipEventDestroy(r->done);
                delete r;
            }
            admitted_any = true;
            break;  // re-scan from the head after every admission
        }
        if (sv->stop && sv->queue.empty() && sv->running.empty()) break;
        if (admitted_any) continue;
        if (!sv->running.empty()) {
            sv->cv_sched.wait_for(lk, std::chrono::microseconds(50));
        } else {
            sv->cv_sched.wait_for(lk, std::chrono::milliseconds(5));
        }
    }
}

}  // namespace
}  // namespace jq

using namespace jq;

extern "C" {

int jq_server_create(uint64_t hbm_budget, int n_streams, int queue_cap, jq_encoding enc, jq_server** out) {
    try {
        set_last_error("");
        if (!out) fail(JQ_EINVAL, "jq_server_create: null output");
        *out = nullptr;
        if (n_streams < 1 || n_streams > 32) fail(JQ_EINVAL, "jq_server_create: 1..32 streams");
        if (queue_cap < 1) fail(JQ_EINVAL, "jq_server_create: queue_cap must be positive");
        if (enc != JQ_C128 && enc != JQ_C64 && enc != JQ_COMPACT) fail(JQ_EINVAL, "jq_server_create: bad encoding");
        if (hbm_budget == 0) fail(JQ_EINVAL, "jq_server_create: zero budget");
        auto sv = new jq_server();
        sv->budget = hbm_budget;
        sv->enc = enc;
        sv->queue_cap = queue_cap;
        JQ_HIP(hipGetDevice(&sv->device));
        for (int i = 0; i < n_streams; ++i) {
            hipStream_t st;
            JQ_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            sv->streams.push_back(st);
        }
        sv->in_flight_per_stream.assign(n_streams, 0);
        const int slots = 65536;
        JQ_HIP(hipHostMalloc((void**)&sv->norms, slots * sizeof(double), hipHostMallocDefault));
        for (int i = slots - 1; i >= 0; --i) sv->free_norms.push_back(i);
        sv->sched = std::thread(scheduler, sv);
        *out = sv;
        return JQ_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    }
}

int jq_server_submit(jq_server* sv, const jq_circuit* c, int blocking, uint64_t* ticket) {
    try {
        set_last_error("");
        if (!sv || !c || !ticket) fail(JQ_EINVAL, "jq_server_submit: null argument");
        const int n = c->n_qubits;
        if (n < 1 || n > 40) fail(JQ_EINVAL, "jq_server_submit: N out of range");
        if (c->n_gates && !c->gates) fail(JQ_EINVAL, "jq_server_submit: null gates");
        auto r = new Request();
        r->n = n;
        r->bytes = (uint64_t)bytes_per_amp(sv->enc) << n;
        try {
            for (uint64_t g = 0; g < c->n_gates; ++g) {
                if (c->gates[g].nq == 0) continue;
                r->ops.push_back(canonicalize(c->gates[g], n));
            }
        } catch (...) {
            delete r;
            throw;
        }
        std::unique_lock<std::mutex> lk(sv->mu);
        if (r->bytes > sv->budget) {
            delete r;
            sv->rejected++;
            fail(JQ_ENOMEM, "jq_server_submit: state of " + std::to_string(n) + " qubits exceeds the HBM budget");
        }
        while ((int)sv->queue.size() >= sv->queue_cap) {
            if (!blocking || sv->stop) {
                delete r;
                fail(JQ_EBUSY, "jq_server_submit: queue full");
            }
            sv->cv_space.wait(lk);
        }
        r->ticket = sv->next_ticket++;
        r->submitted = Clock::now();
        if (!sv->any_submit) {
            sv->first_submit = r->submitted;
            sv->any_submit = true;
        }
        sv->submitted++;
        sv->queue.push_back(r);
        *ticket = r->ticket;
        sv->cv_sched.notify_all();
        return JQ_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    }
}

int jq_server_wait(jq_server* sv, int timeout_ms, jq_result* out) {
    try {
        set_last_error("");
        if (!sv || !out) fail(JQ_EINVAL, "jq_server_wait: null argument");
        std::unique_lock<std::mutex> lk(sv->mu);
        auto ready = [&] { return !sv->done.empty(); };
        if (timeout_ms < 0) sv->cv_done.wait(lk, ready);
        else if (timeout_ms > 0) sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
        if (sv->done.empty()) {
            set_last_error("jq_server_wait: nothing finished");
            return JQ_EBUSY;
        }
        *out = sv->done.front();
        sv->done.pop_front();
        return JQ_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    }
}

int jq_server_release(jq_server* sv, uint64_t ticket) {
    try {
        set_last_error("");
        if (!sv) fail(JQ_EINVAL, "null server");
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->resident.find(ticket);
        if (it == sv->resident.end()) fail(JQ_EINVAL, "jq_server_release: unknown ticket");
        release_request(sv, it->second);
        sv->resident.erase(it);
        sv->cv_sched.notify_all();
        return JQ_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    }
}

int jq_server_stats_get(jq_server* sv, jq_server_stats* out) {
    try {
        set_last_error("");
        if (!sv || !out) fail(JQ_EINVAL, "null argument");
        std::lock_guard<std::mutex> lk(sv->mu);
        std::memset(out, 0, sizeof(*out));
        out->submitted = sv->submitted;
        out->completed = sv->completed;
        out->rejected = sv->rejected;
        out->peak_resident_bytes = sv->peak_bytes;
        if (!sv->latencies.empty()) {
            std::vector<double> l = sv->latencies;
            std::sort(l.begin(), l.end());
            auto pct = [&](double p) {
                const double pos = p * (l.size() - 1);
                const size_t i = (size_t)pos;
                const double f = pos - i;
                return i + 1 < l.size() ? l[i] * (1 - f) + l[i + 1] * f : l[i];
            };
            out->p50_ms = pct(0.50);
            out->p99_ms = pct(0.99);
            double s = 0;
            for (double v : l) s += v;
            out->mean_ms = s / l.size();
            const double span = ms_since(sv->first_submit, sv->last_done) / 1000.0;
            out->throughput_per_s = span > 0 ? sv->completed / span : 0.0;
        }
        return JQ_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    }
}

int jq_server_destroy(jq_server* sv) {
    if (!sv) return JQ_EINVAL;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        // drop requests that were never admitted
        for (Request* r : sv->queue) delete r;
        sv->queue.clear();
        sv->cv_sched.notify_all();
        sv->cv_space.notify_all();
    }
    if (sv->sched.joinable()) sv->sched.join();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        for (auto& kv : sv->resident) release_request(sv, kv.second);
        sv->resident.clear();
    }
    for (auto st : sv->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    if (sv->norms) (void)hipHostFree(sv->norms);
    delete sv;
    return JQ_OK;
}

}  // extern "C"

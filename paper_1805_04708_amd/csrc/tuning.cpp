// Tuning of the single-state path (jq_tuning_get / jq_tuning_set /
// jq_autotune): the fused pass's register width, the planner's weight of a
// pass against its ops, and the per-gate kernels' width per target (one or
// four amplitude pairs per thread), per (device, encoding, N).  Values come from this process (set or
// measured), else from a JSON cache file, else built-in defaults.
#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "internal.hpp"

namespace jq {

namespace {

template <class F>
int guarded_call(F&& f) {
    try {
        set_last_error("");
        f();
        return JQ_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        set_last_error("host allocation failed");
        return JQ_ENOMEM;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return JQ_EDEVICE;
    }
}

struct Entry {
    std::string device;
    int enc = 0;
    int n = 0;
    jq_tuning t{};
};

std::mutex g_mu;
std::vector<Entry> g_process;  // set or measured in this process
std::vector<Entry> g_cache;    // read from the cache file
bool g_cache_read = false;
std::string g_cache_from;      // the path it was read from

constexpr int kMaxDev = 64;
std::string g_dev_key[kMaxDev];

// the smallest state that streams from HBM rather than the 256 MB
// last-level cache (N = 25 for complex128)
constexpr int kStreamingN = 25;

const char* enc_name(int enc) { return enc == JQ_C128 ? "c128" : enc == JQ_C64 ? "c64" : "compact"; }

int enc_from_name(const std::string& s) {
    if (s == "c128") return JQ_C128;
    if (s == "c64") return JQ_C64;
    return -1;
}

std::string cache_path() {
    if (const char* p = std::getenv("JQ_TUNE_CACHE")) return p;
    if (const char* h = std::getenv("HOME")) return std::string(h) + "/.cache/jq/tuning.json";
    return "";
}

// "<arch>:<product name>" of the current device, or "host" when none is visible
std::string device_key() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) {
        (void)hipGetLastError();
        return "host";
    }
    if (g_dev_key[dev].empty()) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) != hipSuccess) {
            (void)hipGetLastError();
            return "host";
        }
        std::string key = std::string(p.gcnArchName) + ":" + p.name;
        for (char& c : key)
            if (c == '"' || c == '\\' || (unsigned char)c < 0x20) c = '_';
        g_dev_key[dev] = key;
    }
    return g_dev_key[dev];
}

// --------------------------------------------------------- cache file --
//
// {"version": 1, "entries": [{"device": "...", "encoding": "c128", "n": 28,
//   "k_reg": 4, "pass_ops": 19.0, "wide_target": 17, "wide_mask": 1966080,
//   "tuned_ms": .., "default_ms": ..}, ...]}
// wide_mask is optional (entries without it take the targets from
// wide_target up) and holds targets below 53 only, so that the number is
// exact as a double.
//
// The reader accepts exactly this shape (objects of string and number
// fields inside "entries"); anything else makes the whole file count as
// empty.

struct Reader {
    const std::string& s;
    size_t i = 0;
    explicit Reader(const std::string& src) : s(src) {}
    void ws() {
        while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
    }
    bool eat(char c) {
        ws();
        if (i < s.size() && s[i] == c) {
            ++i;
            return true;
        }
        return false;
    }
    bool str(std::string& out) {
        ws();
        if (i >= s.size() || s[i] != '"') return false;
        ++i;
        out.clear();
        while (i < s.size() && s[i] != '"') {
            if (s[i] == '\\') return false;  // the writer never escapes
            out += s[i++];
        }
        if (i >= s.size()) return false;
        ++i;
        return true;
    }
    bool num(double& out) {
        ws();
        const char* b = s.c_str() + i;
        char* e = nullptr;
        out = std::strtod(b, &e);
        if (e == b) return false;
        i += (size_t)(e - b);
        return std::isfinite(out);
    }
};

bool valid(int enc, const jq_tuning& t);

constexpr uint64_t kMaskJson = (1ull << 53) - 1;

// Make wide_mask and wide_target agree: a zero mask stands for the targets
// from wide_target up; wide_target becomes the mask's lowest target (64:
// none).
void normalize_wide(jq_tuning& t) {
    if (t.wide_mask == 0) t.wide_mask = t.wide_target >= 64 ? 0 : ~0ull << t.wide_target;
    t.wide_target = t.wide_mask ? __builtin_ctzll(t.wide_mask) : 64;
}

bool parse_entry(Reader& r, Entry& e) {
    if (!r.eat('{')) return false;
    bool have_dev = false, have_enc = false, have_n = false, have_k = false, have_p = false, have_w = false;
    if (r.eat('}')) return false;
    do {
        std::string key;
        if (!r.str(key) || !r.eat(':')) return false;
        if (key == "device" || key == "encoding") {
            std::string v;
            if (!r.str(v)) return false;
            if (key == "device") {
                e.device = v;
                have_dev = true;
            } else {
                e.enc = enc_from_name(v);
                have_enc = e.enc >= 0;
            }
        } else {
            double v;
            if (!r.num(v)) return false;
            if (key == "n") e.n = (int)v, have_n = v == std::floor(v);
            else if (key == "k_reg") e.t.k_reg = (int)v, have_k = v == std::floor(v);
            else if (key == "pass_ops") e.t.pass_ops = v, have_p = true;
            else if (key == "wide_target") e.t.wide_target = (int)v, have_w = v == std::floor(v);
            else if (key == "wide_mask") e.t.wide_mask = (uint64_t)v;
            else if (key == "search") e.t.search = (int)v;
            else if (key == "tuned_ms") e.t.tuned_ms = v;
            else if (key == "default_ms") e.t.default_ms = v;
        }
    } while (r.eat(','));
    if (!r.eat('}')) return false;
    if (!(have_dev && have_enc && have_n && have_k && have_p && have_w)) return false;
    e.t.n_qubits = e.n;
    e.t.source = JQ_TUNE_CACHED;
    if (!(e.n >= 1 && e.n <= JQ_MAX_QUBITS && valid(e.enc, e.t))) return false;
    normalize_wide(e.t);  // an entry without wide_mask: from wide_target
    return true;
}

std::vector<Entry> read_cache_file(const std::string& path) {
    std::vector<Entry> out;
    if (path.empty()) return out;
    std::ifstream f(path);
    if (!f) return out;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string text = ss.str();
    Reader r(text);
    std::string key;
    double version = 0;
    if (!r.eat('{')) return {};
    bool have_entries = false;
    do {
        if (!r.str(key) || !r.eat(':')) return {};
        if (key == "version") {
            if (!r.num(version)) return {};
        } else if (key == "entries") {
            if (!r.eat('[')) return {};
            if (!r.eat(']')) {
                do {
                    Entry e;
                    if (!parse_entry(r, e)) return {};
                    out.push_back(e);
                } while (r.eat(','));
                if (!r.eat(']')) return {};
            }
            have_entries = true;
        } else {
            return {};
        }
    } while (r.eat(','));
    if (!r.eat('}') || version != 1.0 || !have_entries) return {};
    r.ws();
    if (r.i != text.size()) return {};
    return out;
}

void write_cache_file(const std::string& path, const std::vector<Entry>& entries) {
    if (path.empty()) return;
    // create the parent folders ($HOME/.cache/jq, say)
    for (size_t p = path.find('/', 1); p != std::string::npos; p = path.find('/', p + 1))
        (void)::mkdir(path.substr(0, p).c_str(), 0755);
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return;
        f << "{\"version\": 1, \"entries\": [";
        for (size_t i = 0; i < entries.size(); ++i) {
            const Entry& e = entries[i];
            char buf[512];
            std::snprintf(buf, sizeof buf,
                          "%s\n  {\"device\": \"%s\", \"encoding\": \"%s\", \"n\": %d, \"k_reg\": %d, "
                          "\"pass_ops\": %.17g, \"wide_target\": %d, \"wide_mask\": %llu, \"search\": %d, "
                          "\"tuned_ms\": %.17g, \"default_ms\": %.17g}",
                          i ? "," : "", e.device.c_str(), enc_name(e.enc), e.n, e.t.k_reg, e.t.pass_ops,
                          e.t.wide_target, (unsigned long long)(e.t.wide_mask & kMaskJson), e.t.search,
                          e.t.tuned_ms, e.t.default_ms);
            f << buf;
        }
        f << "\n]}\n";
        if (!f) return;
    }
    (void)std::rename(tmp.c_str(), path.c_str());
}

// read the cache file once per path (JQ_TUNE_CACHE may name another file
// later in the process)
void ensure_cache_read() {
    const std::string path = cache_path();
    if (g_cache_read && path == g_cache_from) return;
    g_cache = read_cache_file(path);
    g_cache_from = path;
    g_cache_read = true;
}

int k_max(int enc) { return enc == JQ_C64 ? 6 : 5; }

bool valid(int enc, const jq_tuning& t) {
    if (enc != JQ_C128 && enc != JQ_C64) return false;
    if (t.k_reg < 2 || t.k_reg > k_max(enc)) return false;
    if (!(t.pass_ops > 0.0 && t.pass_ops <= 10000.0)) return false;
    if (t.wide_target < 0 || t.wide_target > 64) return false;
    if (t.search != JQ_SEARCH_AUTO && t.search != JQ_SEARCH_ON && t.search != JQ_SEARCH_OFF) return false;
    return true;
}

const Entry* find(const std::vector<Entry>& v, const std::string& dev, int enc, int n) {
    for (const Entry& e : v)
        if (e.device == dev && e.enc == enc && e.n == n) return &e;
    return nullptr;
}

// the entry of the largest tuned size in [kStreamingN, n]
const Entry* find_streaming(const std::vector<Entry>& v, const std::string& dev, int enc, int n) {
    const Entry* best = nullptr;
    for (const Entry& e : v)
        if (e.device == dev && e.enc == enc && e.n >= kStreamingN && e.n <= n && (!best || e.n > best->n))
            best = &e;
    return best;
}

void upsert(std::vector<Entry>& v, const Entry& e) {
    for (Entry& x : v)
        if (x.device == e.device && x.enc == e.enc && x.n == e.n) {
            x = e;
            return;
        }
    v.push_back(e);
}

}  // namespace

jq_tuning default_tuning(int enc) {
    jq_tuning t{};
    // measured on an MI355X at N = 30 (see the planner's cost model):
    // complex128 K = 5, complex64 K = 6 (40 layers of Haar U(2) and CZ:
    // 388 against 411 ms at K = 4, 222 against 226 ms at K = 5, the fused
    // kernel compiled for the reduced op kinds; circuits with other gates
    // plan at 4 and 5, PlanConfig::k_general_max); a pass streams in the
    // time of 19 (complex128) or 6 (complex64) ops; the per-gate kernels
    // take one pair per thread on every complex128 target (as fast or within
    // 2.5% everywhere, up to 12% faster from target 17 up), and four from
    // target 17 up for complex64, where the better width changes target by
    // target (the tuner chooses per target)
    t.k_reg = enc == JQ_C64 ? 6 : 5;
    t.pass_ops = enc == JQ_C64 ? 6.0 : 19.0;
    t.wide_mask = enc == JQ_C64 ? ~0ull << 17 : 0;
    t.wide_target = enc == JQ_C64 ? 17 : 64;
    t.search = JQ_SEARCH_AUTO;  // on from 1 GiB of state up (the planner's size rule)
    t.n_qubits = 0;
    t.source = JQ_TUNE_DEFAULT;
    return t;
}

jq_tuning tuned_for(int n, int enc) {
    if (enc != JQ_C128 && enc != JQ_C64) return default_tuning(enc);
    std::lock_guard<std::mutex> lk(g_mu);
    const std::string dev = device_key();
    if (const Entry* e = find(g_process, dev, enc, n)) return e->t;
    ensure_cache_read();
    if (const Entry* e = find(g_cache, dev, enc, n)) return e->t;
    if (n >= kStreamingN) {
        const Entry* a = find_streaming(g_process, dev, enc, n);
        const Entry* b = find_streaming(g_cache, dev, enc, n);
        if (a && (!b || a->n >= b->n)) return a->t;
        if (b) return b->t;
    }
    return default_tuning(enc);
}

namespace {

// Deterministic tuning circuit: `layers` layers of random U(2) on every
// qubit (from Euler angles) and CZ on a random perfect matching.
std::vector<GateOp> tuning_circuit(int n, int layers) {
    uint64_t x = 0x9E3779B97F4A7C15ull;
    auto next = [&x] {
        x ^= x << 13;
        x ^= x >> 7;
        x ^= x << 17;
        return x;
    };
    auto unif = [&] { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); };
    std::vector<GateOp> ops;
    for (int l = 0; l < layers; ++l) {
        for (int q = 0; q < n; ++q) {
            const double a = 2 * M_PI * unif(), b = 2 * M_PI * unif(), c = M_PI * unif();
            // U = [[cos c e^{ia}, -sin c e^{ib}], [sin c e^{-ib}, cos c e^{-ia}]]
            jq_gate g;
            std::memset(&g, 0, sizeof g);
            g.kind = JQ_DENSE;
            g.nq = 1;
            g.qubits[0] = q;
            const double cc = std::cos(c), ss = std::sin(c);
            const double m[8] = {cc * std::cos(a), cc * std::sin(a), -ss * std::cos(b), -ss * std::sin(b),
                                 ss * std::cos(b), -ss * std::sin(b), cc * std::cos(a), -cc * std::sin(a)};
            for (int i = 0; i < 8; ++i) g.m[i] = m[i];
            ops.push_back(canonicalize(g, n));
        }
        std::vector<int> perm(n);
        for (int i = 0; i < n; ++i) perm[i] = i;
        for (int i = n - 1; i > 0; --i) std::swap(perm[i], perm[next() % (uint64_t)(i + 1)]);
        for (int i = 0; i + 1 < n; i += 2) {
            jq_gate g;
            std::memset(&g, 0, sizeof g);
            g.kind = JQ_DIAGONAL;
            g.nq = 2;
            g.qubits[0] = perm[i];
            g.qubits[1] = perm[i + 1];
            g.m[0] = g.m[2] = g.m[4] = 1.0;
            g.m[6] = -1.0;
            ops.push_back(canonicalize(g, n));
        }
    }
    return ops;
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    Timer() {
        JQ_HIP(hipEventCreate(&a));
        JQ_HIP(hipEventCreate(&b));
    }
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    template <class F>
    double ms(hipStream_t st, F&& f) {
        JQ_HIP(hipEventRecord(a, st));
        f();
        JQ_HIP(hipEventRecord(b, st));
        JQ_HIP(hipEventSynchronize(b));
        float v = 0.f;
        JQ_HIP(hipEventElapsedTime(&v, a, b));
        return v;
    }
};

struct ScratchState {
    jq_state* s = nullptr;
    ~ScratchState() {
        if (s) (void)jq_state_destroy(s);
    }
};

// A tuned value replaces a default only when it is faster by this factor:
// smaller differences are within the run-to-run spread of the timings, and
// a short tuning circuit exaggerates them.
constexpr double kMargin = 0.98;

// workload: the caller's circuit (canonical ops), or empty for the
// built-in tuning circuit
jq_tuning measure(int n, int enc, const std::vector<GateOp>& workload) {
    ScratchState scratch;
    scratch.s = state_create(n, enc, nullptr, false);
    jq_state* s = scratch.s;
    const std::vector<GateOp> circ = workload.empty() ? tuning_circuit(n, 10) : workload;
    // per-gate timing gates: a dense U(2) on each target
    const std::vector<GateOp> probe = tuning_circuit(n, 1);
    const jq_tuning def = default_tuning(enc);
    Timer tm;

    // register width and planner weight: the whole tuning circuit under
    // every candidate, in two alternating rounds, best of the two
    struct Cand {
        int k;
        double pass_ops;
        double ms;
    };
    std::vector<Cand> cands;
    for (int k = 3; k <= k_max(enc); ++k) {
        if (n < 6 + k) continue;
        for (double f : {0.5, 1.0, 2.0}) cands.push_back({k, def.pass_ops * f, 1e30});
    }
    for (const Cand& c : cands) state_apply_config(s, circ, plan_config_tuned(n, enc, c.k, c.pass_ops));  // warm
    for (int r = 0; r < 2; ++r)
        for (Cand& c : cands) {
            const PlanConfig cfg = plan_config_tuned(n, enc, c.k, c.pass_ops);
            c.ms = std::min(c.ms, tm.ms(s->stream, [&] { state_apply_config(s, circ, cfg); }));
        }
    jq_tuning best = def;
    double def_ms = -1.0, best_ms = 1e30;
    for (const Cand& c : cands) {
        if (c.k == def.k_reg && c.pass_ops == def.pass_ops) def_ms = c.ms;
        if (c.ms < best_ms) {
            best_ms = c.ms;
            best.k_reg = c.k;
            best.pass_ops = c.pass_ops;
        }
    }
    if (def_ms > 0 && !(best_ms < kMargin * def_ms)) {
        best.k_reg = def.k_reg;
        best.pass_ops = def.pass_ops;
        best_ms = def_ms;
    }
    if (def_ms < 0) def_ms = best_ms;

    // the large-state planner steps switched the other way than the size
    // rule has them, for the chosen width and weight
    {
        PlanConfig cfg = plan_config_tuned(n, enc, best.k_reg, best.pass_ops);
        const bool rule_on = cfg.search_rounds > 0;
        cfg.search_rounds = rule_on ? 0 : 2;
        state_apply_config(s, circ, cfg);  // warm
        double t = 1e30;
        for (int r = 0; r < 2; ++r) t = std::min(t, tm.ms(s->stream, [&] { state_apply_config(s, circ, cfg); }));
        if (t < kMargin * best_ms) {
            best.search = rule_on ? JQ_SEARCH_OFF : JQ_SEARCH_ON;
            best_ms = t;
        }
    }

    // per-gate widths: one dense gate on every target from 8 up with one
    // pair per thread (mask 0) and with four (every bit set)
    const int lo = std::min(8, n - 1);
    std::vector<double> t1(n, 0.0), t4(n, 0.0);
    for (int t = lo; t < n; ++t) {
        GateOp op = probe[t];  // the U(2) on qubit t
        for (const uint64_t wide : {uint64_t(0), ~uint64_t(0)}) {
            sv_apply_op(enc, s->buf, n, op, wide, s->stream);  // warm
            double v = 1e30;
            for (int r = 0; r < 3; ++r)
                v = std::min(v, tm.ms(s->stream, [&] { sv_apply_op(enc, s->buf, n, op, wide, s->stream); }));
            (wide ? t4 : t1)[t] = v;
        }
    }
    // below lo the default; from lo up four pairs where they are 2% faster;
    // from n up (a larger state using this entry) as on target n - 1
    uint64_t mask = def.wide_mask & ((1ull << lo) - 1);
    for (int t = lo; t < n; ++t)
        if (t4[t] < kMargin * t1[t]) mask |= 1ull << t;
    if ((mask >> (n - 1)) & 1) mask |= ~0ull << n;
    best.wide_mask = mask;
    best.wide_target = 0;
    normalize_wide(best);
    best.n_qubits = n;
    best.source = JQ_TUNE_MEASURED;
    best.tuned_ms = best_ms;
    best.default_ms = def_ms;
    return best;
}

}  // namespace

}  // namespace jq

using namespace jq;

extern "C" {

int jq_tuning_get(int n_qubits, int enc, jq_tuning* out) {
    return guarded_call([&] {
        if (!out) fail(JQ_EINVAL, "jq_tuning_get: null output");
        if (n_qubits < 1 || n_qubits > JQ_MAX_QUBITS) fail(JQ_EINVAL, "jq_tuning_get: N must be in [1, 63]");
        if (enc != JQ_C128 && enc != JQ_C64 && enc != JQ_COMPACT) fail(JQ_EINVAL, "jq_tuning_get: bad encoding");
        *out = tuned_for(n_qubits, enc);
    });
}

int jq_tuning_set(int n_qubits, int enc, const jq_tuning* t) {
    return guarded_call([&] {
        if (n_qubits < 1 || n_qubits > JQ_MAX_QUBITS) fail(JQ_EINVAL, "jq_tuning_set: N must be in [1, 63]");
        if (enc != JQ_C128 && enc != JQ_C64) fail(JQ_EINVAL, "jq_tuning_set: only JQ_C128 and JQ_C64 are tuned");
        if (t && !valid(enc, *t)) fail(JQ_EINVAL, "jq_tuning_set: a field is out of range");
        std::lock_guard<std::mutex> lk(g_mu);
        const std::string dev = device_key();
        if (!t) {
            g_process.erase(std::remove_if(g_process.begin(), g_process.end(),
                                           [&](const Entry& e) { return e.device == dev && e.enc == enc && e.n == n_qubits; }),
                            g_process.end());
            return;
        }
        Entry e;
        e.device = dev;
        e.enc = enc;
        e.n = n_qubits;
        e.t = *t;
        e.t.n_qubits = n_qubits;
        e.t.source = JQ_TUNE_SET;
        normalize_wide(e.t);
        upsert(g_process, e);
    });
}

int jq_autotune(int n_qubits, int enc, int flags, const jq_gate* gates, size_t count, jq_tuning* out) {
    return guarded_call([&] {
        if (n_qubits < 10 || n_qubits > 34) fail(JQ_EINVAL, "jq_autotune: N must be in [10, 34]");
        if (enc != JQ_C128 && enc != JQ_C64) fail(JQ_EINVAL, "jq_autotune: only JQ_C128 and JQ_C64 are tuned");
        if (flags & ~(JQ_TUNE_FORCE | JQ_TUNE_NO_CACHE)) fail(JQ_EINVAL, "jq_autotune: unknown flags");
        if (count && !gates) fail(JQ_EINVAL, "jq_autotune: null gates");
        std::vector<GateOp> workload;
        for (size_t i = 0; i < count; ++i) {
            if (gates[i].nq == 0) continue;  // identity
            try {
                workload.push_back(canonicalize(gates[i], n_qubits));
            } catch (const Error& e) {
                fail(e.code, "jq_autotune: gate " + std::to_string(i) + ": " + e.what());
            }
        }
        std::string dev;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            dev = device_key();
            if (dev == "host") fail(JQ_EDEVICE, "jq_autotune: no GPU visible");
            if (!(flags & JQ_TUNE_NO_CACHE) && !(flags & JQ_TUNE_FORCE)) {
                ensure_cache_read();
                if (const Entry* e = find(g_cache, dev, enc, n_qubits)) {
                    upsert(g_process, *e);
                    if (out) *out = e->t;
                    return;
                }
            }
        }
        const jq_tuning t = measure(n_qubits, enc, workload);
        std::lock_guard<std::mutex> lk(g_mu);
        Entry e;
        e.device = dev;
        e.enc = enc;
        e.n = n_qubits;
        e.t = t;
        upsert(g_process, e);
        if (!(flags & JQ_TUNE_NO_CACHE)) {
            // merge with the file as it is now (another process may have
            // written entries since it was first read)
            std::vector<Entry> merged = read_cache_file(cache_path());
            Entry c = e;
            c.t.source = JQ_TUNE_CACHED;
            upsert(merged, c);
            write_cache_file(cache_path(), merged);
            g_cache = merged;
            g_cache_from = cache_path();
            g_cache_read = true;
        }
        if (out) *out = t;
    });
}

}  // extern "C"

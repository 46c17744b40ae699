"""Throughput of state-vector gate application on one MI355X.

One step = the whole hot path on one synthetic circuit: reset the state to
|0...0>, lower the named gates (host), plan fused passes (host), run every
kernel, and take the FP64 norm and a one-qubit marginal.  The workload is a
30-qubit complex128 state (16 GiB) under 40 layers of Haar-random U(2) on
every qubit plus CZ on a random perfect matching: 1800 gates.

Prints one JSON line.  `value` is gates/s of the whole step (inputs resident
in HBM); `roofline` is for the dominant kernel (the fused tile pass),
timed with HIP events on the stream it runs on; `cpu_baseline` is the CPU
oracle on a bounded sample of the same circuit on this host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "gates/s + HBM GB/s (% peak) at N=30; p50/p99 latency on a served circuit mix"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6   # vector FP64: 256 CUs x 128 flop/clk x 2.4 GHz
PEAK_FP32_TFLOPS = 157.3  # vector FP32 (dual issue)
# diagonal gates whose entries are +-1 (sign flips: no arithmetic)
SIGN_ONLY = {"Z", "CZ"}
DENSE_1Q = {"H", "Y", "MAT1", "U2", "U3", "+X", "-X", "+Y", "-Y", "U2H"}


def circuit_flops(circuit, n):
    """Algorithmic real flops of a circuit on 2^n amplitudes: a dense 2x2 on
    the pairs of the controlled subspace costs 14 per amplitude (4 complex
    products, 2 complex sums per pair), a diagonal phase 6 per amplitude it
    multiplies, sign flips and permutations nothing."""
    total = 0.0
    for g in circuit:
        name, qubits = g[0], g[1]
        ctrl = len(g[3]) if len(g) > 3 else 0
        if name in SIGN_ONLY or name in ("X", "CNOT", "TOFFOLI", "SWAP", "I"):
            continue
        if name in DENSE_1Q:
            total += 14.0 * 2.0 ** (n - ctrl)
        elif name in ("CP", "U"):
            total += 6.0 * 2.0 ** (n - 2 - ctrl)
        else:  # one-qubit phase gates (S, T, R, U1, RZ, ...)
            total += 6.0 * 2.0 ** (n - 1 - ctrl)
    return total


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=30)
    p.add_argument("--layers", type=int, default=40)
    p.add_argument("--enc", default="c128", choices=["c128", "c64"])
    p.add_argument("--fusion", type=int, default=0)
    p.add_argument("--seed", type=int, default=2018)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-extras", action="store_true")
    p.add_argument("--extras", default="all", metavar="LIST",
                   help="comma-separated extras to run (per_target, c64, batch, serve, compact, compact_dense, "
                        "shor, aux, large), or all")
    p.add_argument("--cpu-gates", type=int, default=3, help="gates of the circuit the CPU oracle times")
    p.add_argument("--metrics-log", metavar="PATH",
                   help="append this run's records to a JSONL file: one line for the headline workload "
                        "(config, seed, gates, fused passes, time, gates/s, GB/s, fraction of peak, counter "
                        "bytes) and one per extra (errors, latencies, CPU timings with core counts)")
    p.add_argument("--no-autotune", action="store_true",
                   help="keep the built-in tuning instead of measuring it on this device first")
    p.add_argument("--copy-calibration", type=int, default=4096, metavar="MIB",
                   help="size of the plain torch device copy reported as the copy ceiling (and used to "
                        "calibrate the traffic counters); 0 skips it")
    return p.parse_args()


KERNEL_SOURCES = ["kernels_sv.hip", "fused_ops.hpp", "device_common.hpp", "internal.hpp", "planner.cpp"]


def kernel_source_hash():
    import hashlib
    csrc = os.path.join(ROOT, "paper_1805_04708_amd", "csrc")
    data = b"".join(open(os.path.join(csrc, f), "rb").read() for f in KERNEL_SOURCES)
    return hashlib.sha256(data).hexdigest()[:16]


def traffic_from_profiles(kernel, workload):
    """HBM bytes per launch from the recorded rocprofv3 FETCH_SIZE/WRITE_SIZE
    runs (scaled by the copy-kernel calibration), or None if there is no
    record or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(f"{kernel}:{workload}")
    except Exception:
        return None
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


# batched circuits the CPU leg runs (the first of the 4096; lowering them in
# Python dominates its time)
CPU_BATCH_SAMPLE = 512


VALU_PEAK_PER_S = 256 * 4 * 2.4e9 / 4  # wave64 VALU instructions: 256 CUs x 4 SIMDs, 4 cycles each
VALU_SOURCES = ["kernels_compact.hip", "fused_ops.hpp", "device_common.hpp", "internal.hpp", "planner.cpp"]


def valu_roofline(kernel, workload, avg_ms):
    """VALU-issue roofline of a VALU-bound kernel: its VALU instructions per
    launch from the recorded rocprofv3 SQ_INSTS_VALU run (profiles/valu.json)
    over the live launch time, against the issue peak; None if there is no
    record or the sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "valu.json")
    try:
        rec = json.load(open(path)).get(f"{kernel}:{workload}")
    except Exception:
        return None
    csrc = os.path.join(ROOT, "paper_1805_04708_amd", "csrc")
    h = hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read() for f in VALU_SOURCES)).hexdigest()[:16]
    if not rec or rec.get("source_hash") != h:
        return None
    achieved = rec["valu_insts_per_launch"] / (avg_ms * 1e-3)
    return {"bound": "alu", "unit": "VALU instr/s", "achieved": achieved, "peak": VALU_PEAK_PER_S,
            "frac": achieved / VALU_PEAK_PER_S, "valu_insts_per_launch": rec["valu_insts_per_launch"]}


def cpu_baseline(n, circuit, gates, batch_states=None, batch_count=CPU_BATCH_SAMPLE, batch_seed=4096):
    """The CPU side, on this host's cores.

    value: the oracle (plain single-threaded FP64 C) on the first `gates`
    gates of the circuit at N (a bounded sample; the whole circuit would take
    hours).  paper_openmp: the paper's own CPU method (Sec. 3.1: the pair
    loops split at the target bit, OpenMP over the outer or the inner loop by
    the paper's trip-count test; bit-identical to the oracle) on the same
    sample with every core.  configs: the 16-qubit 200-gate circuit at one
    thread and at every core, and the first batch_count of the 4096 batched
    circuits in parallel across cores, whose FP64 states are also the
    reference for the error of the GPU's batched states (batch_states:
    encoding -> list of states in circuit order)."""
    import numpy as np
    from oracle import core as O
    from oracle import paper_cpu as PC
    from paper_1805_04708_amd import workloads as W

    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((line.split(":", 1)[1].strip() for line in f if line.startswith("model name")), None)
    except OSError:
        pass
    threads = PC.max_threads()

    sample = circuit[:gates]
    psi = O.zero_state(n)
    t0 = time.perf_counter()
    O.run(psi, n, sample)
    dt = time.perf_counter() - t0
    del psi
    psi = O.zero_state(n)
    t0 = time.perf_counter()
    PC.run(psi, n, sample, threads=threads)
    dt_omp = time.perf_counter() - t0
    del psi

    c0 = W.random_circuit(16, 200, seed=16)
    t0 = time.perf_counter()
    O.run(O.zero_state(16), 16, c0)
    c0_oracle = time.perf_counter() - t0
    c0_omp = {}
    for th in sorted({1, threads}):
        t0 = time.perf_counter()
        PC.run(O.zero_state(16), 16, c0, threads=th)
        c0_omp[th] = time.perf_counter() - t0

    inst = W.batch_instances(4096, base_seed=batch_seed)[:batch_count]
    ns = [m for m, _ in inst]
    states = [O.zero_state(m) for m in ns]
    recs = PC.pack_many([c for _, c in inst])
    t0 = time.perf_counter()
    PC.run_many(states, ns, recs, threads=threads)
    c3 = time.perf_counter() - t0
    c3_out = {"circuits": batch_count, "of": 4096, "seconds": c3, "circuits_per_s": batch_count / c3,
              "cores": threads}
    for enc, got in (batch_states or {}).items():
        errs = np.array([np.linalg.norm(g - r) / np.linalg.norm(r) for g, r in zip(got, states)])
        fids = np.array([abs(np.vdot(r, g)) ** 2 / (np.vdot(r, r).real * np.vdot(g, g).real)
                         for g, r in zip(got, states)])
        c3_out[f"gpu_batch_{enc}_vs_fp64"] = {"checked": len(errs), "max_rel_l2": float(errs.max()),
                                              "median_rel_l2": float(np.median(errs)),
                                              "min_fidelity": float(fids.min())}
    return {"value": len(sample) / dt, "unit": "gates/s", "cores": 1, "kind": "oracle",
            "sample": f"first {len(sample)} gates of the same circuit at N={n}, single-threaded FP64 C oracle, "
                      f"{dt:.1f} s",
            "paper_openmp": {"value": len(sample) / dt_omp, "unit": "gates/s", "cores": threads,
                             "sample": f"the same {len(sample)} gates, the paper's OpenMP loop split (Sec. 3.1), "
                                       f"{dt_omp:.2f} s"},
            "configs": {
                "n16_200_gates": {"oracle_1_core_s": c0_oracle,
                                  "paper_openmp_s": {str(k): v for k, v in c0_omp.items()},
                                  "gates_per_s_all_cores": 200 / c0_omp[threads]},
                "batch_sample": c3_out},
            "host": {"nproc": os.cpu_count(), "omp_threads": threads, "model": model}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1805_04708_amd import jq
    from paper_1805_04708_amd import workloads as W

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    n = args.n
    circuit = W.layered_u2_cz(n, args.layers, seed=args.seed)
    G = len(circuit)

    # the planner's register width and pass weight and the per-gate
    # threshold, measured on this device for this state size with the
    # workload's circuit as the tuning circuit (on a scratch state, outside
    # the timed steps)
    if args.no_autotune:
        tuning = jq.tuning_get(n, args.enc)
    else:
        t0 = time.perf_counter()
        tuning = jq.autotune(n, args.enc, circuit, force=True, no_cache=True)
        tuning["seconds"] = time.perf_counter() - t0

    state = jq.State(n, args.enc).set_stream(stream)
    bpa = 16 if args.enc == "c128" else 8

    def step():
        state.init(jq.JQ_INIT_ZERO)
        arr = jq.gates(circuit)                      # lowering (host)
        state.apply_circuit(arr, fusion=args.fusion)  # planning + kernels
        nrm = state.norm()                           # FP64 reduction (synchronises)
        p = state.probabilities([n - 1])
        return nrm, p

    for _ in range(args.warmup):
        nrm, _ = step()
    torch.cuda.synchronize()

    state.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        nrm, p = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = state.profile_read()
    state.profile(False)

    ms_per_step = 1000.0 * dt / args.steps
    value = G * args.steps / dt
    dom = "fused" if "fused" in stats else max(stats, key=lambda k: stats[k]["ms"])
    d = stats[dom]
    avg_ms = d["ms"] / d["launches"]
    bytes_per_launch = d["bytes"] / d["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    workload = f"{args.enc}_n{n}"
    traffic = traffic_from_profiles(dom, workload)
    kernel_ms = sum(v["ms"] for v in stats.values())
    alg_bytes = sum(v["bytes"] for v in stats.values())

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.enc == "c128" else "f32",
        "data": "synthetic",
        "config": {"workload": f"layered Haar-U(2) + CZ-matching circuit, N={n}, {args.enc}, "
                               f"{args.layers} layers ({G} gates), from |0...0>",
                   "n_qubits": n, "encoding": args.enc, "layers": args.layers, "gates": G,
                   "fusion": "auto" if args.fusion == 0 else args.fusion, "seed": args.seed,
                   "tuning": tuning},
        "norm": nrm,
        "hbm_gbps_step": alg_bytes / (dt / args.steps * args.steps) / 1e9 if dt > 0 else None,
        "kernel_ms_per_step": kernel_ms / args.steps,
        "kernels": {k: {"launches_per_step": v["launches"] / args.steps, "avg_ms": v["ms"] / v["launches"],
                        "gbps": v["bytes"] / v["launches"] / (v["ms"] / v["launches"] * 1e-3) / 1e9}
                    for k, v in stats.items()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic,
                     "alg_bytes_per_launch": bytes_per_launch, "avg_launch_ms": avg_ms},
    }
    if dom == "fused":
        # the same kernel against the FP64 vector peak: algorithmic flops of
        # the circuit spread over its fused launches
        flops = circuit_flops(circuit, n) / (d["launches"] / args.steps)
        out["roofline"]["alu"] = {"bound": "alu", "achieved": flops / (avg_ms * 1e-3) / 1e12,
                                  "peak": PEAK_FP64_TFLOPS if args.enc == "c128" else PEAK_FP32_TFLOPS,
                                  "unit": "TFLOP/s",
                                  "frac": flops / (avg_ms * 1e-3) / 1e12 /
                                          (PEAK_FP64_TFLOPS if args.enc == "c128" else PEAK_FP32_TFLOPS),
                                  "alg_flops_per_launch": flops}

    wanted = set() if args.no_extras else (
        {"per_target", "unfused", "c64", "batch", "serve", "compact", "compact_dense", "shor", "aux", "large",
         "paper_circuits"}
        if args.extras == "all" else set(args.extras.split(",")))
    if "per_target" in wanted:
        out["per_target"] = per_target(state, n, bpa)
        out["cz_by_min_qubit"] = cz_by_min_qubit(state, n)
    if "c64" in wanted and args.enc == "c128":
        # the timed steps leave the circuit's complex128 result in `state`
        state.init(jq.JQ_INIT_ZERO)
        state.apply_circuit(jq.gates(circuit), fusion=args.fusion)
        state.synchronize()
        out["c64_same_circuit"] = c64_same_circuit(n, circuit, args.fusion, state)
    if "unfused" in wanted:
        out["unfused"] = unfused_extra(state, circuit, args.layers)

    state.close()
    torch.cuda.synchronize()

    batch_states = {}
    extras = [("batch", "batch", lambda: batch_extra(keep=batch_states)), ("serve", "serve", serve_extra),
              ("compact", "compact", compact_extra), ("compact_dense", "compact_dense", compact_dense_extra),
              ("shor", "shor", shor_extra), ("aux", "aux", aux_extra), ("large", "large_states", large_extra),
              ("paper_circuits", "paper_circuits", paper_circuits_extra)]
    for name, key, fn in extras:
        if name in wanted:
            out[key] = fn()

    if args.copy_calibration:
        # a plain device copy: the practical streaming ceiling of this GPU,
        # and the reference for scaling the HBM traffic counters
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        best = None
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            dst.copy_(src)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        out["copy_calibration"] = {"bytes_read": nbytes, "bytes_written": nbytes,
                                   "gbps": 2 * nbytes / (best * 1e-3) / 1e9, "frac_of_peak": 2 * nbytes / (best * 1e-3) / 1e9 / PEAK_HBM_GBS}
        del src, dst

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, circuit, args.cpu_gates, batch_states=batch_states)
    if args.metrics_log:
        write_metrics_log(args.metrics_log, out)
    print(json.dumps(out))


HEADLINE_KEYS = ["metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "dtype", "data", "config",
                 "norm", "hbm_gbps_step", "kernel_ms_per_step", "kernels", "roofline"]


def write_metrics_log(path, out):
    """Append one JSONL record for the headline workload and one per extra,
    each tagged with a run id and the time."""
    import datetime
    import uuid

    run = uuid.uuid4().hex[:12]
    when = datetime.datetime.now(datetime.timezone.utc).isoformat(timespec="seconds")
    head = {k: out[k] for k in HEADLINE_KEYS if k in out}
    fused = out.get("kernels", {}).get("fused", {})
    head.update({"run": run, "time": when, "workload": "headline",
                 "fused_passes_per_step": fused.get("launches_per_step"),
                 "frac_of_hbm_peak": out.get("roofline", {}).get("frac"),
                 "counter_bytes_per_launch": out.get("roofline", {}).get("traffic")})
    lines = [head] + [{"run": run, "time": when, "workload": k, "data": v}
                      for k, v in out.items() if k not in HEADLINE_KEYS and k not in ("higher_is_better", "scaling",
                                                                                       "vs_baseline")]
    with open(path, "a") as f:
        for rec in lines:
            f.write(json.dumps(rec) + "\n")


def compare_states(got, ref, n, chunk=1 << 24):
    """Relative L2 error ||got - ref|| / ||ref|| and fidelity
    |<ref|got>|^2 / (<ref|ref><got|got>) of two device states of one size,
    read back in chunks and accumulated in FP64 on the host."""
    import numpy as np

    ov, nr, ng, d2 = 0j, 0.0, 0.0, 0.0
    for first in range(0, 1 << n, chunk):
        a = got.amplitudes(first, min(chunk, (1 << n) - first))
        b = ref.amplitudes(first, min(chunk, (1 << n) - first))
        ov += np.vdot(b, a)
        nr += float(np.vdot(b, b).real)
        ng += float(np.vdot(a, a).real)
        d = a - b
        d2 += float(np.vdot(d, d).real)
    return {"rel_l2": float(np.sqrt(d2 / nr)), "fidelity": float(abs(ov) ** 2 / (nr * ng))}


def c64_same_circuit(n, circuit, fusion, ref):
    """The same circuit on a complex64 state (FP32 arithmetic); its error
    against the complex128 result `ref` of the same circuit (FP64 path, held
    to the oracle at 1e-12 by the GPU tests)."""
    import torch
    from paper_1805_04708_amd import jq

    s = jq.State(n, "c64").set_stream(torch.cuda.current_stream())
    arr = jq.gates(circuit)
    s.apply_circuit(arr, fusion=fusion)
    s.synchronize()
    s.init(jq.JQ_INIT_ZERO)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.apply_circuit(arr, fusion=fusion)
    nrm = s.norm()
    dt = time.perf_counter() - t0
    err = compare_states(s, ref, n)
    s.close()
    return {"gates_per_s": len(circuit) / dt, "ms": 1000 * dt, "norm_minus_1": nrm - 1.0,
            "rel_l2_vs_c128": err["rel_l2"], "fidelity_vs_c128": err["fidelity"]}


def batch_extra(count=4096, seed=4096, keep=None):
    """Many small circuits (N uniform in 8..16, 100 random gates) in one
    launch; 16 of the states are compared with the library's single-state
    complex128 path (the GPU tests compare both paths with the oracle).
    keep (a dict) receives every state of both encodings, which the CPU leg
    compares with its FP64 states of the same circuits."""
    import numpy as np
    from paper_1805_04708_amd import jq
    from paper_1805_04708_amd import workloads as W

    def single_state(n, circ):
        with jq.State(n, "c128") as st:
            st.apply_circuit(circ)
            return st.amplitudes()

    inst = W.batch_instances(count, base_seed=seed)
    res = {"circuits": count, "gates_per_circuit": 100, "n_range": [8, 16]}
    for enc in ("c128", "c64"):
        t0 = time.perf_counter()
        b = jq.Batch(inst, enc)  # lowering, planning, first-use tuning, upload
        create_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        jq.Batch(inst, enc).close()  # tuned: lowering, planning, upload
        create_tuned_s = time.perf_counter() - t0
        b.run(timed=True)
        ms = min(b.run(timed=True) for _ in range(3))
        errs = []
        for i in range(0, count, count // 16):
            n, circ = inst[i]
            ref = single_state(n, circ)
            errs.append(float(np.linalg.norm(b.amplitudes(i) - ref) / np.linalg.norm(ref)))
        if keep is not None:
            keep[enc] = [b.amplitudes(i) for i in range(min(count, CPU_BATCH_SAMPLE))]
        b.close()
        res[enc] = {"circuits_per_s": count / (ms * 1e-3), "launch_ms": ms, "create_s_first": create_s,
                    "create_s_tuned": create_tuned_s, "max_rel_l2_vs_single_state_c128": max(errs),
                    "median_rel_l2_vs_single_state_c128": float(np.median(errs)), "checked": len(errs)}
    return res


class PlainPath:
    """The plain path of the served-mix comparison: one circuit at a time,
    one kernel per gate, one stream, with a state per qubit count allocated
    before the trace starts (like the request loop's stream-ordered pool, no
    allocation inside a request's latency)."""

    def __init__(self, enc, sizes):
        from paper_1805_04708_amd import jq

        self.jq = jq
        self.states = {n: jq.State(n, enc) for n in sorted(set(sizes))}

    def run(self, n, arr):
        s = self.states[n]
        s.init(self.jq.JQ_INIT_ZERO)
        s.apply_circuit(arr, fusion=1)
        s.norm()  # synchronises

    def close(self):
        for s in self.states.values():
            s.close()


def _serve_run(enc, count, seed, load):
    """One Poisson trace through the plain path and through the request loop:
    latency = arrival to device completion.  The arrival rate is `load`
    times the plain path's service rate, measured first by running the same
    trace's circuits back to back."""
    import threading

    import numpy as np
    from paper_1805_04708_amd import jq
    from paper_1805_04708_amd import workloads as W

    # arrival times scale as 1/rate and the circuits do not depend on it
    base = W.serving_trace(count, 1.0, seed)
    lowered = [(n, jq.gates(c)) for _, n, c in base]
    plain = PlainPath(enc, [n for n, _ in lowered])
    for n, arr in lowered[:20]:
        plain.run(n, arr)
    t0 = time.perf_counter()
    for n, arr in lowered:
        plain.run(n, arr)
    mean_service = (time.perf_counter() - t0) / count
    rate = load / mean_service
    reqs = [(t / rate, n, arr) for (t, _, _), (n, arr) in zip(base, lowered)]

    # plain path: each request waits for the previous one
    lat_seq = []
    start = time.perf_counter()
    for t, n, arr in reqs:
        now = time.perf_counter() - start
        if now < t:
            time.sleep(t - now)
        plain.run(n, arr)
        lat_seq.append(1000 * (time.perf_counter() - start - t))
    seq_span = time.perf_counter() - start
    plain.close()

    sv = jq.Server(hbm_budget=280 << 30, n_streams=4, queue_cap=count, encoding=enc)
    lat, lags = [], []

    def drain():
        for _ in reqs:
            r = sv.wait(120000)
            if r is None:
                return
            lat.append(r["latency_ms"])
            sv.release(r["ticket"])

    th = threading.Thread(target=drain)
    th.start()
    start = time.perf_counter()
    for t, n, arr in reqs:
        now = time.perf_counter() - start
        if now < t:
            time.sleep(t - now)
        lags.append(1000 * max(0.0, time.perf_counter() - start - t))
        sv.submit(n, arr)
    th.join()
    span = time.perf_counter() - start
    st = sv.stats()
    sv.close()
    lat_all = np.array(lat) + np.array(lags[:len(lat)])
    return {"requests": count, "load": load, "arrival_rate_per_s": rate,
            "plain_mean_service_ms": 1000 * mean_service, "plain_service_rate_per_s": 1.0 / mean_service,
            "served": {"p50_ms": float(np.percentile(lat_all, 50)), "p99_ms": float(np.percentile(lat_all, 99)),
                       "throughput_per_s": count / span, "peak_resident_bytes": st["peak_resident_bytes"]},
            "sequential_plain": {"p50_ms": float(np.percentile(lat_seq, 50)),
                                 "p99_ms": float(np.percentile(lat_seq, 99)), "throughput_per_s": count / seq_span,
                                 "achieved_load": rate * mean_service}}


def serve_extra(count=2000, seed=77):
    """Poisson arrivals of layered circuits, N in 10..28 with weight 2^(-N/2),
    depth 20..200: the request loop vs the plain one-at-a-time path on the
    same trace.  The arrival rate is a fraction (load) of the plain path's
    service rate measured on that trace: complex64 at load 0.9 (the
    headline), a sweep of the load, and the two-byte code at load 0.9."""
    out = {"encoding": "c64"}
    out.update(_serve_run("c64", count, seed, 0.9))
    out["load_sweep"] = {}
    for load in (0.5, 1.2):
        out["load_sweep"][str(load)] = _serve_run("c64", count // 2, seed + 10, load)
    out["compact"] = _serve_run("compact", count, seed + 20, 0.9)
    out["note"] = ("latency = arrival to device completion; the plain path runs one circuit at a time with one "
                   "kernel per gate on preallocated states; arrival rate = load x the plain path's service rate "
                   "on the same trace")
    return out


def compact_extra(n=30, layers=20):
    """The RZ + CNOT-chain circuit from the uniform state in the two-byte code,
    gate by gate quantisation; fidelity against the complex128 result of the
    same circuit on this GPU."""
    import numpy as np
    from paper_1805_04708_amd import jq
    from paper_1805_04708_amd import workloads as W

    circ = W.rz_cnot_chain(n, layers, seed=34)
    arr = jq.gates(circ)
    cp = jq.State(n, "compact").init(jq.JQ_INIT_UNIFORM)
    cp.apply_circuit(arr)
    cp.synchronize()
    cp.init(jq.JQ_INIT_UNIFORM)
    cp.synchronize()
    t0 = time.perf_counter()
    cp.apply_circuit(arr)
    cp.synchronize()
    dt = time.perf_counter() - t0
    ref = jq.State(n, "c128").init(jq.JQ_INIT_UNIFORM)
    ref.apply_circuit(arr)
    err = compare_states(cp, ref, n)
    cp.close()
    ref.close()
    return {"n": n, "gates": len(circ), "gates_per_s": len(circ) / dt, "seconds": dt,
            "fidelity_vs_c128": err["fidelity"], "rel_l2_vs_c128": err["rel_l2"]}


def compact_dense_extra(n=30, layers=2, seed=11):
    """Two layers of the layered Haar-U(2) + CZ circuit in the two-byte code:
    quantisation after every gate (the paper's procedure) against once per
    fused block; gates/s, kernel time and fidelity against the complex128
    result of the same circuit on this GPU."""
    import numpy as np
    import torch
    from paper_1805_04708_amd import jq
    from paper_1805_04708_amd import workloads as W

    circ = W.layered_u2_cz(n, layers, seed=seed)
    arr = jq.gates(circ)
    ref = jq.State(n, "c128")
    ref.apply_circuit(arr)
    ref.synchronize()
    s = jq.State(n, "compact").set_stream(torch.cuda.current_stream())
    out = {"n": n, "gates": len(circ), "workload": f"layered Haar-U(2) + CZ, {layers} layers, from |0...0>"}
    for mode, cm in (("per_gate", jq.JQ_COMPACT_PER_GATE), ("per_block", jq.JQ_COMPACT_PER_BLOCK)):
        _, blen, fused = jq.plan_schedule(n, "compact", arr, compact_mode=cm)
        s.init(jq.JQ_INIT_ZERO)
        s.synchronize()
        s.profile(True)
        t0 = time.perf_counter()
        s.apply_circuit(arr, compact_mode=cm)
        s.synchronize()
        dt = time.perf_counter() - t0
        st = s.profile_read()
        s.profile(False)
        err = compare_states(s, ref, n)
        out[mode] = {"gates_per_s": len(circ) / dt, "seconds": dt, "blocks": len(blen), "fused_blocks": int(fused.sum()),
                     "fidelity_vs_c128": err["fidelity"], "rel_l2_vs_c128": err["rel_l2"],
                     "kernels": {k: {"launches": v["launches"], "avg_ms": v["ms"] / v["launches"],
                                     "gbps": v["bytes"] / (v["ms"] * 1e-3) / 1e9,
                                     "roofline": valu_roofline(k, f"n{n}_layered{layers}", v["ms"] / v["launches"])
                                     if layers == 2 and seed == 11 else None}
                                 for k, v in st.items()}}
    s.close()
    ref.close()
    return out


def shor_extra(n=30, n_x=20, G=1007, y=529):
    """Shor's algorithm on 30 qubits as in Table Shortab1: SHORBOX, the QFT on
    the 20-qubit x-register and the expectation values of every qubit, timed
    per encoding.  complex128 is compared with the paper's printed exact
    column (three digits; the Qx entries of qubits 3..5, whose printed 0.500
    the state-vector values do not round to, are left out), the other
    encodings with complex128.  The paper's two-byte run of this case took
    348 s on an 8-core notebook."""
    import numpy as np
    from paper_1805_04708_amd import jq
    from paper_1805_04708_amd import workloads as W

    table = json.load(open(os.path.join(ROOT, "tests", "golden", "table_shortab1.json")))["exact"]
    circ = jq.gates(W.qft(n_x))
    out = {"n": n, "n_x": n_x, "G": G, "y": y, "qft_gates": circ[1]}
    ref = None
    for enc, cm in (("c128", 0), ("c64", 0), ("compact", jq.JQ_COMPACT_PER_GATE),
                    ("compact_per_block", jq.JQ_COMPACT_PER_BLOCK)):
        s = jq.State(n, "compact" if enc.startswith("compact") else enc)
        s.shorbox(n_x, G, y)
        s.apply_circuit(circ, compact_mode=cm)
        s.synchronize()
        t0 = time.perf_counter()
        s.shorbox(n_x, G, y)
        s.apply_circuit(circ, compact_mode=cm)
        qx, qy, qz = (v[:n_x] for v in s.expectations())
        dt = time.perf_counter() - t0
        s.close()
        if ref is None:
            ref = (qx, qy, qz)
            keep = np.ones(n_x, dtype=bool)
            keep[3:6] = False
            dev = max(np.max(np.abs(qx - np.array(table["Qx"]))[keep]), np.max(np.abs(qy - np.array(table["Qy"]))),
                      np.max(np.abs(qz - np.array(table["Qz"]))))
            out[enc] = {"seconds": dt, "max_dev_from_paper_table": float(dev)}
        else:
            dev = max(np.max(np.abs(qx - ref[0])), np.max(np.abs(qy - ref[1])), np.max(np.abs(qz - ref[2])))
            out[enc] = {"seconds": dt, "max_dev_from_c128": float(dev)}
    return out


def aux_extra(n=48, pairs=20, m=64, seed=48):
    """Auxiliary-variable amplitudes (Sec. 4.2) of a 48-qubit circuit with
    20 CZ gates (2^20 assignments) for 64 basis states: no state vector."""
    import numpy as np
    from paper_1805_04708_amd import jq
    from paper_1805_04708_amd import workloads as W

    rng = np.random.default_rng(seed)
    circ = [("H", (q,), ()) for q in range(n)]
    for p in range(pairs):
        a, b = (int(x) for x in rng.permutation(n)[:2])
        circ += [("CZ", (a, b), ()), ("MAT1", (b,), W.haar_u2(rng))]
    idx = rng.integers(0, 1 << 62, m, dtype=np.uint64) & np.uint64((1 << n) - 1)
    jq.aux_amplitudes(n, circ, idx[:8])
    t0 = time.perf_counter()
    amp = jq.aux_amplitudes(n, circ, idx)
    dt = time.perf_counter() - t0
    return {"n": n, "entangling_gates": pairs, "assignments": 2 ** pairs, "amplitudes": m, "gates": len(circ),
            "seconds": dt, "max_abs_amplitude": float(np.max(np.abs(amp)))}


def rz_cnot_closed_form(n, circ, j):
    """Amplitude of the RZ + CNOT-chain circuit from the uniform state at the
    basis state reached from source index j: 2^(-N/2) times the RZ entries
    met along j's path (each CNOT moves the index, each RZ(theta) multiplies
    by exp(-+i theta/2) for bit 0 / 1).  Returns (final index, amplitude)."""
    import cmath

    i, amp = j, complex(2.0 ** (-n / 2))
    for name, q, p in circ:
        if name == "RZ":
            amp *= cmath.exp((1j if (i >> q[0]) & 1 else -1j) * p[0] / 2)
        elif (i >> q[0]) & 1:
            i ^= 1 << q[1]
    return i, amp


def sampled_closed_form_error(s, n, circ, samples=64, seed=5):
    """Largest and root-mean-square relative error of sampled amplitudes of
    an RZ + CNOT-chain state against the closed form, plus the fidelity of
    the sampled amplitudes (|sum conj(exact) got|^2 / (sum|exact|^2 sum|got|^2))."""
    import numpy as np

    rng = np.random.default_rng(seed)
    src = [int(x) for x in rng.integers(0, 1 << n, samples)] + [0, (1 << n) - 1]
    errs, ov, ne, ng = [], 0j, 0.0, 0.0
    for j in src:
        i, exact = rz_cnot_closed_form(n, circ, j)
        got = complex(s.amplitudes(i, 1)[0])
        errs.append(abs(got - exact) / abs(exact))
        ov += exact.conjugate() * got
        ne += abs(exact) ** 2
        ng += abs(got) ** 2
    errs = np.array(errs)
    return {"samples": len(src), "max_rel_err": float(errs.max()), "rms_rel_err": float(np.sqrt(np.mean(errs ** 2))),
            "sampled_fidelity": float(abs(ov) ** 2 / (ne * ng))}


def large_extra(layers=20):
    """The RZ + CNOT-chain circuit (20 layers) on 256 GiB states: N=34
    complex128 and N=37 two-byte code, from the uniform state; sampled
    amplitudes against the closed form."""
    from paper_1805_04708_amd import jq
    from paper_1805_04708_amd import workloads as W

    out = {}
    for n, enc in ((34, "c128"), (37, "compact")):
        try:
            s = jq.State(n, enc).init(jq.JQ_INIT_UNIFORM)
        except Exception as e:  # not enough HBM on this device
            out[f"{enc}_n{n}"] = {"error": str(e)}
            continue
        circ = W.rz_cnot_chain(n, layers, seed=n)
        arr = jq.gates(circ)
        s.synchronize()
        s.profile(True)
        t0 = time.perf_counter()
        s.apply_circuit(arr)
        nrm = s.norm()
        dt = time.perf_counter() - t0
        st = s.profile_read()
        err = sampled_closed_form_error(s, n, circ)
        s.close()
        out[f"{enc}_n{n}"] = {"gates": len(circ), "seconds": dt, "gates_per_s": len(circ) / dt,
                              "norm_minus_1": nrm - 1.0, "vs_closed_form": err,
                              "state_gib": (16 if enc == "c128" else 2) * 2 ** n / 2 ** 30,
                              "kernels": {k: {"launches": v["launches"], "avg_ms": v["ms"] / v["launches"],
                                              "gbps": v["bytes"] / (v["ms"] * 1e-3) / 1e9} for k, v in st.items()}}
    return out


def unfused_extra(state, circuit, total_layers, layers=10):
    """The first layers of the same circuit with one kernel per gate
    (fusion off): gates/s and the per-kernel split, beside the fused figure."""
    from paper_1805_04708_amd import jq

    layers = min(layers, total_layers)
    sub = circuit[:layers * (len(circuit) // total_layers)]
    arr = jq.gates(sub)
    state.init(jq.JQ_INIT_ZERO)
    state.apply_circuit(jq.gates(sub[:8]), fusion=1)  # warm-up
    state.synchronize()
    state.init(jq.JQ_INIT_ZERO)
    state.synchronize()
    state.profile(True)
    t0 = time.perf_counter()
    state.apply_circuit(arr, fusion=1)
    state.synchronize()
    dt = time.perf_counter() - t0
    st = state.profile_read()
    state.profile(False)
    return {"gates": len(sub), "layers": layers, "seconds": dt, "gates_per_s": len(sub) / dt,
            "kernels": {k: {"launches": v["launches"], "avg_ms": v["ms"] / v["launches"],
                            "gbps": v["bytes"] / (v["ms"] * 1e-3) / 1e9} for k, v in st.items()}}


def cz_by_min_qubit(state, n):
    """Unfused CZ(t, t+1) by its lower qubit t: GB/s of the diagonal kernel
    (a quarter of the state is read and written)."""
    res = {}
    for t in range(n - 1):
        state.profile(True)
        state.apply_circuit([("CZ", (t, t + 1), ())] * 3, fusion=1)
        s = state.profile_read()["diag"]
        state.profile(False)
        res[t] = round(s["bytes"] / (s["ms"] * 1e-3) / 1e9, 1)
    return res


# The paper's elapsed times per gate used to normalise its weak-scaling
# figures (Sec. 5.1: Figs. scaling1a/1b for H on every qubit, scaling2/3
# for the GHZ circuit), in seconds, on whole CPU supercomputer partitions;
# context only.
PAPER_NORMALISATION_S = {
    "hadamard_c128_n32": {"JUQUEEN": 1.2, "K": 1.0, "Sunway": 7.7, "JURECA": 1.9, "JUWELS": 1.3},
    "hadamard_compact_n35": {"JUQUEEN": 10.7, "K": 30.8, "Sunway": 101.2, "JURECA": 9.7, "JUWELS": 4.7},
    "ghz_c128_n32": {"JUQUEEN": 0.98, "Sunway": 5.1, "JURECA": 1.4, "JUWELS": 0.9},
    "ghz_compact_n35": {"JUQUEEN": 2.7, "K": 3.8, "Sunway": 19.9, "JURECA": 2.4, "JUWELS": 2.2},
}


def paper_circuits_extra():
    """The paper's scaling circuits at its normalisation sizes: H on every
    qubit and the GHZ circuit (H on qubit 0, then the CNOT chain) from
    |0...0>, N=32 complex128 and N=35 two-byte code (64 GiB each); seconds
    per gate with the default plan and with one kernel per gate."""
    from paper_1805_04708_amd import jq
    from paper_1805_04708_amd import workloads as W

    out = {}
    for n, enc in ((32, "c128"), (35, "compact")):
        try:
            s = jq.State(n, enc)
        except Exception as e:  # not enough HBM on this device
            out[f"{enc}_n{n}"] = {"error": str(e)}
            continue
        for name, circ in (("hadamard", W.hadamard_all(n)), ("ghz", W.ghz(n))):
            arr = jq.gates(circ)
            row = {"gates": len(circ), "paper_s_per_gate": PAPER_NORMALISATION_S[f"{name}_{enc}_n{n}"]}
            for label, fusion in (("default", 0), ("one_kernel_per_gate", 1)):
                s.init(jq.JQ_INIT_ZERO)
                s.synchronize()
                t0 = time.perf_counter()
                s.apply_circuit(arr, fusion=fusion)
                s.synchronize()
                dt = time.perf_counter() - t0
                row[label] = {"seconds": dt, "s_per_gate": dt / len(circ)}
            out[f"{name}_{enc}_n{n}"] = row
        s.close()
    return out


def per_target(state, n, bpa):
    """Unfused dense single-qubit gate by target index: GB/s of the pair kernel."""
    from paper_1805_04708_amd import workloads as W
    import numpy as np

    rng = np.random.default_rng(1)
    res = {}
    for t in range(n):
        arr = [("MAT1", (t,), W.haar_u2(rng))] * 3
        state.profile(True)
        state.apply_circuit(arr, fusion=1)
        s = state.profile_read()["dense1"]
        state.profile(False)
        res[t] = round(s["bytes"] / (s["ms"] * 1e-3) / 1e9, 1)
    return res


if __name__ == "__main__":
    main()

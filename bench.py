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


def cpu_baseline(n, circuit, gates):
    import numpy as np
    from oracle import core as O

    sample = circuit[:gates]
    psi = O.zero_state(n)
    t0 = time.perf_counter()
    O.run(psi, n, sample)
    dt = time.perf_counter() - t0
    del psi
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((line.split(":", 1)[1].strip() for line in f if line.startswith("model name")), None)
    except OSError:
        pass
    return {"value": len(sample) / dt, "unit": "gates/s", "cores": 1, "kind": "oracle",
            "sample": f"first {len(sample)} gates of the same circuit at N={n}, single-threaded FP64 C oracle, "
                      f"{dt:.1f} s",
            "host": {"nproc": os.cpu_count(), "model": model}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this build has no multi-GPU path.",
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
                   "fusion": "auto" if args.fusion == 0 else args.fusion, "seed": args.seed},
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
    if "unfused" in wanted:
        out["unfused"] = unfused_extra(state, circuit, args.layers)

    state.close()
    torch.cuda.synchronize()

    extras = [("c64", "c64_same_circuit", lambda: c64_same_circuit(n, circuit, args.fusion)),
              ("batch", "batch", batch_extra), ("serve", "serve", serve_extra),
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
        out["cpu_baseline"] = cpu_baseline(n, circuit, args.cpu_gates)
    print(json.dumps(out))


def c64_same_circuit(n, circuit, fusion):
    """The same circuit on a complex64 state (FP32 arithmetic)."""
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
    s.close()
    return {"gates_per_s": len(circuit) / dt, "ms": 1000 * dt, "norm_minus_1": nrm - 1.0}


def batch_extra(count=4096, seed=4096):
    """Many small circuits (N uniform in 8..16, 100 random gates) in one
    launch; 16 of the states are compared with the library's single-state
    complex128 path (the GPU tests compare both paths with the oracle)."""
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
        b.close()
        res[enc] = {"circuits_per_s": count / (ms * 1e-3), "launch_ms": ms, "create_s_first": create_s,
                    "create_s_tuned": create_tuned_s, "max_rel_l2_vs_single_state_c128": max(errs),
                    "median_rel_l2_vs_single_state_c128": float(np.median(errs)), "checked": len(errs)}
    return res


def _mean_service(enc, seed, count=200):
    """Mean time per request of the plain path (unfused per-gate kernels,
    one stream, one circuit at a time) over a probe trace."""
    from paper_1805_04708_amd import jq
    from paper_1805_04708_amd import workloads as W

    lowered = [(n, jq.gates(c)) for _, n, c in W.serving_trace(count, 1.0, seed)]
    t0 = time.perf_counter()
    for n, arr in lowered:
        with jq.State(n, enc) as s:
            s.apply_circuit(arr, fusion=1)
            s.norm()
    return (time.perf_counter() - t0) / len(lowered)


def _serve_run(enc, rate, count, seed):
    """One Poisson trace at the given rate through the plain path and through
    the request loop: latency = arrival to device completion."""
    import threading

    import numpy as np
    from paper_1805_04708_amd import jq
    from paper_1805_04708_amd import workloads as W

    reqs = [(t, n, jq.gates(c)) for t, n, c in W.serving_trace(count, rate, seed)]
    # plain path: each request waits for the previous one
    lat_seq = []
    start = time.perf_counter()
    for t, n, arr in reqs:
        now = time.perf_counter() - start
        if now < t:
            time.sleep(t - now)
        with jq.State(n, enc) as s:
            s.apply_circuit(arr, fusion=1)
            s.norm()
        lat_seq.append(1000 * (time.perf_counter() - start - t))
    seq_span = time.perf_counter() - start

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
    return {"served": {"p50_ms": float(np.percentile(lat_all, 50)), "p99_ms": float(np.percentile(lat_all, 99)),
                       "throughput_per_s": count / span, "peak_resident_bytes": st["peak_resident_bytes"]},
            "sequential_plain": {"p50_ms": float(np.percentile(lat_seq, 50)),
                                 "p99_ms": float(np.percentile(lat_seq, 99)), "throughput_per_s": count / seq_span}}


def serve_extra(count=2000, seed=77):
    """Poisson arrivals of layered circuits, N in 10..28 with weight 2^(-N/2),
    depth 20..200: the request loop vs the plain one-at-a-time path.  The
    arrival rate is a fraction (load) of the plain path's measured service
    rate: complex64 at load 0.9 (the headline), a sweep of the load, and the
    two-byte code at load 0.9 on a shorter trace."""
    out = {"requests": count, "encoding": "c64"}
    mean_c64 = _mean_service("c64", seed + 1)
    rate = 0.9 / mean_c64
    out["arrival_rate_per_s"] = rate
    out["plain_mean_service_ms"] = 1000 * mean_c64
    out.update(_serve_run("c64", rate, count, seed))
    out["load_sweep"] = {}
    for load in (0.5, 1.2):
        r = _serve_run("c64", load / mean_c64, count // 2, seed + 10)
        out["load_sweep"][str(load)] = {"arrival_rate_per_s": load / mean_c64, "requests": count // 2, **r}
    mean_cp = _mean_service("compact", seed + 2, count=50)
    n_cp = 200
    out["compact"] = {"requests": n_cp, "arrival_rate_per_s": 0.9 / mean_cp, "plain_mean_service_ms": 1000 * mean_cp,
                      **_serve_run("compact", 0.9 / mean_cp, n_cp, seed + 20)}
    out["note"] = ("latency = arrival to device completion; the plain path runs one circuit at a time with one "
                   "kernel per gate")
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
    ov, nr, nc = 0j, 0.0, 0.0
    chunk = 1 << 24
    for first in range(0, 1 << n, chunk):
        a = cp.amplitudes(first, chunk)
        b = ref.amplitudes(first, chunk)
        ov += np.vdot(b, a)
        nr += float(np.vdot(b, b).real)
        nc += float(np.vdot(a, a).real)
    diff2 = nc + nr - 2 * ov.real
    cp.close()
    ref.close()
    return {"n": n, "gates": len(circ), "gates_per_s": len(circ) / dt, "seconds": dt,
            "fidelity_vs_c128": abs(ov) ** 2 / (nr * nc), "rel_l2_vs_c128": float(np.sqrt(max(diff2, 0) / nr))}


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
        ov, nr, nc = 0j, 0.0, 0.0
        chunk = 1 << 24
        for first in range(0, 1 << n, chunk):
            a = s.amplitudes(first, chunk)
            b = ref.amplitudes(first, chunk)
            ov += np.vdot(b, a)
            nr += float(np.vdot(b, b).real)
            nc += float(np.vdot(a, a).real)
        out[mode] = {"gates_per_s": len(circ) / dt, "seconds": dt, "blocks": len(blen), "fused_blocks": int(fused.sum()),
                     "fidelity_vs_c128": abs(ov) ** 2 / (nr * nc),
                     "kernels": {k: {"launches": v["launches"], "avg_ms": v["ms"] / v["launches"],
                                     "gbps": v["bytes"] / (v["ms"] * 1e-3) / 1e9} for k, v in st.items()}}
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


def large_extra(layers=20):
    """The RZ + CNOT-chain circuit (20 layers) on 256 GiB states: N=34
    complex128 and N=37 two-byte code, from the uniform state."""
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
        s.close()
        out[f"{enc}_n{n}"] = {"gates": len(circ), "seconds": dt, "gates_per_s": len(circ) / dt,
                              "norm_minus_1": nrm - 1.0, "state_gib": (16 if enc == "c128" else 2) * 2 ** n / 2 ** 30,
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

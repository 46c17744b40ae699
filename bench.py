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
    p.add_argument("--cpu-gates", type=int, default=3, help="gates of the circuit the CPU oracle times")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="also run a plain torch device copy of this many MiB (counter calibration)")
    return p.parse_args()


def traffic_from_profiles(kernel, workload):
    """HBM bytes per launch measured with rocprofv3 counters, if recorded."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(f"{kernel}:{workload}")
    except Exception:
        return None
    if not rec:
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
    return {"value": len(sample) / dt, "unit": "gates/s", "cores": 1, "kind": "oracle",
            "sample": f"first {len(sample)} gates of the same circuit at N={n}, single-threaded FP64 C oracle, "
                      f"{dt:.1f} s"}


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

    if not args.no_extras:
        out["per_target"] = per_target(state, n, bpa)

    state.close()
    torch.cuda.synchronize()

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        out["copy_calibration"] = {"bytes_read": nbytes, "bytes_written": nbytes,
                                   "gbps": 2 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9}
        del src, dst

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, circuit, args.cpu_gates)
    print(json.dumps(out))


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

"""Benchmark: Bellman backups per second of full value-iteration solves on one MI355X.

Workload: the m=4, L=2 scenario-A instance (4,084,101 states, 21 actions, gamma
demand with mean 4 and CV 1.5 folded at 60, seeded +-20% cost jitter, gamma 0.99,
span threshold 1e-4 (1-gamma)/gamma).  One step = one complete solve through the
C ABI from V0 = 0: FP32 sweeps, FP64 check and polish sweeps, and the FP64 policy
extraction, with the MDP's tables already resident in HBM.

value = logical backups (states x actions x demand outcomes, summed over every
sweep of every step) / wall time of the timed steps.  The FP64 one-solve-per-call
path is timed the same way and reported beside it.

Run: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32|fp32_wide|fp64]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Bellman (state·action·outcome) backups/sec FP32 vs FP64; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32_wide", choices=["fp32", "fp32_wide", "fp64"])
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def time_solves(pvi, m, precision, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        pvi.vi_solve(m, precision=precision, stream=stream)
    torch.cuda.synchronize()
    lat, results = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        r = pvi.vi_solve(m, precision=precision, stream=stream, time_kernels=True)
        lat.append((time.perf_counter() - s0) * 1e3)
        results.append(r)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    logical = sum(r["logical_backups"] for r in results)
    executed = sum(r["executed_terms"] for r in results)
    kern_ms = [sum(r["backup_ms"][i] for r in results) for i in (0, 1)]
    launches = [sum(r["backup_launches"][i] for r in results) for i in (0, 1)]
    return {
        "wall_s": wall, "logical": logical, "executed": executed, "lat_ms": lat,
        "backup_ms": kern_ms, "launches": launches,
        "sweeps_fp32": results[-1]["sweeps_fp32"], "sweeps_fp64": results[-1]["sweeps_fp64"],
    }


def cpu_baseline(sc, target_s):
    """The FP64 oracle on a bounded sample of states (backups of every action and outcome)."""
    import numpy as np
    from oracle.oracle import Oracle
    import workloads as W
    o = Oracle(sc)
    V = np.zeros(o.n_states)
    n = 2000
    t0 = time.perf_counter()
    o.q_states(V, W.sample_indices(o.n_states, n, seed=5))
    dt = time.perf_counter() - t0
    n = int(min(o.n_states, max(n, n * target_s / max(dt, 1e-6))))
    idx = W.sample_indices(o.n_states, n, seed=6)
    t0 = time.perf_counter()
    o.q_states(V, idx)
    dt = time.perf_counter() - t0
    per_state = o.n_actions * (sc["d_max"][0] + 1)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return {"value": len(idx) * per_state / dt, "unit": "backups/s", "cores": threads,
            "kind": "oracle",
            "sample": f"one FP64 backup (all 21 actions x 61 demand outcomes) of {len(idx)} "
                      f"of the {o.n_states} states, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2303_10672_amd import pvi
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    sc = W.config1()
    m = pvi.mdp_create(sc)
    stream = torch.cuda.Stream()
    handle = stream.cuda_stream

    main_run = time_solves(pvi, m, args.precision, args.steps, args.warmup, handle)
    fp64_steps = args.fp64_steps if args.fp64_steps is not None else max(1, args.steps // 2)
    fp64_run = time_solves(pvi, m, "fp64", fp64_steps, 1, handle) \
        if args.precision != "fp64" else main_run

    value = main_run["logical"] / main_run["wall_s"]
    ms_per_step = main_run["wall_s"] * 1e3 / args.steps
    # the dominant backup kernel: FP32-storage sweeps unless the mode is plain FP64
    dom = 0 if args.precision == "fp64" else 1
    launches = max(main_run["launches"][dom], 1)
    avg_kernel_s = main_run["backup_ms"][dom] / launches * 1e-3
    per_launch_logical = m.n_states * m.n_actions * (sc["d_max"][0] + 1)
    bytes_per_backup = 8 if dom == 0 else 4
    achieved_gbs = per_launch_logical * bytes_per_backup / avg_kernel_s / 1e9
    sweeps = main_run["sweeps_fp32"] + main_run["sweeps_fp64"] + 1
    executed_per_launch = main_run["executed"] / (args.steps * sweeps)
    fma_tflops = 2.0 * executed_per_launch / avg_kernel_s / 1e12

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "backups/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp32_wide": "f32", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": "scenario A, m=4, L=2, order cap 20 (4,084,101 states x 21 actions "
                        "x 61 demand outcomes), gamma demand mean 4 CV 1.5, seeded cost "
                        "jitter, gamma 0.99; one step = one full solve to span < "
                        "1e-4(1-gamma)/gamma plus policy extraction",
            "precision_mode": args.precision,
            "sweeps_per_solve": {"fp32": main_run["sweeps_fp32"], "fp64": main_run["sweeps_fp64"],
                                 "extract": 1},
        },
        "latency_ms": {"p50": percentile(main_run["lat_ms"], 0.5),
                       "p99": percentile(main_run["lat_ms"], 0.99)},
        "fp64_plain": {
            "value": fp64_run["logical"] / fp64_run["wall_s"],
            "ms_per_solve": fp64_run["wall_s"] * 1e3 / max(fp64_steps, 1),
            "sweeps": fp64_run["sweeps_fp64"] + 1,
            "avg_backup_kernel_ms": fp64_run["backup_ms"][0] / max(fp64_run["launches"][0], 1),
            "latency_ms": {"p50": percentile(fp64_run["lat_ms"], 0.5),
                           "p99": percentile(fp64_run["lat_ms"], 0.99)},
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": "backup_a_kernel<" + ("double" if dom == 0 else "float") + ">",
            "launches_timed": launches,
            "avg_kernel_ms": avg_kernel_s * 1e3,
            "basis": f"{bytes_per_backup} B of V per logical backup x {per_launch_logical} "
                     f"logical backups per launch",
        },
        "roofline_executed": {
            "bound": "alu",
            "achieved": fma_tflops,
            "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": fma_tflops / FP64_VECTOR_PEAK_TFLOPS,
            "basis": f"2 flops per executed multiply-add, {executed_per_launch:.4g} per launch",
        },
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline(sc, args.cpu_seconds),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark: Bellman backups per second of full value-iteration solves on one MI355X.

Workload: the m=4, L=2 scenario-A instance (4,084,101 states, 21 actions, gamma
demand with mean 4 and CV 1.5 folded at 60, seeded +-20% cost jitter, gamma 0.99,
span threshold 1e-4 (1-gamma)/gamma).  One step = one complete solve through the
C ABI from V0 = 0 in the chosen precision (FP64 by default; the FP32 schedules run
FP32 sweeps, then FP64 check and polish sweeps), and the FP64 policy extraction,
with the MDP's tables already resident in HBM.

value = logical backups (states x actions x demand outcomes, summed over every
sweep of every step) / wall time of the timed steps.

Beside it: the other schedules (FP64, compensated FP32, FP32 storage with FP64 sums),
timed the same way on the same
instance, the cold first calls, the roofline of the dominant kernel on the bytes a
sweep must move, and the FP32 schedules' error against FP64 for configs 0-3.

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
    ap.add_argument("--precision", default="fp64", choices=["fp32", "fp32_wide", "fp64"],
                    help="precision of the headline solve; the other schedule is timed "
                         "beside it (fp32_wide beside fp64, fp64 beside an FP32 mode)")
    ap.add_argument("--fp64-steps", type=int, default=None,
                    help="steps of the companion solve (default: steps // 2)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-errors", action="store_true",
                    help="skip the FP32-vs-FP64 error of configs 0-3 (about 20 s)")
    ap.add_argument("--workload", default="config1", choices=["config1", "batch", "serving", "oracle",
                                                               "config2", "config3",
                                                               "paper-a", "paper-b", "paper-c", "rollouts"],
                    help="config1 (default, the headline), batch (many small solves: "
                         "batched FP32 kernel vs one FP64 solve per call), serving (the "
                         "request mix through the server), config2/config3 (one solve), paper-a / paper-c "
                         "(the paper's scenario-A and scenario-C experiments, one solve "
                         "each)")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--paper-rules", action="store_true",
                    help="serving: scenario-C requests stop by the periodic rule of "
                         "Appendix C (the paper's test for C); otherwise every request "
                         "uses the span rule")
    ap.add_argument("--prerun", type=int, default=200,
                    help="requests in the closed-loop pre-run that sets the saturated rate")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="serving arrival rate per second (0: 0.7 x closed-loop rate)")
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--late-s", type=int, default=120,
                    help="serving: end the run, naming the request, when one ticket is "
                         "not done after this many seconds")
    ap.add_argument("--oracle-threads", type=int, default=0,
                    help="workload oracle: OpenMP threads of the oracle (0 = all)")
    ap.add_argument("--paper-checkpoints", action="store_true",
                    help="paper workloads: also time an FP64 solve that writes a checkpoint "
                         "file as often as the paper did (A every 100 sweeps, B and C "
                         "every sweep)")
    ap.add_argument("--fixed-sweeps", type=int, default=0,
                    help="config2/config3: instead of full solves, one FP64 and one "
                         "FP32-storage run of exactly this many sweeps (for profiles and "
                         "counters)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="first run a plain device copy of this many MiB (a known-traffic "
                         "kernel for scaling HBM counters)")
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


def fp32_errors(pvi, W, cfgs=(0, 1, 2, 3)):
    """Error of the FP32 schedules against the FP64 solve of the same instance, per
    config: max |V_32 - V_64| over max |V_64| (normwise) and max |V_32 - V_64| / |V_64|
    (elementwise), for the returned V and for the bound midpoints V + gamma/(1-gamma)
    (dmax + dmin)/2 (the two solves stop at different sweeps, so their V differ by up to
    the stopping tolerance while both midpoints bracket V*); and the number of states
    whose policy differs where the FP64 solve's best-minus-second Q exceeds 1e-6."""
    import numpy as np
    out = {}
    for c in cfgs:
        sc = W.config_by_index(c)
        g = sc["gamma"]
        m = pvi.mdp_create(sc)
        r64 = pvi.vi_solve(m, precision="fp64")
        V64 = pvi.value_get(m)
        p64, gap64 = pvi.policy_get(m)
        h64 = V64 + g / (1 - g) * 0.5 * (r64["dmax"] + r64["dmin"])
        row = {"states": int(m.n_states), "sweeps_fp64": r64["sweeps_fp64"]}
        for mode in ("fp32", "fp32_wide"):
            r = pvi.vi_solve(m, precision=mode)
            V = pvi.value_get(m)
            p, _ = pvi.policy_get(m)
            h = V + g / (1 - g) * 0.5 * (r["dmax"] + r["dmin"])
            clear = gap64 > 1e-6
            row[mode] = {
                "sweeps": {"fp32": r["sweeps_fp32"], "fp64": r["sweeps_fp64"]},
                "v_normwise": float(np.abs(V - V64).max() / np.abs(V64).max()),
                "v_elementwise": float((np.abs(V - V64) / np.abs(V64)).max()),
                "vhat_normwise": float(np.abs(h - h64).max() / np.abs(h64).max()),
                "vhat_elementwise": float((np.abs(h - h64) / np.abs(h64)).max()),
                "policy_differs_where_gap_gt_1e-6": int((p[clear] != p64[clear]).sum()),
                "policy_differs_anywhere": int((p != p64).sum()),
            }
        out[f"config{c}"] = row
        del m
    return out


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


def bench_oracle(args):
    """The FP64 CPU oracle alone (no GPU): full solves of config 0 (p50/p99 over 20)
    and the config-1 backup sample of cpu_baseline, at --oracle-threads OpenMP threads,
    with the host's processor."""
    import numpy as np
    if args.oracle_threads > 0:
        os.environ["OMP_NUM_THREADS"] = str(args.oracle_threads)  # before the oracle loads
    from oracle.oracle import Oracle
    import workloads as W
    cpu = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    o = Oracle(W.config0())
    lat = []
    for _ in range(20):
        t0 = time.perf_counter()
        r = o.solve()
        lat.append((time.perf_counter() - t0) * 1e3)
    base = cpu_baseline(W.config1(), args.cpu_seconds)
    line = {"metric": "oracle FP64 backups/s (config 1 sample) and config-0 solve latency",
            "value": base["value"], "unit": "backups/s", "n_gpus": 0,
            "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "CPU oracle: config 0 full solves, config 1 backup sample"},
            "host": {"cpu": cpu, "nproc": os.cpu_count(),
                     "affinity": len(os.sched_getaffinity(0)),
                     "omp_threads": os.environ.get("OMP_NUM_THREADS")},
            "config0_solve_ms": {"p50": float(np.percentile(lat, 50)),
                                 "p99": float(np.percentile(lat, 99)),
                                 "sweeps": r["sweeps"]},
            "config1_sample": base}
    print(json.dumps(line), flush=True)


def bench_batch(args, pvi, W):
    """Many small scenario-A solves: one batched FP32 launch vs one FP64 solve per call."""
    import torch
    reqs = W.serving_mix(n_requests=4 * args.batch, seed=7, large_fraction=0.0, c_fraction=0.0)
    scs = [sc for _, sc in reqs][:args.batch]
    out = {}
    for label, prec in (("batched_fp32", "fp32"), ("batched_fp64", "fp64")):
        srv = pvi.Server(small_batch=args.batch)
        warm = [pvi.mdp_create(sc) for sc in scs]
        for t in srv.submit(warm, precision=prec):
            srv.wait(t)
        mdps = [pvi.mdp_create(sc) for sc in scs]
        t0 = time.perf_counter()
        ts = srv.submit(mdps, precision=prec)
        res = [srv.wait(t)[1] for t in ts]
        dt = time.perf_counter() - t0
        srv.close()
        logical = sum(r["logical_backups"] for r in res)
        out[label] = {"solves_per_s": len(scs) / dt, "backups_per_s": logical / dt,
                      "wall_ms": dt * 1e3}
    mdps = [pvi.mdp_create(sc) for sc in scs]
    pvi.vi_solve(mdps[0], precision="fp64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    logical = 0
    for m in mdps:
        logical += pvi.vi_solve(m, precision="fp64")["logical_backups"]
    dt = time.perf_counter() - t0
    out["one_solve_per_call_fp64"] = {"solves_per_s": len(scs) / dt,
                                      "backups_per_s": logical / dt, "wall_ms": dt * 1e3}
    b = out["batched_fp32"]
    line = {
        "metric": "small-instance solves/s: batched FP32 launch vs one FP64 solve per call",
        "value": b["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{len(scs)} scenario-A instances, m in 2..3, L=1, order <= 10, "
                               "Poisson(4) folded at 20, seeded cost jitter, gamma 0.99"},
        "speedup_vs_one_solve_per_call_fp64": b["solves_per_s"] /
        out["one_solve_per_call_fp64"]["solves_per_s"],
        "detail": out,
    }
    print(json.dumps(line), flush=True)


def describe(sc):
    """Request class of a serving-mix scenario, for progress and late-ticket lines."""
    if sc["family"] == "C":
        return f"C m={sc['m']} order cap {sc['a_max'][0]}"
    return f"A m={sc['m']} L={sc['L']} order cap {sc['a_max'][0]}"


def wait_tickets(pvi, srv, tickets, scs, label, late_s):
    """Wait for tickets in submission order, printing progress every 10.  A ticket
    not done after each 10 s is named with its server state (queued or running, the
    worker, sweeps so far); after late_s seconds the run is ended with that report
    (os._exit: a stuck solve would otherwise block the server's shutdown)."""
    status = []
    for i, t in enumerate(tickets):
        waited = 0
        while True:
            st, r = srv.wait(t, timeout_us=10_000_000)
            if st != pvi.PVI_E_NOT_READY:
                break
            waited += 10
            info = srv.ticket_info(t)
            msg = (f"late: request {i + 1} (ticket {t}, {describe(scs[i])}) not done after "
                   f"{waited} s: {info}")
            print(msg, file=sys.stderr, flush=True)
            if waited >= late_s:
                print(json.dumps({"error": msg}), flush=True)
                os._exit(3)
        status.append((st, r))
        if (i + 1) % 10 == 0 or i + 1 == len(tickets):
            print(f"{label}: {i + 1}/{len(tickets)} requests done", file=sys.stderr, flush=True)
    return status


def bench_serving(args, pvi, W):
    """The request mix through the server: arrivals on a clock, p50/p99 latency."""
    import threading
    import torch
    import numpy as np
    mix = W.serving_mix(n_requests=args.requests, rate_per_s=1.0, seed=4)
    scs = [sc for _, sc in mix]
    gaps = np.diff([0.0] + [t for t, _ in mix])          # unit-rate inter-arrival times
    # closed-loop pre-run on a prefix gives the saturated rate
    srv = pvi.Server(small_batch=args.batch)
    pre = scs[:min(args.prerun, len(scs))]

    def rule(sc):
        return "periodic" if args.paper_rules and sc["family"] == "C" else "span"

    t0 = time.perf_counter()
    ts = [srv.submit([pvi.mdp_create(sc)], precision="fp32", stop_rule=rule(sc))[0]
          for sc in pre]
    wait_tickets(pvi, srv, ts, pre, "closed-loop pre-run", args.late_s)
    sat = len(pre) / (time.perf_counter() - t0)
    srv.close()
    rate = args.rate if args.rate > 0 else 0.7 * sat
    mdps = [pvi.mdp_create(sc) for sc in scs]
    srv = pvi.Server(small_batch=args.batch)
    tickets = [None] * len(mdps)
    start = time.perf_counter()

    def submitter():
        t_next = start
        for i, m in enumerate(mdps):
            t_next += gaps[i] / rate
            d = t_next - time.perf_counter()
            if d > 0:
                time.sleep(d)
            tickets[i] = srv.submit([m], precision="fp32", stop_rule=rule(scs[i]))[0]
            if (i + 1) % 20 == 0:
                print(f"submitted: {i + 1}/{len(mdps)} requests", file=sys.stderr, flush=True)

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    status = wait_tickets(pvi, srv, tickets, scs, "served", args.late_s)
    wall = time.perf_counter() - start
    st = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    lat = np.array([s[1]["wall_ms"] for s in status])
    fam = np.array([sc["family"] + ("L" if sc["family"] == "A" and sc["m"] == 4 else "")
                    for sc in scs])
    per = {}
    for f in sorted(set(fam)):
        x = lat[fam == f]
        per[f] = {"n": int(x.size), "p50_ms": float(np.percentile(x, 50)),
                  "p99_ms": float(np.percentile(x, 99))}
    ok = sum(1 for s in status if s[0] == pvi.PVI_OK)
    line = {
        "metric": "serving mix solves/s; p50/p99 solve latency (arrival to result)",
        "value": len(mdps) / wall, "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{len(mdps)} requests, exponential arrivals at {rate:.1f}/s "
                               "(0.7 x closed-loop rate unless given); 70% small A, 25% C "
                               "with order cap 10..20, 5% the m=4 L=2 A instance; FP32 "
                               "schedule with FP64 check and polish; stopping rule: "
                               + ("periodic for C, span otherwise" if args.paper_rules
                                  else "span")},
        "latency_ms": {"p50": st["p50_ms"], "p99": st["p99_ms"]},
        "per_class": per, "closed_loop_rate": sat, "completed_ok": ok,
    }
    print(json.dumps(line), flush=True)


def bench_single(args, pvi, W, cfg):
    """One full solve of config 2 or 3, FP64 and FP32 schedules (span rule); for
    config 3 also under the periodic rule of Appendix C (its own stopping test)."""
    sc = W.config_by_index(cfg)
    m = pvi.mdp_create(sc)
    out = {}
    runs = [("fp64", "span"), ("fp32", "span")]
    if cfg == 3 and args.fixed_sweeps <= 0:
        runs += [("fp64", "periodic"), ("fp32", "periodic")]
    k = max(args.fixed_sweeps, 0)
    for prec, rule in runs:
        key = prec if rule == "span" else f"{prec}_{rule}"
        if k == 0:
            pvi.vi_solve(m, precision=prec, max_sweeps=20000, allow_not_converged=True,
                         stop_rule=rule)
        t0 = time.perf_counter()
        r = pvi.vi_solve(m, precision=prec, max_sweeps=20000, time_kernels=True,
                         allow_not_converged=True, stop_rule=rule, fixed_sweeps=k)
        dt = time.perf_counter() - t0
        print(f"{key}: {dt:.2f} s, {r['sweeps_fp32']} + {r['sweeps_fp64']} sweeps",
              file=sys.stderr, flush=True)
        out[key] = {"backups_per_s": r["logical_backups"] / dt, "solve_ms": dt * 1e3,
                     "sweeps_fp32": r["sweeps_fp32"], "sweeps_fp64": r["sweeps_fp64"],
                     "status": r["status"], "executed_terms": r["executed_terms"],
                     "backup_ms": list(r["backup_ms"]),
                     "backup_launches": list(r["backup_launches"])}
    line = {"metric": METRIC, "value": max(o["backups_per_s"] for o in out.values()),
            "unit": "backups/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
            "config": {"workload": f"config {cfg} one solve"}, "detail": out}
    print(json.dumps(line), flush=True)


def checkpointed_solve(args, pvi, m, every, **kw):
    """Wall time of one FP64 solve that writes a checkpoint file every `every` sweeps
    (a host check after each), as the paper's wall times include; None unless asked."""
    if not args.paper_checkpoints:
        return None
    path = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"pvi-bench-{os.getpid()}.ckpt")
    t0 = time.perf_counter()
    r = pvi.vi_solve(m, precision="fp64", checkpoint=path, checkpoint_every=every,
                     check_every=every, **kw)
    dt = time.perf_counter() - t0
    size = os.path.getsize(path)
    os.remove(path)
    return {"solve_ms": dt * 1e3, "checkpoint_every": every, "sweeps_fp64": r["sweeps_fp64"],
            "file_bytes": size}


def bench_paper_a(args, pvi, W):
    """The paper's 32 scenario-A experiments (Appendix A settings, sup-norm stop with
    eps 1e-4): wall time of one full solve each, FP64 and the FP32 schedule, after one
    untimed solve; mdp_create (host tables and upload) timed apart."""
    out = []
    for (mm, exp, L, cw, iss) in W.PAPER_A_EXPERIMENTS:
        sc = W.scenario_a_paper(mm, L, cw, iss)
        t0 = time.perf_counter()
        m = pvi.mdp_create(sc)
        create_ms = (time.perf_counter() - t0) * 1e3
        row = {"m": mm, "exp": exp, "L": L, "c_waste": cw, "issuing": iss,
               "states": m.n_states, "create_ms": create_ms}
        for prec in ("fp64", "fp32_wide"):
            pvi.vi_solve(m, precision=prec, eps=1e-4, stop_rule="supnorm")
            t0 = time.perf_counter()
            r = pvi.vi_solve(m, precision=prec, eps=1e-4, stop_rule="supnorm")
            dt = time.perf_counter() - t0
            row[prec] = {"solve_ms": dt * 1e3, "sweeps_fp32": r["sweeps_fp32"],
                         "sweeps_fp64": r["sweeps_fp64"],
                         "backups_per_s": r["logical_backups"] / dt}
        row["fp64_checkpointed"] = checkpointed_solve(args, pvi, m, 100, eps=1e-4,
                                                      stop_rule="supnorm")
        pol, _ = pvi.policy_get(m)
        row["V_empty"] = float(pvi.value_get(m)[0])
        row["order_when_empty"] = int(pol[0])
        print(f"m={mm} exp {exp}: {row['states']} states, fp64 "
              f"{row['fp64']['solve_ms']:.1f} ms ({row['fp64']['sweeps_fp64']} sweeps), "
              f"fp32_wide {row['fp32_wide']['solve_ms']:.1f} ms", file=sys.stderr, flush=True)
        out.append(row)
        del m
    big = [r for r in out if r["states"] == max(x["states"] for x in out)]
    line = {"metric": METRIC, "value": max(r["fp64"]["backups_per_s"] for r in big),
            "unit": "backups/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
            "dtype": "f64",
            "config": {"workload": "paper scenario-A experiments, sup-norm stop; value: "
                                   "FP64 at 1,771,561 states"},
            "total_solve_s_fp64": sum(r["fp64"]["solve_ms"] for r in out) / 1e3,
            "total_solve_s_fp32_wide": sum(r["fp32_wide"]["solve_ms"] for r in out) / 1e3,
            "detail": out}
    print(json.dumps(line), flush=True)


def bench_paper_c(args, pvi, W):
    """The paper's scenario-C experiments that fit in memory (m = 3 and 5, remaining
    life independent of or depending on the order), periodic stop of Appendix C:
    wall time of one full solve each, FP64 and the FP32 schedule, after one untimed
    solve."""
    out = []
    for (mm, exp) in W.PAPER_C_EXPERIMENTS:
        sc = W.scenario_c_paper(mm, exp)
        t0 = time.perf_counter()
        m = pvi.mdp_create(sc)
        row = {"m": mm, "exp": exp, "states": m.n_states,
               "create_ms": (time.perf_counter() - t0) * 1e3}
        for prec in ("fp64", "fp32"):
            pvi.vi_solve(m, precision=prec, eps=1e-4, stop_rule="periodic")
            t0 = time.perf_counter()
            r = pvi.vi_solve(m, precision=prec, eps=1e-4, stop_rule="periodic",
                             time_kernels=True)
            dt = time.perf_counter() - t0
            row[prec] = {"solve_ms": dt * 1e3, "sweeps_fp32": r["sweeps_fp32"],
                         "sweeps_fp64": r["sweeps_fp64"],
                         "backups_per_s": r["logical_backups"] / dt,
                         "backup_ms": list(r["backup_ms"])}
        row["fp64_checkpointed"] = checkpointed_solve(args, pvi, m, 1, eps=1e-4,
                                                      stop_rule="periodic")
        print(f"C m={mm} exp {exp}: {row['states']} states, fp64 "
              f"{row['fp64']['solve_ms']:.1f} ms ({row['fp64']['sweeps_fp64']} sweeps), fp32 "
              f"{row['fp32']['solve_ms']:.1f} ms", file=sys.stderr, flush=True)
        out.append(row)
        del m
    line = {"metric": METRIC, "value": max(r["fp64"]["backups_per_s"] for r in out),
            "unit": "backups/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
            "dtype": "f64",
            "config": {"workload": "paper scenario-C experiments (m 3 and 5), periodic stop"},
            "detail": out}
    print(json.dumps(line), flush=True)


def bench_paper_b(args, pvi, W):
    """The paper's scenario-B experiments (lead time 1, gamma = 1, V0 = expected revenue,
    span stop; P1-P4: exactly 100 sweeps): one solve each after one untimed solve."""
    out = []
    for (mm, exp) in W.PAPER_B_EXPERIMENTS:
        sc = W.scenario_b_paper(mm, exp)
        t0 = time.perf_counter()
        m = pvi.mdp_create(sc)
        row = {"m": mm, "exp": exp, "states": m.n_states, "actions": m.n_actions,
               "create_ms": (time.perf_counter() - t0) * 1e3}
        fixed = 100 if exp.startswith("P") else 0
        for prec in ("fp64", "fp32"):
            kw = {"fixed_sweeps": fixed} if fixed else {}
            pvi.vi_solve(m, precision=prec, **kw)
            t0 = time.perf_counter()
            r = pvi.vi_solve(m, precision=prec, time_kernels=True, **kw)
            dt = time.perf_counter() - t0
            row[prec] = {"solve_ms": dt * 1e3, "sweeps_fp32": r["sweeps_fp32"],
                         "sweeps_fp64": r["sweeps_fp64"],
                         "backups_per_s": r["logical_backups"] / dt,
                         "backup_ms": list(r["backup_ms"]),
                         "backup_launches": list(r["backup_launches"])}
        row["fp64_checkpointed"] = checkpointed_solve(args, pvi, m, 1,
                                                      **({"fixed_sweeps": fixed} if fixed
                                                         else {}))
        print(f"B m={mm} exp {exp}: {row['states']} states, fp64 "
              f"{row['fp64']['solve_ms']:.1f} ms ({row['fp64']['sweeps_fp64']} sweeps), fp32 "
              f"{row['fp32']['solve_ms']:.1f} ms", file=sys.stderr, flush=True)
        out.append(row)
        del m
    line = {"metric": METRIC, "value": max(r["fp64"]["backups_per_s"] for r in out),
            "unit": "backups/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
            "dtype": "f64",
            "config": {"workload": "paper scenario-B experiments (lead time 1, gamma 1)"},
            "detail": out}
    print(json.dumps(line), flush=True)


def bench_rollouts(args, pvi, W):
    """Policy evaluation and simulation optimization on the GPU (Simulation section):
    10,000 rollouts of 100 + 365 days of the solved policy of the paper's largest
    scenario-A and scenario-C runs, and heuristic grids over the same rollouts."""
    import numpy as np
    import torch
    runs = []
    cases = [
        ("A m=5 L=2 FIFO C_w=7 (1,771,561 states)", W.scenario_a_paper(5, 2, 7.0, "fifo"),
         "supnorm", "base_stock", [[S] for S in range(11)]),
        ("C m=5 exp 1 (1,361,367 states)", W.scenario_c_paper(5, 1), "periodic", "s_S",
         [[lo, hi] * 7 for lo in range(0, 21, 2) for hi in range(lo + 1, 21, 2)]),
        ("B two products (config 2 shape, 50,625 states)", W.config2(), "span",
         "mod_base_stock", [[a, b] for a in range(0, 29) for b in range(0, 29)]),
        # m = 8: 12,607,619,787 states, no value iteration; the paper's (s, S) fit first
        ("C m=8 exp 1 (12,607,619,787 states, heuristics only)", W.scenario_c_paper(8, 1),
         None, "s_S", [[8, 19, 8, 15, 8, 18, 7, 18, 8, 14, 3, 13, 4, 16]] +
         [[lo, hi] * 7 for lo in range(0, 21, 2) for hi in range(lo + 1, 21, 2)]),
    ]
    for label, sc, rule, kind, grid in cases:
        m = pvi.mdp_create(sc)
        if rule is not None:
            pvi.vi_solve(m, precision="fp64", eps=sc["eps"], stop_rule=rule)
        row = {"workload": label}
        todo = ([("vi_policy", {})] if rule is not None else []) + \
            [(kind + "_grid", {"policy": kind, "params": grid})]
        for what, kw in todo:
            pvi.policy_rollouts(m, n_rollouts=1000, per_rollout=False, **kw)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = pvi.policy_rollouts(m, n_rollouts=10000, per_rollout=False, **kw)
            dt = time.perf_counter() - t0
            npol = r["stats"].shape[0]
            best = int(np.argmax(r["stats"][:, 0]))
            row[what] = {"policies": npol, "ms": dt * 1e3,
                         "rollout_days_per_s": npol * 10000 * 465 / dt,
                         "best_policy": best, "best_mean_return": float(r["stats"][best, 0]),
                         "best_return_sd": float(r["stats"][best, 1])}
            print(f"{label} {what}: {npol} x 10000 rollouts in {dt * 1e3:.1f} ms",
                  file=sys.stderr, flush=True)
        runs.append(row)
        del m
    line = {"metric": "rollout days per second (10,000 rollouts of 465 days per policy)",
            "value": max(r[k]["rollout_days_per_s"] for r in runs for k in r if k != "workload"),
            "unit": "rollout-days/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
            "data": "synthetic", "config": {"workload": "policy rollouts and heuristic grids"},
            "detail": runs}
    print(json.dumps(line), flush=True)


TRAFFIC_PROFILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                               "backup_a_kernel_m4L2_hbm_traffic.md")
KERNEL_SOURCE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2303_10672_amd",
                             "csrc", "kernels_a.hip")


def measured_traffic():
    """HBM bytes per full FP64 sweep of the scenario-A backup, from the committed
    counter summary, or None when the kernel source has changed since it was taken
    (the summary records the source's SHA-256)."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_PROFILE).read()
        src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    sha = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    fetch = re.search(r"hbm_fetch_bytes_per_launch:\s*([0-9.eE+]+)", text)
    write = re.search(r"hbm_write_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not (sha and fetch and write) or sha.group(1) != src:
        return None
    return float(fetch.group(1)), float(write.group(1))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    if args.workload == "oracle":
        return bench_oracle(args)
    import torch
    from paper_2303_10672_amd import pvi
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration_mb > 0:
        n = args.copy_calibration_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "batch":
        return bench_batch(args, pvi, W)
    if args.workload == "serving":
        return bench_serving(args, pvi, W)
    if args.workload in ("config2", "config3"):
        return bench_single(args, pvi, W, int(args.workload[-1]))
    if args.workload == "paper-a":
        return bench_paper_a(args, pvi, W)
    if args.workload == "paper-c":
        return bench_paper_c(args, pvi, W)
    if args.workload == "paper-b":
        return bench_paper_b(args, pvi, W)
    if args.workload == "rollouts":
        return bench_rollouts(args, pvi, W)
    sc = W.config1()
    stream = torch.cuda.Stream()
    handle = stream.cuda_stream
    # cold calls, reported apart from the timed steps: the first solve of the process
    # (code objects loaded, device buffers allocated, tables uploaded, graphs captured)
    # and the first solve of a second handle in the warm process
    cold = {}
    for key in ("process_first_call_ms", "new_handle_first_call_ms"):
        mc = pvi.mdp_create(sc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pvi.vi_solve(mc, precision=args.precision, stream=handle)
        torch.cuda.synchronize()
        cold[key] = (time.perf_counter() - t0) * 1e3
        del mc
    m = pvi.mdp_create(sc)

    main_run = time_solves(pvi, m, args.precision, args.steps, args.warmup, handle)
    fp64_steps = args.fp64_steps if args.fp64_steps is not None else max(1, args.steps // 2)
    others = [p for p in ("fp64", "fp32", "fp32_wide") if p != args.precision]
    runs = {args.precision: main_run}
    for p in others:
        runs[p] = time_solves(pvi, m, p, fp64_steps, 1, handle)
    fp64_run = runs["fp64"]
    cold["warm_p50_ms"] = percentile(main_run["lat_ms"], 0.5)

    value = main_run["logical"] / main_run["wall_s"]
    ms_per_step = main_run["wall_s"] * 1e3 / args.steps
    # the dominant backup kernel: FP32-storage sweeps unless the mode is plain FP64
    dom = 0 if args.precision == "fp64" else 1
    launches = max(main_run["launches"][dom], 1)
    avg_kernel_s = main_run["backup_ms"][dom] / launches * 1e-3
    # algorithmic bytes of one sweep: read V once and write V' once (FP64: 16 B per
    # state, FP32 storage: 8 B); the gathers of V[s'] re-read that same table
    state_bytes = 16 if dom == 0 else 8
    achieved_gbs = m.n_states * state_bytes / avg_kernel_s / 1e9
    per_launch_logical = m.n_states * m.n_actions * (sc["d_max"][0] + 1)
    logical_gbs = per_launch_logical * (8 if dom == 0 else 4) / avg_kernel_s / 1e9
    sweeps = main_run["sweeps_fp32"] + main_run["sweeps_fp64"] + 1
    executed_per_launch = main_run["executed"] / (args.steps * sweeps)
    fma_tflops = 2.0 * executed_per_launch / avg_kernel_s / 1e12

    # counters were taken on the FP64 kernel: only that kernel's line carries them
    meas = measured_traffic() if dom == 0 else None
    traffic = (meas[0] + meas[1]) if meas else None
    traffic_detail = None
    if meas:
        # the measured bytes over the same average launch time: the HBM rate the kernel
        # really draws, against the same peak
        measured_gbs = traffic / avg_kernel_s / 1e9
        traffic_detail = {"unit": "bytes per launch", "fetch": meas[0], "write": meas[1],
                          "source": os.path.relpath(TRAFFIC_PROFILE,
                                                    os.path.dirname(os.path.abspath(__file__))),
                          "algorithmic": float(state_bytes * m.n_states),
                          "measured_over_algorithmic": traffic / (state_bytes * m.n_states),
                          "measured_gbs": measured_gbs,
                          "measured_frac": measured_gbs / HBM_PEAK_GBS}

    def schedule(p):
        r = runs[p]
        return {
            "value": r["logical"] / r["wall_s"],
            "ms_per_solve": percentile(r["lat_ms"], 0.5),
            "latency_ms": {"p50": percentile(r["lat_ms"], 0.5),
                           "p99": percentile(r["lat_ms"], 0.99)},
            "sweeps": {"fp32": r["sweeps_fp32"], "fp64": r["sweeps_fp64"], "extract": 1},
            "avg_backup_kernel_ms": {
                "fp32_storage": r["backup_ms"][1] / max(r["launches"][1], 1),
                "fp64": r["backup_ms"][0] / max(r["launches"][0], 1)},
        }
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
        "fp64_plain": schedule("fp64"),
        "fp32_compensated": schedule("fp32"),
        "fp32_fp64_sums": schedule("fp32_wide"),
        "cold_calls": cold,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_detail": traffic_detail,
            "kernel": "backup_a_kernel<" + ("double" if dom == 0 else "float") + ">",
            "launches_timed": launches,
            "avg_kernel_ms": avg_kernel_s * 1e3,
            "basis": f"{state_bytes} B per state per sweep (read V, write V') x "
                     f"{m.n_states} states per launch",
        },
        "roofline_logical_gathers": {
            "achieved": logical_gbs, "unit": "GB/s", "frac_of_hbm_peak": logical_gbs / HBM_PEAK_GBS,
            "basis": f"{8 if dom == 0 else 4} B of V per logical backup x {per_launch_logical} "
                     "logical backups per launch (above 1: the gathers are served from "
                     "LDS, L2 and the Infinity Cache, not HBM)",
        },
        "roofline_executed": {
            "bound": "alu",
            "achieved": fma_tflops,
            "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": fma_tflops / FP64_VECTOR_PEAK_TFLOPS,
            "basis": f"2 flops per executed multiply-add, {executed_per_launch:.4g} per launch",
        },
        "fp32_error_vs_fp64": None if args.no_errors else fp32_errors(pvi, W),
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline(sc, args.cpu_seconds),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

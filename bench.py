#!/usr/bin/env python
"""Benchmark of the SN-like DLR step on one MI355X.

Workload: the 1024 x 1024 log-normal random medium (sigma_a = exp(1.5 g), 16-cell
Gaussian correlation, seed 3), left-edge inflow at T_b = 1, 32 x 64 product
ordinates (2048 directions), rank 32, dt = 0.002; FP32 sweeps and projections
with FP64 selection, QR/SVD, L-step and temperature update (SI tolerance 1e-6).
One "step" is one DLR time step (Algorithm 1) with all inputs resident in HBM.

Prints one JSON line: cell-angle sweep updates per second of the whole timed run
(value), DLR steps/s, the sweep kernel against the HBM roofline (HIP-event
timed inside the library on its own stream) and the FP64 CPU oracle timed on a
bounded sample of the same workload on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "cell-angle sweep updates/s + DLR steps/s at 1024², r=32; p50/p99 solve latency"


def source_hash(name):
    with open(os.path.join(ROOT, "paper_2601_18705_amd", "csrc", name), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(record, source="k_sweep.hip"):
    """HBM bytes per launch from a committed rocprofv3 counter record (profiles/<record>.json),
    when it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", record + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("sweep_source_sha") != source_hash(source):
        return None
    return rec.get("hbm_bytes_per_launch")


def make_problem(name):
    from synth import problems
    if name == "random_medium":
        p = problems.random_medium()
    elif name == "checkerboard":
        p = problems.checkerboard()
    elif name == "slab_beam":
        p = problems.slab_beam()
    else:
        raise SystemExit(f"unknown workload {name}")
    return p


def host_info():
    """Host CPU model and logical core count (the oracle's baseline is timed on these)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def cpu_baseline(p, steps, threads=1):
    """The FP64 oracle on the host: `steps` DLR steps from the cold start (initial factors
    not timed).  threads = 1 pins BLAS to one thread; threads = None lets it use every core
    the process may run on (the oracle's C sweep itself is single-threaded)."""
    from threadpoolctl import threadpool_limits

    from oracle import dlr_oracle as O
    cores = threads if threads is not None else (len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                                                 else os.cpu_count())
    with threadpool_limits(limits=threads):
        quad = O.quadrature(p["n_polar"], p["n_azim"])
        st = O.dlr_initial_state(p, quad)
        ca = 0
        t0 = time.perf_counter()
        for _ in range(steps):
            st, s = O.dlr_step(p, quad, st)
            ca += s["si_iters"] * p["nx"] * p["ny"] * p["rank"]
        dt = time.perf_counter() - t0
    return {"value": ca / dt, "unit": "cell-angle updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} DLR step(s) of the same workload from its cold start, FP64, "
                      f"{'1 thread' if threads == 1 else f'BLAS on {cores} threads, C sweep on one'} "
                      f"({dt:.1f} s, {ca} cell-angle updates)",
            "steps_per_s": steps / dt}


def serving_leg(window_s, max_s, budget_gib, max_requests=10000):
    """Continuous batching over the seeded Poisson request stream (200 requests/s) for a fixed
    window of arrivals; the loop stops at max_s wall seconds.  FP32 sweeps.  Reports what
    arrived, completed and is left (admitted or queued), p50/p99 time-to-solution of the
    completed requests, and aggregate cell-angle updates/s."""
    from paper_2601_18705_amd import dlrtrt, serve
    from synth import problems
    specs = problems.request_specs(count=max_requests, window_s=window_s)

    def fp32(build):
        def make():
            prob = build()
            prob["precision"], prob["si_tol"] = dlrtrt.DLR_FP32_SWEEP, 1e-6
            return prob
        return make
    reqs = [(t, fp32(build), ns) for t, build, ns, _ in specs]

    def progress(passes, done, inflight, queued):
        if passes % 50 == 0:
            print(f"[bench] serving pass {passes}: done {done} in flight {inflight} queued {queued}",
                  file=sys.stderr, flush=True)

    res = serve.serve(reqs, hbm_budget=int(budget_gib * (1 << 30)), max_wall_s=max_s, progress=progress)
    return {"requests_in_window": len(reqs), "arrival_window_s": window_s, "arrived": res["arrived"],
            "completed": res["completed"], "failed": len(res["failed"]),
            "unfinished_admitted": res["unfinished_admitted"], "unfinished_queued": res["unfinished_queued"],
            "sustained_completions_per_s": res["completed"] / res["wall_s"],
            "p50_s": res["p50_s"], "p99_s": res["p99_s"], "ca_per_s": res["ca_per_s"], "wall_s": res["wall_s"],
            "hbm_budget_gib": budget_gib,
            "stream": "seeded Poisson 200 req/s; 64^2-1024^2 grids, ranks 8-32, 20-200 steps, 512 ordinates, "
                      "checkerboard or log-normal medium; latency counts from arrival (problem built on admission)"}


def sn_leg(workload, precision, si_tol, steps, dlr_steps_per_s):
    """Plain discrete ordinates on the same problem: every ordinate swept each source iteration."""
    import torch
    from paper_2601_18705_amd import dlrtrt
    p = make_problem(workload)
    p["precision"], p["si_tol"] = precision, si_tol
    nq, N = p["n_polar"] * p["n_azim"], p["nx"] * p["ny"]
    with dlrtrt.Instance(p, method="sn") as inst:
        inst.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ca, sweep_ms, launches = 0, 0.0, 0
        for _ in range(steps):
            inst.step(1)
            st = inst.read_stats()
            ca += st["si_iters"] * N * nq
            sweep_ms += st["sweep_ms"]
            launches += st["si_iters"]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    sb = 4 if precision != dlrtrt.DLR_FP64 else 8
    # src0 read and psi write per ordinate; sigma_t and s_e once per orientation copy (4)
    bytes_per_launch = N * nq * 2 * sb + 4 * N * 2 * sb
    avg = sweep_ms / 1e3 / max(launches, 1)
    return {"ordinates": nq, "steps": steps, "sn_steps_per_s": steps / wall,
            "cell_angle_updates_per_s": ca / wall, "si_iterations_per_step": launches / steps,
            "sweep_avg_launch_ms": avg * 1e3, "sweep_algorithmic_bytes_per_launch": bytes_per_launch,
            "sweep_achieved_GBs": bytes_per_launch / avg / 1e9,
            "dlr_speedup_steps_per_s": dlr_steps_per_s / (steps / wall)}


def augmented_leg(workload, precision, si_tol, steps, plain_step_wall):
    """The augmented-basis variant on the same problem and precision: the Galerkin space of the step
    holds the swept columns and the old basis (2r columns) and the SVD truncates back to rank r.
    Steps 3..steps+2 are timed (after two untimed ones), beside the plain step's same steps."""
    import torch
    from paper_2601_18705_amd import dlrtrt
    p = make_problem(workload)
    p["precision"], p["si_tol"] = precision, si_tol
    N, r = p["nx"] * p["ny"], p["rank"]
    with dlrtrt.Instance(p, method="augmented") as inst:
        inst.step(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ca, dev_ms, si = 0, 0.0, []
        for _ in range(steps):
            inst.step(1)
            st = inst.read_stats()
            ca += st["si_iters"] * N * r
            dev_ms += st["step_ms"]
            si.append(int(st["si_iters"]))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    same = plain_step_wall[2:2 + steps]
    plain = len(same) / sum(same) if len(same) == steps else None
    return {"galerkin_rank": 2 * r, "steps": f"3..{2 + steps}", "steps_per_s": steps / wall,
            "cell_angle_updates_per_s": ca / wall, "device_ms_per_step": dev_ms / steps,
            "si_iterations_per_step": sum(si) / steps,
            "plain_steps_per_s_same_steps": plain,
            "cost_vs_plain": (plain / (steps / wall)) if plain else None}


def q1_leg(n, nd, reps):
    """The bilinear (Q1) DG sweep operator on its own: n x n cells, nd directions, sigma_t of
    the random medium plus 1/(c dt), FP32 and FP64, inputs resident in HBM."""
    import numpy as np
    import torch
    from paper_2601_18705_amd import dlrtrt
    from synth import problems
    out = {"grid": f"{n}x{n}", "directions": nd,
           "bytes_model": "per cell-direction: 4 source + 4 psi values; sigma_t once per cell"}
    for name, prec, npdt in (("fp32", dlrtrt.DLR_FP32_SWEEP, np.float32), ("fp64", dlrtrt.DLR_FP64, np.float64)):
        inp = problems.q1_sweep_inputs(n, n, nd, seed=3, sigma_shift=500.0, dtype=npdt)
        dev = torch.device("cuda:0")
        t = {k: torch.from_numpy(inp[k]).to(dev) for k in ("sigma_t", "src", "inflow_x", "inflow_y")}
        psi = torch.empty_like(t["src"])
        with dlrtrt.Q1Sweep(n, n, inp["hx"], inp["hy"], inp["mu"], inp["eta"], prec) as op:
            op.time(t["sigma_t"], t["src"], t["inflow_x"], t["inflow_y"], psi, 2)
            ms = op.time(t["sigma_t"], t["src"], t["inflow_x"], t["inflow_y"], psi, reps)
        sb = np.dtype(npdt).itemsize
        byts = nd * n * n * 8 * sb + n * n * sb
        out[name] = {"ms_per_sweep": ms, "cell_direction_updates_per_s": nd * n * n / (ms * 1e-3),
                     "algorithmic_bytes": byts, "achieved_GBs": byts / (ms * 1e-3) / 1e9,
                     "frac_hbm_peak": byts / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
                     "traffic": load_traffic(f"q1_counters_{n}x{n}_nd{nd}_{name}", "k_q1.hip")}
        del t, psi
    # the FP64 oracle on a bounded sample (one direction on 48 x 48 cells)
    from oracle import q1_oracle
    smp = problems.q1_sweep_inputs(48, 48, 1, seed=3, sigma_shift=500.0)
    t0 = time.perf_counter()
    q1_oracle.sweep(48, 48, smp["hx"], smp["hy"], smp["mu"], smp["eta"], smp["sigma_t"], smp["src"],
                    smp["inflow_x"], smp["inflow_y"])
    out["cpu_oracle"] = {"cell_direction_updates_per_s": 48 * 48 / (time.perf_counter() - t0), "cores": 1,
                         "sample": "one direction on 48 x 48 cells (pure-Python cell loop, numpy 4x4 solves)"}
    return out


def dsa_leg(n, steps):
    """Diffusion synthetic acceleration on an optically thick, hot checkerboard (sigma = 10^4 in
    alternating unit blocks, T = 1, 512 ordinates, r = 16, FP64 sweeps, SI tolerance 1e-10): source
    iterations and time per step without and with the acceleration (the same fixed point)."""
    import numpy as np
    import torch
    from paper_2601_18705_amd import dlrtrt
    from synth import problems
    p = problems.checkerboard(n=n, nsteps=steps)
    p["sigma_a"] = problems.checkerboard_sigma(p, thick=1e4, thin=1.0)
    p["T_init"] = np.full(n * n, 1.0)
    p["si_tol"], p["si_max_iter"] = 1e-10, 100000
    out = {"workload": f"checkerboard {n}^2, sigma 1e4 / 1, T = 1, q16x32, r16, FP64, SI tol 1e-10"}
    fields = {}
    for name, dsa in (("plain", 0), ("dsa", 1)):
        with dlrtrt.Instance(dict(p, dsa=dsa)) as inst:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            si = []
            for _ in range(steps):
                inst.step(1)
                si.append(int(inst.read_stats()["si_iters"]))
            wall = time.perf_counter() - t0
            fields[name] = inst.read_fields()[1]
        out[name] = {"si_iterations_per_step": si, "ms_per_step": wall * 1e3 / steps}
    out["T_rel_diff"] = float(np.max(np.abs(fields["dsa"] - fields["plain"])) / np.max(np.abs(fields["plain"])))
    return out


def batch_run(count, steps, graphs=True):
    """The batched-instances workload: count independent problems admitted at once and
    advanced together for `steps` steps (FP32 sweeps, FP64 energy update); with graphs, the
    steps after the first run from the recorded graphs of the composition."""
    from paper_2601_18705_amd import dlrtrt
    from synth import problems
    insts = problems.batch_instances(count=count, nsteps=steps)
    import torch
    torch.cuda.init()
    with dlrtrt.Batch() as b:
        b.set_graphs(1 if graphs else 0)
        slots = {}
        for prob in insts:
            prob["precision"], prob["si_tol"] = dlrtrt.DLR_FP32_SWEEP, 1e-6
            slots[b.admit(prob, steps)] = prob
        ca = 0
        t0 = time.perf_counter()
        for k in range(steps):
            b.advance()
            for slot, prob in slots.items():
                st = b.read_stats(slot)
                ca += int(st["si_iters"]) * int(prob["nx"]) * int(prob["ny"]) * int(prob["rank"])
            if k % 10 == 9:
                print(f"[bench] batch step {k + 1}/{steps}", file=sys.stderr, flush=True)
        wall = time.perf_counter() - t0
        done = b.poll()
        recorded = b.graph_steps()
    return {"instances": count, "steps": steps, "wall_s": wall, "ca_per_s": ca / wall,
            "instance_steps_per_s": count * steps / wall, "finished": len(done), "graph_steps": recorded}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200,
                    help="timed DLR steps from the cold start (200 = the whole configured trajectory)")
    ap.add_argument("--warmup", type=int, default=5, help="untimed steps on a separate instance first")
    ap.add_argument("--workload", default="random_medium")
    ap.add_argument("--cpu-steps", type=int, default=4, help="oracle steps timed for the CPU baseline (0 = skip; 4 take about 10 s)")
    ap.add_argument("--fp64", action="store_true", help="plain FP64 path (sweeps in FP64, SI tol 1e-14)")
    ap.add_argument("--fp64-steps", type=int, default=10,
                    help="steps of the FP64-sweep comparison leg at the same SI tolerance (0 = skip)")
    ap.add_argument("--aug-steps", type=int, default=20,
                    help="steps of the augmented-basis variant on the same workload (0 = skip)")
    ap.add_argument("--sn-steps", type=int, default=3,
                    help="steps of the plain SN comparison leg over every ordinate (0 = skip)")
    ap.add_argument("--q1-reps", type=int, default=20,
                    help="timed launches of the bilinear DG sweep leg, 1024^2 cells x 32 directions (0 = skip)")
    ap.add_argument("--dsa-n", type=int, default=128,
                    help="grid of the DSA leg (thick hot checkerboard, two steps without and with DSA; 0 = skip)")
    ap.add_argument("--batch-count", type=int, default=256,
                    help="instances of the batched leg (0 = skip): 64^2-256^2 grids, ranks 4-24, 50 steps each")
    ap.add_argument("--serve-window-s", type=float, default=30.0,
                    help="arrival window of the serving leg in seconds (0 = skip)")
    ap.add_argument("--serve-max-s", type=float, default=45.0, help="wall-time cap of the serving leg")
    ap.add_argument("--serve-budget-gib", type=float, default=16.0, help="HBM budget of the serving batch")
    ap.add_argument("--batch", type=int, default=0, metavar="COUNT",
                    help="run only the batched-instances workload (COUNT problems, 50 steps)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="after the timed run, run a plain elementwise kernel over a buffer of this size (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU; --gpus must be 1 "
                                   "(the step is not sharded across GPUs)"}))
        sys.exit(2)

    import torch
    from paper_2601_18705_amd import dlrtrt

    if args.batch:
        res = batch_run(args.batch, 50)
        print(json.dumps({"metric": "batched cell-angle updates/s (independent instances, one sweep launch per "
                                    "source iteration)", "value": res["ca_per_s"], "unit": "cell-angle updates/s",
                          "n_gpus": 1, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": f"batch_{args.batch}_instances_64-256sq_r4-24_512ord_50steps"},
                          **res}), flush=True)
        return

    def problem():
        p = make_problem(args.workload)
        if args.fp64:
            p["precision"], p["si_tol"] = dlrtrt.DLR_FP64, 1e-14
        else:
            p["precision"], p["si_tol"] = dlrtrt.DLR_FP32_SWEEP, 1e-6
        return p

    p = problem()
    N, r = p["nx"] * p["ny"], p["rank"]
    print(f"[bench] workload {p['name']} precision {'fp64' if args.fp64 else 'fp32-sweep'} "
          f"warmup {args.warmup} steps {args.steps}", file=sys.stderr, flush=True)
    torch.cuda.init()
    if args.warmup > 0:
        with dlrtrt.Instance(p) as warm:
            warm.step(args.warmup)
    torch.cuda.synchronize()
    inst = dlrtrt.Instance(p)
    torch.cuda.synchronize()
    ca = 0
    sweep_ms = 0.0
    si_ms = 0.0
    launches = 0
    step_ms = 0.0
    svd_sweeps = 0
    si_hist = []
    step_wall = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        inst.step(1)
        st = inst.read_stats()
        step_wall.append(time.perf_counter() - ts)
        ca += st["si_iters"] * N * r
        sweep_ms += st["sweep_ms"]
        si_ms += st["si_ms"]
        launches += st["si_iters"]
        step_ms += st["step_ms"]
        svd_sweeps += st["svd_sweeps"]
        si_hist.append(int(st["si_iters"]))
        if k % 50 == 49:
            print(f"[bench] step {k + 1}/{args.steps} si {st['si_iters']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    E, T = inst.read_fields()
    shape = inst.sweep_shape()   # chosen by the library's tuner on the warm-up instance
    inst.close()

    sweep_bytes = 4 if not args.fp64 else 8
    bytes_per_launch = N * r * 2 * sweep_bytes + N * 2 * sweep_bytes   # src0 read, psi write; sigma_t, s_e read
    avg_launch_s = sweep_ms / 1e3 / max(launches, 1)
    achieved = bytes_per_launch / avg_launch_s / 1e9
    # the whole source-iteration phase (Algorithm 1 step 4): the sweep plus the scalar-flux passes, which
    # read Psi and write phi and the four orientation copies of s_e (reading phi_old and sigma_s)
    flux_bytes = N * r * sweep_bytes + 3 * N * 8 + 4 * N * sweep_bytes
    avg_iter_s = si_ms / 1e3 / max(launches, 1)
    a4_achieved = (bytes_per_launch + flux_bytes) / avg_iter_s / 1e9 if avg_iter_s > 0 else None
    traffic = load_traffic("sweep_counters_" + p["name"] + ("_fp64" if args.fp64 else "_fp32"))

    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 2.0, out=b)   # one elementwise kernel: reads and writes n * 4 bytes
        torch.cuda.synchronize()

    last = step_wall[-20:]
    out = {
        "metric": METRIC,
        "value": ca / wall,
        "unit": "cell-angle updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.fp64 else "f32",
        "data": "synthetic (seeded log-normal random medium; no dataset)",
        "config": {"workload": p["name"], "nx": p["nx"], "ny": p["ny"], "directions": p["n_polar"] * p["n_azim"],
                   "rank": r, "dt": p["dt"], "si_tol": p["si_tol"], "timed_steps": "1..%d from the cold start" % args.steps,
                   "precision": "fp64" if args.fp64 else "fp32 sweeps+projections, fp64 selection/QR/SVD/L-step/T"},
        "dlr_steps_per_s": args.steps / wall,
        "dlr_steps_per_s_last20": len(last) / sum(last),
        "sweep_cell_angle_updates_per_s": ca / (sweep_ms / 1e3),
        "si_iterations_per_step": launches / args.steps,
        "si_iterations_per_step_last20": sum(si_hist[-20:]) / len(si_hist[-20:]),
        "si_iterations_histogram": {str(k): si_hist.count(k) for k in sorted(set(si_hist))},
        "device_ms_per_step": step_ms / args.steps,
        "svd_sweeps_per_step": svd_sweeps / args.steps,
        "latency_p50_p99_s": None,
        "serving": None,
        "roofline": {"kernel": "k_sweep", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": bytes_per_launch, "avg_launch_ms": avg_launch_s * 1e3,
                     "launch_shape": {"prefetch_chunks": shape[0], "grid_blocks": shape[1], "chosen_by": "tuner"}},
        "a4_phase": {"what": "sweep + scalar-flux passes per source iteration", "avg_iteration_ms": avg_iter_s * 1e3,
                     "algorithmic_bytes": bytes_per_launch + flux_bytes, "achieved": a4_achieved,
                     "unit": "GB/s", "frac": (a4_achieved / HBM_PEAK_GBS) if a4_achieved else None},
        "checksum": {"E_r_sum": float(E.sum()), "T_sum": float(T.sum())},
        "host": host_info(),
    }
    if args.fp64_steps > 0 and not args.fp64:
        print("[bench] FP64-sweep leg", file=sys.stderr, flush=True)
        p64 = make_problem(args.workload)
        p64["precision"], p64["si_tol"] = dlrtrt.DLR_FP64, p["si_tol"]
        with dlrtrt.Instance(p64) as i64:
            i64.step(2)
            torch.cuda.synchronize()
            t64 = time.perf_counter()
            i64.step(args.fp64_steps)
            torch.cuda.synchronize()
            w64 = time.perf_counter() - t64
        f32_early = args.fp64_steps / sum(step_wall[2:2 + args.fp64_steps]) if len(step_wall) >= 2 + args.fp64_steps else None
        out["fp64_sweep_leg"] = {"dlr_steps_per_s": args.fp64_steps / w64, "steps": f"3..{2 + args.fp64_steps}",
                                 "si_tol": p64["si_tol"],
                                 "fp32_steps_per_s_same_steps": f32_early,
                                 "fp32_speedup": (f32_early / (args.fp64_steps / w64)) if f32_early else None}
    if args.aug_steps > 0:
        print("[bench] augmented-basis leg", file=sys.stderr, flush=True)
        out["augmented_leg"] = augmented_leg(args.workload, p["precision"], p["si_tol"], args.aug_steps, step_wall)
    if args.sn_steps > 0:
        print("[bench] plain SN leg", file=sys.stderr, flush=True)
        out["plain_sn_leg"] = sn_leg(args.workload, p["precision"], p["si_tol"], args.sn_steps,
                                     args.steps / wall)
    if args.q1_reps > 0:
        print("[bench] bilinear DG sweep leg", file=sys.stderr, flush=True)
        out["q1_sweep_leg"] = q1_leg(1024, 32, args.q1_reps)
    if args.dsa_n > 0:
        print("[bench] DSA leg", file=sys.stderr, flush=True)
        out["dsa_leg"] = dsa_leg(args.dsa_n, 2)
    if args.batch_count > 0:
        print(f"[bench] batched leg: {args.batch_count} instances", file=sys.stderr, flush=True)
        out["batch_leg"] = batch_run(args.batch_count, 50)
        eager = batch_run(args.batch_count, 50, graphs=False)
        out["batch_leg"]["eager_steps"] = {k: eager[k] for k in ("wall_s", "ca_per_s", "instance_steps_per_s")}
    if args.serve_window_s > 0:
        print(f"[bench] serving leg: {args.serve_window_s:g} s of arrivals", file=sys.stderr, flush=True)
        sv = serving_leg(args.serve_window_s, args.serve_max_s, args.serve_budget_gib)
        out["serving"] = sv
        out["latency_p50_p99_s"] = [sv["p50_s"], sv["p99_s"]]
    if args.cpu_steps > 0:
        print("[bench] timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(make_problem(args.workload), args.cpu_steps, threads=1)
        out["cpu_baseline_all_cores"] = cpu_baseline(make_problem(args.workload), args.cpu_steps, threads=None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark of the time-dependent HJ level-set solve on one MI355X.

A "step" of this benchmark is one whole solve of the workload (grid tables,
alpha^max reduction, float64 CFL schedule, every Runge-Kutta stage of every
time step, tube clamp), with V0 already resident in HBM.  The headline value
is float32 grid-point updates per second (points x CFL steps / wall time);
the float64 form of the same solve is timed beside it.

Default workload: the 4D dynamic car, 80^4 nodes on [-5,5]^2 x [0,4] x
[-pi,pi), |a| <= 1, |w| <= 1, disc target r = 0.5, TVD-RK3, CFL 0.8,
horizon 3 s, tube (BRT).  Other workloads (--workload): dubins3d (60x60x36,
float64 form), game6d (36^6, RK2), pe3d (the 3D relative pursuit-evasion
game, 100^3, horizon 1.5, first order, costate box per stage), ttr3d (time
to reach by Lax-Friedrichs sweeping, Dubins 100^3), batch (512 Dubins
solves), serve.
--space-order 2 runs a single-solve workload with second-order ENO
differences and, unless --rk says otherwise, TVD-RK2 (the paper's
second-order pairing).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point updates/s FP32 vs FP64 + % HBM roofline; p50/p99 solve latency"
HBM_PEAK_GBPS = 8000.0


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or
    None when there is none or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    from paper_2204_05520_amd.profiling import kernel_source_hash
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def time_solves(odp, spec, V0, precision, steps, warmup, stream, tile_chunk=0, xcd_group=0,
                space_order=1):
    import torch
    grid = odp.Grid.from_spec(spec.grid)
    opts = odp.make_opts(precision, spec.rk_order, spec.cfl, spec.mode, 0, 0.0, 0, tile_chunk,
                         odp._stream_handle(stream), xcd_group, space_order=space_order)
    wsb = odp.odp_hj_workspace_bytes(grid, spec.dyn, spec.tau, opts)
    ws = torch.empty(wsb, dtype=torch.uint8, device=V0.device)
    out = torch.empty_like(V0)
    stats = None
    # the autotuner's one-time timing runs in an untimed call
    for _ in range(max(warmup, 1 if tile_chunk == odp.ODP_TILE_AUTOTUNE else 0)):
        stats = odp.odp_hj_solve(grid, spec.dyn, V0, None, spec.tau, opts, ws, out)
    torch.cuda.synchronize()
    kernel_ms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        st = odp.odp_hj_solve(grid, spec.dyn, V0, None, spec.tau, opts, ws, out)
        kernel_ms.append(st.kernel_ms)
        stats = st
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, stats, kernel_ms, out


def cpu_baseline(spec, V0_np, budget_steps=2, space_order=1):
    """The oracle as it stands on the host cores, on a bounded sample: the
    first `budget_steps` CFL steps of the same workload."""
    import oracle
    oracle.build(force=False)
    amax, dt = oracle.cfl_dt(spec.grid, spec.dyn, spec.cfl)
    tau = [0.0, budget_steps * dt * (1 - 1e-12)]
    t0 = time.perf_counter()
    res = oracle.solve(spec.grid, spec.dyn, V0_np, tau, rk_order=spec.rk_order, cfl=spec.cfl,
                       brt=spec.mode == 1, space_order=space_order)
    wall = time.perf_counter() - t0
    pts = spec.grid.npts * res.steps
    return {"value": pts / wall, "unit": "grid-point updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"first {res.steps} CFL steps (float64, RK{spec.rk_order}"
                      f"{', ENO2' if space_order == 2 else ''}) of the same "
                      f"{'x'.join(map(str, spec.grid.n))} solve, {wall:.1f} s"}


def bench_single(args, W, odp):
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    if args.workload == "dyncar4d":
        spec = W.config_dyncar4d(n=args.n or 80)
        kname, precs = "stage_dyncar4d", ((32,) if args.fp32_only else (32, 64))
    elif args.workload == "game6d":
        spec = W.config_game6d(n=args.n or 36)
        kname, precs = "stage_game6d", (32,)
    elif args.workload == "pe3d":
        spec = W.config_pe3d(n=args.n or 100)
        kname, precs = "stage_pe3d", (32, 64)
    else:
        spec = W.config_dubins3d()
        kname, precs = "stage_dubins3d", (64, 32)
    if args.rk:
        spec.rk_order = args.rk
    if args.space_order == 2:
        spec.rk_order = args.rk or 2
        spec.name = spec.name.replace("_rk", "_eno2_rk").rsplit("_rk", 1)[0] + f"_rk{spec.rk_order}_brt"
        kname = kname.replace("stage_", "stage_eno2_")
    elif args.rk:
        spec.name = spec.name.rsplit("_rk", 1)[0] + f"_rk{spec.rk_order}_brt"
    stream = torch.cuda.Stream()
    results = {}
    V0_np = None
    for prec in precs:
        dt = torch.float32 if prec == 32 else torch.float64
        if spec.grid.npts > 50_000_000:
            V0 = W.make_v0_torch(spec, dev, dt)
        else:
            V0_np = W.make_v0(spec)
            V0 = torch.tensor(V0_np, dtype=dt, device=dev)
        with torch.cuda.stream(stream):
            wall, st, kms, out = time_solves(odp, spec, V0, prec, args.steps, args.warmup, stream,
                                             args.tile_chunk, space_order=args.space_order)
        P = spec.grid.npts
        nsteps = st.steps
        nlaunch = nsteps * spec.rk_order
        avg_launch_s = (sum(kms) / len(kms)) / 1e3 / nlaunch
        bytes_per_launch = st.alg_bytes / nlaunch
        results[prec] = {
            "pt_updates_per_s": P * nsteps * args.steps / wall,
            "ms_per_solve": wall / args.steps * 1e3,
            "kernel_ms": sum(kms) / len(kms),
            "steps": nsteps,
            "avg_launch_us": avg_launch_s * 1e6,
            "alg_bytes_per_launch": bytes_per_launch,
            "achieved_gbps": bytes_per_launch / avg_launch_s / 1e9,
        }
        print(f"# fp{prec}: {results[prec]}", file=sys.stderr, flush=True)
        del V0, out
        torch.cuda.empty_cache()
    head = 32 if 32 in results else precs[0]
    r = results[head]
    traffic = measured_traffic(f"{kname}_fp{head}", spec.name)
    roof = {"bound": "hbm", "achieved": r["achieved_gbps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": r["achieved_gbps"] / HBM_PEAK_GBPS, "traffic": traffic,
            "kernel": (f"{'stage_point_kernel' if args.space_order == 2 or args.workload == 'pe3d' else 'stage_kernel'}"
                       f" fp{head}" + (" (costate-box pass + update per stage)" if args.workload == "pe3d" else "")),
            "avg_launch_us": r["avg_launch_us"],
            "alg_bytes_per_launch": r["alg_bytes_per_launch"]}
    line = {
        "metric": METRIC, "value": r["pt_updates_per_s"], "unit": "grid-point updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_solve"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if head == 32 else "f64", "data": "synthetic",
        "config": {"workload": spec.name, "grid": spec.grid.n, "rk_order": spec.rk_order,
                   "tiles": "autotuned" if args.tile_chunk == -1 else args.tile_chunk,
                   "cfl": spec.cfl, "horizon": spec.tau[-1], "mode": "BRT",
                   "space_order": args.space_order,
                   "cfl_steps_per_solve": r["steps"]},
        "roofline": roof,
    }
    if 64 in results and 32 in results:
        line["fp64_value"] = results[64]["pt_updates_per_s"]
        line["fp64_ms_per_step"] = results[64]["ms_per_solve"]
        line["fp64_roofline_frac"] = results[64]["achieved_gbps"] / HBM_PEAK_GBPS
        line["fp32_over_fp64"] = results[32]["pt_updates_per_s"] / results[64]["pt_updates_per_s"]
    if not args.no_cpu:
        import numpy as np
        if V0_np is None:
            V0_np = W.make_v0(spec) if spec.grid.npts <= 200_000_000 else None
        if V0_np is not None:
            line["cpu_baseline"] = cpu_baseline(spec, V0_np, space_order=args.space_order)
    return line


def bench_ttr(args, W, odp):
    """Time to reach by Lax-Friedrichs sweeping (Jacobi form) for the Dubins
    car (v = 1, |w| <= 1, the turn minimising the time), 100^3 on
    [-4,4]^2 x [-pi,pi), disc target of radius 1, eps 1e-5 (the paper's TTR
    example), float32 and float64; one step = one solve to convergence."""
    import numpy as np
    import torch
    n = args.n or 100
    g = W.GridSpec([n, n, n], [-4.0, -4.0, -W.PI], [4.0, 4.0, W.PI], [0, 0, 1])
    d = W.DynSpec(W.DYN_DUBINS3D, [1.0, 1.0], W.MINIMISE, W.MAXIMISE)
    l = W.cylinder_v0(g, 1.0)
    st = torch.cuda.Stream()
    res = {}
    for prec in (32, 64):
        dt = torch.float32 if prec == 32 else torch.float64
        tg = torch.tensor(l, dtype=dt, device="cuda:0")
        with torch.cuda.stream(st):
            for _ in range(max(args.warmup, 1)):
                _, s_ = odp.ttr_solve(g, d, tg, precision=prec, eps=1e-5, stream=st)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                _, s_ = odp.ttr_solve(g, d, tg, precision=prec, eps=1e-5, stream=st)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / args.steps
        res[prec] = {"ms_per_solve": wall * 1e3, "iters": s_["iters"], "kernel_ms": s_["kernel_ms"],
                     "pt_updates_per_s": g.npts * s_["iters"] / wall,
                     "achieved_gbps": s_["alg_bytes"] / (s_["kernel_ms"] * 1e6),
                     "us_per_iter": s_["kernel_ms"] * 1e3 / s_["iters"]}
        print(f"# ttr fp{prec}: {res[prec]}", file=sys.stderr, flush=True)
    r = res[32]
    line = {
        "metric": METRIC, "value": r["pt_updates_per_s"], "unit": "grid-point updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_solve"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"ttr_dubins3d_{n}x{n}x{n}", "eps": 1e-5, "iterations": r["iters"]},
        "roofline": {"bound": "hbm", "achieved": r["achieved_gbps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": r["achieved_gbps"] / HBM_PEAK_GBPS, "traffic": None,
                     "kernel": "ttr_kernel fp32 (one Jacobi sweep per launch)",
                     "avg_launch_us": r["us_per_iter"]},
        "fp64_value": res[64]["pt_updates_per_s"], "fp64_ms_per_step": res[64]["ms_per_solve"],
        "fp64_iterations": res[64]["iters"],
    }
    if not args.no_cpu:
        import oracle
        oracle.build(force=False)
        gs = W.GridSpec([40, 40, 40], [-4.0, -4.0, -W.PI], [4.0, 4.0, W.PI], [0, 0, 1])
        t0 = time.perf_counter()
        o = oracle.ttr_solve(gs, d, W.cylinder_v0(gs, 1.0), eps=1e-5)
        wall = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": gs.npts * o.iters / wall, "unit": "grid-point updates/s", "cores": 1,
                                "kind": "oracle",
                                "sample": f"Gauss-Seidel sweeps of the same problem at 40^3 to eps 1e-5: "
                                          f"{o.iters} sweeps, {wall:.1f} s (the sweep is serial)"}
    return line


def bench_batch(args, W, odp):
    """512 Dubins solves of uneven grids in one odp_hj_batch call (float32),
    beside the same solves run one by one in float64 through odp_hj_solve."""
    import torch
    dev = torch.device("cuda:0")
    specs = W.batch_dubins3d()
    stream = torch.cuda.Stream()
    V32 = [torch.tensor(W.make_v0(s), dtype=torch.float32, device=dev) for s in specs]
    outs = [torch.empty_like(v) for v in V32]
    plan = odp.BatchPlan(specs, V32, outs, precision=32, tile_chunk=args.tile_chunk)
    ws = torch.empty(plan.workspace_bytes(), dtype=torch.uint8, device=dev)
    with torch.cuda.stream(stream):
        for _ in range(max(args.warmup, 1 if args.tile_chunk == odp.ODP_TILE_AUTOTUNE else 0)):
            stats = plan.run(stream, ws)
        torch.cuda.synchronize()
        # the call is stream-ordered (no statistics requested): one call's
        # host work overlaps the previous call's kernels
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(args.steps):
            plan.run(stream, ws, want_stats=False)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        stats = plan.run(stream, ws)  # (untimed) step counts and algorithmic bytes
        torch.cuda.synchronize()
    pts = sum(s.grid.npts * st["steps"] for s, st in zip(specs, stats))
    alg = sum(st["alg_bytes"] for st in stats)
    kernel_s = e0.elapsed_time(e1) / 1e3 / args.steps
    # float64, one odp_hj_solve per member
    V64 = [torch.tensor(W.make_v0(s), dtype=torch.float64, device=dev) for s in specs]
    with torch.cuda.stream(stream):
        for s, v in zip(specs[:8], V64[:8]):
            odp.solve(s, v, precision=64, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s, v in zip(specs, V64):
            odp.solve(s, v, precision=64, stream=stream)
        torch.cuda.synchronize()
        wall64 = time.perf_counter() - t0
    line = {
        "metric": METRIC, "value": pts / wall, "unit": "grid-point updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batch512_dubins3d_rk1_brt", "solves": len(specs),
                   "tiles": "autotuned" if args.tile_chunk == -1 else args.tile_chunk,
                   "points": sum(s.grid.npts for s in specs), "point_steps": pts},
        "roofline": {"bound": "hbm", "achieved": alg / kernel_s / 1e9, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": alg / kernel_s / 1e9 / HBM_PEAK_GBPS, "traffic": None,
                     "kernel": "stage_kernel fp32 (batched launches)"},
        "fp64_per_solve_value": pts / wall64, "fp64_per_solve_ms": wall64 * 1e3,
        "batch_over_per_solve": wall64 / wall,
        # algorithmic bytes over the calls' wall time and over their device
        # time (events on the stream around the timed calls: prologue kernels
        # and uploads included)
        "wall_roofline_frac": alg / wall / 1e9 / HBM_PEAK_GBPS,
        "kernel_roofline_frac": alg / kernel_s / 1e9 / HBM_PEAK_GBPS,
        "host_overhead_ms": wall * 1e3 - kernel_s * 1e3,
    }
    return line


def bench_serve(args, W, odp):
    """Poisson arrivals (200/s) of mixed 3D Dubins / 4D car requests into the
    continuous-batching server; latency = the server's submit -> completion
    clock; p50/p99 over the requests after the warm-up ones."""
    import threading
    import numpy as np
    warm = 200
    nreq = args.serve_requests
    reqs = W.serve_requests(count=warm + nreq)
    print(f"# serve: preparing {len(reqs)} host V0 arrays", file=sys.stderr, flush=True)
    V0s = [W.make_v0(r.spec).astype(np.float32) for r in reqs]
    outs = [np.empty_like(v) for v in V0s]
    srv = odp.Server(budget_bytes=96 << 30, max_slots=512, precision=32, rk_order=1)
    tickets = [None] * len(reqs)
    lat = [None] * len(reqs)
    sub_t = [None] * len(reqs)
    done_t = [None] * len(reqs)
    steps = [0] * len(reqs)
    pts = [0] * len(reqs)
    algb = [0.0] * len(reqs)
    lock = threading.Lock()
    t0 = time.perf_counter()

    def submitter(k, nthreads):
        for i in range(k, len(reqs), nthreads):
            delay = reqs[i].arrival_s - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            t = srv.submit(reqs[i].spec, V0s[i], rk_order=reqs[i].spec.rk_order)
            with lock:
                tickets[i] = t
                sub_t[i] = time.perf_counter() - t0

    threads = [threading.Thread(target=submitter, args=(k, 4)) for k in range(4)]
    for th in threads:
        th.start()
    remaining = set(range(len(reqs)))
    while remaining:
        progressed = False
        time.sleep(0.002)
        if srv.counts()[2] == 0:
            continue
        for i in list(remaining):
            with lock:
                t = tickets[i]
            if t is None:
                continue
            rc, st = srv.poll(t, outs[i])
            if rc == 0:
                done_t[i] = time.perf_counter() - t0
                lat[i] = st["latency_ms"]
                steps[i] = st["steps"]
                pts[i] = reqs[i].spec.grid.npts * st["steps"]
                algb[i] = st["alg_bytes"]
                remaining.discard(i)
                progressed = True
    wall = time.perf_counter() - t0
    for th in threads:
        th.join()
    srv.close()
    meas = np.array(lat[warm:])
    # client clock: from the request's scheduled (Poisson) arrival to the poll
    # that saw it done (includes any lag of the submitting threads)
    client = np.array([(done_t[i] - reqs[i].arrival_s) * 1e3 for i in range(warm, len(reqs))])
    lag = np.array([(sub_t[i] - reqs[i].arrival_s) * 1e3 for i in range(warm, len(reqs))])
    t_first = reqs[warm].arrival_s
    span = wall - t_first
    line = {
        "metric": METRIC, "value": float(sum(pts[warm:]) / span), "unit": "grid-point updates/s",
        "n_gpus": 1, "steps": nreq, "warmup": warm, "ms_per_step": float(np.mean(client)),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "serve_poisson200_mixed_dubins3d_dyncar4d", "requests": nreq,
                   "rate_per_s": 200.0},
        "latency_ms": {"p50": float(np.percentile(client, 50)), "p90": float(np.percentile(client, 90)),
                       "p99": float(np.percentile(client, 99)), "max": float(client.max()),
                       "clock": "client: scheduled arrival to observed completion"},
        "server_latency_ms": {"p50": float(np.percentile(meas, 50)), "p90": float(np.percentile(meas, 90)),
                              "p99": float(np.percentile(meas, 99)), "max": float(meas.max()),
                              "clock": "server: submit to completion"},
        "submit_lag_ms": {"p50": float(np.percentile(lag, 50)), "p99": float(np.percentile(lag, 99))},
        "completed_per_s": nreq / span,
        # the measured requests' own arrival rate (first to last arrival)
        "offered_per_s": nreq / (reqs[-1].arrival_s - t_first),
        # time from the last arrival to the last completion: the run ends with
        # this drain, which completed_per_s includes; a backlog would make it
        # grow past the latency tail
        "drain_after_last_arrival_ms": (wall - reqs[-1].arrival_s) * 1e3,
        "alg_tbps_over_run": sum(algb[warm:]) / span / 1e12,
        "offered_alg_tbps": sum(algb[warm:]) / (reqs[-1].arrival_s - t_first) / 1e12,
    }
    return line


def _max_abs_diff(a, b, chunk=1 << 26):
    """max |a - b| in float64 over two device arrays, in chunks."""
    a, b = a.reshape(-1), b.reshape(-1)
    m = 0.0
    for i in range(0, a.numel(), chunk):
        m = max(m, float((a[i:i + chunk].double() - b[i:i + chunk].double()).abs().max()))
    return m


def leg_small3d(args, W, odp):
    """The 60x60x36 Dubins solve (float64 plain form and float32): a 1 MB
    grid that stays in the caches, so it is launch-bound; reported per CFL
    step."""
    a = argparse.Namespace(**vars(args))
    a.workload, a.n, a.steps, a.warmup, a.no_cpu, a.space_order, a.rk = "dubins3d", 0, 20, 2, True, 1, 0
    ln = bench_single(a, W, odp)
    steps = ln["config"]["cfl_steps_per_solve"]
    out = {"grid": ln["config"]["grid"], "cfl_steps_per_solve": steps,
           "fp64_ms_per_solve": ln["fp64_ms_per_step"] if "fp64_ms_per_step" in ln else ln["ms_per_step"],
           "fp32_ms_per_solve": ln["ms_per_step"] if ln["dtype"] == "f32" else None,
           "fp32_pt_updates_per_s": ln["value"], "fp64_pt_updates_per_s": ln.get("fp64_value")}
    out["fp64_us_per_step"] = out["fp64_ms_per_solve"] * 1e3 / steps
    out["fp32_us_per_step"] = ln["ms_per_step"] * 1e3 / steps
    out["bound"] = "launch latency (HIP graph of the whole stepping, cached per shape)"
    return out


def leg_game6d(args, W, odp):
    """The 36^6 game (2.18e9 points, RK2, T = 2, 73 steps): float32 timed and
    held, then the float64 plain form; the roofline fraction of the float32
    stage launches, the float32 speed-up and the float32 max-norm error
    against the float64 solve over the whole horizon."""
    import torch
    dev = torch.device("cuda:0")
    spec = W.config_game6d()
    stream = torch.cuda.Stream()
    res = {}
    outs = {}
    for prec, dt, steps in ((32, torch.float32, 2), (64, torch.float64, 1)):
        V0 = W.make_v0_torch(spec, dev, dt)
        with torch.cuda.stream(stream):
            wall, st, kms, out = time_solves(odp, spec, V0, prec, steps, 1, stream, -1)
        nl = st.steps * spec.rk_order
        avg = (sum(kms) / len(kms)) / 1e3 / nl
        res[prec] = {"ms_per_solve": wall / steps * 1e3, "pt_updates_per_s": spec.grid.npts * st.steps * steps / wall,
                     "steps": st.steps, "avg_launch_us": avg * 1e6,
                     "frac": st.alg_bytes / nl / avg / 1e9 / HBM_PEAK_GBPS}
        print(f"# game6d fp{prec}: {res[prec]}", file=sys.stderr, flush=True)
        outs[prec] = out
        del V0
        torch.cuda.empty_cache()
    err = _max_abs_diff(outs[32], outs[64])
    del outs
    torch.cuda.empty_cache()
    S = spec.grid.domain_scale()
    return {"grid": spec.grid.n, "cfl_steps_per_solve": res[32]["steps"],
            "fp32_pt_updates_per_s": res[32]["pt_updates_per_s"], "fp32_ms_per_solve": res[32]["ms_per_solve"],
            "fp32_roofline_frac": res[32]["frac"], "fp32_avg_stage_launch_us": res[32]["avg_launch_us"],
            "fp64_pt_updates_per_s": res[64]["pt_updates_per_s"], "fp64_ms_per_solve": res[64]["ms_per_solve"],
            "fp64_roofline_frac": res[64]["frac"],
            "fp32_over_fp64": res[32]["pt_updates_per_s"] / res[64]["pt_updates_per_s"],
            "fp32_vs_fp64_max_abs_err": err, "fp32_vs_fp64_err_over_S": err / S}


def leg_batch(args, W, odp):
    a = argparse.Namespace(**vars(args))
    a.steps, a.warmup = 5, 1
    ln = bench_batch(a, W, odp)
    keep = ("value", "ms_per_step", "fp64_per_solve_ms", "batch_over_per_solve")
    out = {k: ln[k] for k in keep}
    out["pt_updates_per_s"] = out.pop("value")
    out["wall_ms_per_batch"] = out.pop("ms_per_step")
    out.update({k: ln[k] for k in ("wall_roofline_frac", "kernel_roofline_frac", "host_overhead_ms") if k in ln})
    return out


def leg_serve(args, W, odp):
    ln = bench_serve(args, W, odp)
    keep = ("latency_ms", "server_latency_ms", "completed_per_s", "offered_per_s", "drain_after_last_arrival_ms",
            "alg_tbps_over_run",
            "offered_alg_tbps",
            "phases_ms")
    out = {k: ln[k] for k in keep if k in ln}
    out["requests"] = ln["config"]["requests"]
    out["rate_per_s"] = ln["config"]["rate_per_s"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="dyncar4d",
                    choices=["dyncar4d", "dubins3d", "game6d", "pe3d", "ttr3d", "batch", "serve"])
    ap.add_argument("--n", type=int, default=0)
    ap.add_argument("--tile-chunk", type=int, default=-1,
                    help="planes per block; -1 (default): the library's autotuner, which times "
                         "candidate tilings once per shape (in the untimed warm-up)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--calib-copy", action="store_true",
                    help="first issue one plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--fp32-only", action="store_true")
    ap.add_argument("--space-order", type=int, default=1, choices=[1, 2],
                    help="2: second-order ENO differences (single-solve workloads)")
    ap.add_argument("--rk", type=int, default=0, choices=[0, 1, 2, 3],
                    help="Runge-Kutta order override (0: the workload's; 2 with --space-order 2)")
    ap.add_argument("--only", action="store_true",
                    help="the default 4D workload alone (without the other four configurations' keys)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; multi-GPU sharding is a design "
                                   "note only (slab halo exchange over xGMI), so --gpus must be 1"}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    import paper_2204_05520_amd as odp
    from paper_2204_05520_amd import workloads as W
    odp.lib()
    if args.calib_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.workload in ("dyncar4d", "game6d", "dubins3d", "pe3d"):
        line = bench_single(args, W, odp)
        if args.workload == "dyncar4d" and not args.only and args.space_order == 1 and not args.n:
            # the other four configurations, measured in the same run
            legs = {}
            for name, fn in (("dubins3d_60x60x36_rk1_brt", leg_small3d), ("game6d_36^6_rk2_brt", leg_game6d),
                             ("batch512_dubins3d_rk1_brt", leg_batch),
                             ("serve_poisson200_mixed_dubins3d_dyncar4d", leg_serve)):
                print(f"# leg {name}", file=sys.stderr, flush=True)
                t0 = time.perf_counter()
                legs[name] = fn(args, W, odp)
                legs[name]["leg_wall_s"] = time.perf_counter() - t0
                torch.cuda.empty_cache()
            line["configs"] = legs
    elif args.workload == "batch":
        line = bench_batch(args, W, odp)
    elif args.workload == "ttr3d":
        line = bench_ttr(args, W, odp)
    else:
        line = bench_serve(args, W, odp)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark workloads beyond the single periodic grid (used by bench.py).

cavities: many lid-driven cavities of uneven size (side log-uniform on
          [32, 512], lid speed U[0.01, 0.1], seed 4), FP16 shifted storage with
          FP32 arithmetic, each run until its residual max |u_t - u_{t-100}| is
          <= 1e-8 (FP64 reduction, every 100 steps) or its step cap.  Timed as one
          batch (fused launches, graph bursts) and as the plain form (one grid at a
          time with the library's default kernel for that grid and graph bursts,
          the same residual checks).  A sample of the final fields is compared bit
          for bit between the two and against an FP64 run of the same number of
          steps.
serve:    a Poisson stream of cavity and porous-channel requests (sizes 32..2048,
          step budgets 1e3..1e5, seed 5) served by the continuous-batching server
          and by the plain FIFO; p50 / p99 latency and aggregate MLUPS.
"""
import time

import numpy as np

from . import inputs as I

METRIC = "MLUPS + % HBM roofline (LBMTau1 D2Q9); batched p50/p99 vs plain per-grid"


def _cavity_grid(L, u, prec):
    from .grid import Grid
    flags, rho, jx, jy, per = I.cavity(L, u)
    g = Grid(L, L, prec=prec, periodic=per)
    g.set_geometry(flags, rho, jx, jy)
    g.fluid = int((flags == I.FLUID).sum())
    return g, (flags, rho, jx, jy)


def run_cavities(n, cap, tol, torch, log, burst=100, seed=4, tune=True, shape=None, plain=True):
    """The uneven-cavity population (n cavities, seed 4) run batched and one grid at a
    time, each grid to residual <= tol (tol < 0: never) or cap steps.  The batch's tile
    shape is the autotuner's (tune; its time is not counted), or `shape`
    (fuse, rows, lds, vec_cap), else the heuristic.  Returns the record: MLUPS of both forms, stop
    reasons, the alone-vs-mix identity on a sample of final fields, and the FP16
    storage error against FP64 runs of the same steps."""
    from . import _capi as C
    from .batch import Batch
    from .serve import GpuBackend
    pop = I.cavity_population(n=n, seed=seed)
    lups_total = 0.0

    # ---- batched: all cavities resident, one fused launch per step
    log(f"[cavities] batched: {len(pop)} cavities, cap {cap} steps")
    grids = [_cavity_grid(L, u, "f16s") for L, u in pop]
    b = Batch(sum(g.nbytes for g, _ in grids) + (1 << 20), len(grids))
    slots = [b.admit(g, cap, tol) for g, _ in grids]
    tuned = None
    if shape is not None:
        b.set_shape(*shape)
    elif tune:
        t0 = time.perf_counter()
        sh, ms = b.autotune(burst_steps=20, reps=2)
        tuned = dict(shape=sh, ms_per_20_steps=round(ms, 4), seconds=round(time.perf_counter() - t0, 2))
        log(f"[cavities] autotuned tile shape {sh}: {ms:.3f} ms per 20 steps ({tuned['seconds']} s)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bursts = 0
    while len(b.poll()) < len(grids):
        b.run(burst)
        bursts += 1
        if bursts % 200 == 0:
            log(f"[cavities] batched: {bursts} bursts, {len(b.poll())} done")
    t_batch = time.perf_counter() - t0
    shape_used = b.shape()
    info = [b.slot_info(s) for s in slots]
    steps = [st for _, st, _ in info]
    reasons = {C.SLOT_BUDGET: "cap", C.SLOT_CONVERGED: "converged", C.SLOT_NONFINITE: "nonfinite"}
    why = [reasons[s] for s, _, _ in info]
    for (g, _), s in zip(grids, steps):
        lups_total += g.fluid * s
    sample = list(range(0, len(grids), max(1, len(grids) // 8)))
    batched_fields = {}
    for k, s in enumerate(slots):
        b.evict(s)
        if k in sample:
            batched_fields[k] = grids[k][0].read_moments()
    for g, _ in grids:
        g.close()
    b.close()
    mlups_batch = lups_total / t_batch / 1e6
    log(f"[cavities] batched: {t_batch:.2f} s, {mlups_batch:.0f} MLUPS")

    # ---- plain: one grid at a time with its own default kernel and graph bursts,
    # the same residual checks every `burst` steps
    log("[cavities] plain" if plain else "[cavities] plain form skipped")
    be = GpuBackend(1 << 30, 1, prec="f16s")
    t0 = time.perf_counter()
    same = True
    for k, (L, u) in enumerate(pop if plain else []):
        g, _ = _cavity_grid(L, u, "f16s")
        state, nst, _ = be.run_alone(g, cap, tol, burst)
        same &= nst == steps[k]
        if k in batched_fields:
            same &= all(np.array_equal(a, c) for a, c in zip(g.read_moments(), batched_fields[k]))
        g.close()
        if k % 64 == 63:
            log(f"[cavities] plain: {k + 1} grids, {time.perf_counter() - t0:.1f} s")
    t_plain = time.perf_counter() - t0 if plain else float("nan")
    be.close()
    mlups_plain = lups_total / t_plain / 1e6
    log(f"[cavities] plain: {t_plain:.2f} s, {mlups_plain:.0f} MLUPS, identical {same}")

    # ---- error of the FP16 storage against FP64 runs of the same steps (sample)
    errs = []
    for k in sample[:4] if plain else []:
        L, u = pop[k]
        g, (flags, *_r) = _cavity_grid(L, u, "f64")
        g.step(steps[k])
        ref = g.read_moments()
        g.close()
        fl = flags == I.FLUID
        jscale = max(np.abs(ref[1][fl]).max(), np.abs(ref[2][fl]).max())
        ej = max(np.abs(batched_fields[k][1] - ref[1])[fl].max(), np.abs(batched_fields[k][2] - ref[2])[fl].max())
        errs.append(dict(L=L, steps=steps[k], max_abs_j=float(ej), rel_to_max_j=float(ej / jscale)))
    return dict(cavities=len(pop), cap=cap, tol=tol, fluid_lups=lups_total, steps=int(sum(steps)),
                tile_shape=shape_used, autotune=tuned,
                batched=dict(seconds=round(t_batch, 3), mlups=round(mlups_batch, 1)),
                plain=dict(seconds=round(t_plain, 3), mlups=round(mlups_plain, 1)),
                speedup=round(t_plain / t_batch, 2), stop_reasons={r: why.count(r) for r in set(why)},
                alone_vs_mix_identical=bool(same), error_vs_f64_sample=errs)


def bench_cavities(args, torch, log):
    cap, tol = args.max_steps, 1e-8
    shape = None
    if getattr(args, "batch_shape", None):
        f, *rest = [int(v) for v in args.batch_shape.split(":")]
        rows, extra = rest[:5], rest[5:]
        shape = (f, rows, extra[0] if extra else 0, extra[1] if len(extra) > 1 else 0)
    r = run_cavities(args.cavities, cap, tol, torch, log, tune=not args.no_tune, shape=shape,
                     plain=not getattr(args, "batched_only", False))
    return {
        "metric": METRIC,
        "value": r["batched"]["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": r["steps"],
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{r['cavities']} lid-driven cavities, side log-uniform [32, 512], lid U[0.01, 0.1], "
                               f"seed 4, FP16 shifted storage, to residual <= 1e-8 or {cap} steps",
                   "cavities": r["cavities"], "fluid_lups": r["fluid_lups"]},
        "batched": r["batched"],
        "plain": r["plain"],
        "speedup": r["speedup"],
        "tile_shape": r["tile_shape"],
        "autotune": r["autotune"],
        "stop_reasons": r["stop_reasons"],
        "alone_vs_mix_identical": r["alone_vs_mix_identical"],
        "error_vs_f64_sample": r["error_vs_f64_sample"],
    }


def run_serve(n_requests, load, budget, torch, log, slots=64):
    """The request stream (seed 5) at `load` times the server's capacity measured on a
    burst of 24 requests: the continuous-batching server and the plain FIFO on the same
    requests.  Returns (capacity req/s, rate, requests, server summary, plain summary)."""
    from .serve import GpuBackend, PlainFifo, Server, requests_from_stream, summarize

    def progress(tag):
        def f(n, now):
            if n % 10 == 0:
                log(f"[serve] {tag}: {n} done at {now:.1f} s")
        return f
    # capacity: how fast the server drains a burst of requests that all arrive at once
    probe = requests_from_stream(I.request_stream(n=24, seed=55, rate=1e9))
    for r in probe:
        r.arrival = 0.0
    be = GpuBackend(budget, slots, prec="f16s")
    t0 = time.perf_counter()
    Server(be, budget, slots, progress=progress("capacity probe")).serve(probe)
    cap = len(probe) / (time.perf_counter() - t0)
    be.close()
    rate = load * cap
    log(f"[serve] capacity {cap:.2f} req/s; offered load {load} -> {rate:.2f} req/s")
    reqs = requests_from_stream(I.request_stream(n=n_requests, seed=5, rate=rate))
    be = GpuBackend(budget, slots, prec="f16s")
    t0 = time.perf_counter()
    served = Server(be, budget, slots, progress=progress("server")).serve(reqs)
    wall_s = time.perf_counter() - t0
    be.close()
    s_srv = summarize(served, wall_s)
    log(f"[serve] server: p50 {s_srv['p50_s']:.3f} s p99 {s_srv['p99_s']:.3f} s {s_srv['mlups']:.0f} MLUPS")
    be = GpuBackend(budget, 1, prec="f16s")
    t0 = time.perf_counter()
    plain = PlainFifo(be, progress=progress("plain"), budget=budget).serve(reqs)
    wall_p = time.perf_counter() - t0
    be.close()
    s_pl = summarize(plain, wall_p)
    log(f"[serve] plain: p50 {s_pl['p50_s']:.3f} s p99 {s_pl['p99_s']:.3f} s {s_pl['mlups']:.0f} MLUPS")
    return cap, rate, reqs, served, s_srv, s_pl


def bench_serve(args, torch, log):
    budget = int(getattr(args, "budget_mib", 1024)) << 20
    cap, rate, reqs, served, s_srv, s_pl = run_serve(args.requests, args.load, budget, torch, log)
    return {
        "metric": METRIC,
        "value": round(s_srv["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": int(sum(r.steps for r in served)),
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{len(reqs)} Poisson requests at {rate:.3f}/s (load {args.load} of the "
                               f"measured capacity {cap:.3f}/s), half cavities half porous channels, "
                               f"side 32..2048, budgets 1e3..1e5 steps, FP16 storage, {budget >> 20} MiB HBM "
                               "budget, 64 slots",
                   "requests": len(reqs), "rate_per_s": rate, "load": args.load, "budget_mib": budget >> 20},
        "server": s_srv,
        "plain": s_pl,
    }

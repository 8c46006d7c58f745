"""Benchmark workloads beyond the single periodic grid (used by bench.py).

cavities: many lid-driven cavities of uneven size (side log-uniform on
          [32, 512], lid speed U[0.01, 0.1], seed 4), FP16 shifted storage with
          FP32 arithmetic, each run until its residual max |u_t - u_{t-100}| is
          <= 1e-8 (FP64 reduction, every 100 steps) or its step cap.  Timed as one
          batch (fused launches, graph bursts) and as the plain form (one grid at a
          time, one launch per step, same residual checks).  A sample of the
          final fields is compared bit for bit between the two and against an
          FP64 run of the same number of steps.
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


def bench_cavities(args, torch, log):
    from . import _capi as C
    from .batch import Batch
    from .serve import GpuBackend
    pop = I.cavity_population(n=args.cavities, seed=4)
    cap, tol, burst = args.max_steps, 1e-8, 100
    lups_total = 0.0

    # ---- batched: all cavities resident, one fused launch per step
    log(f"[cavities] batched: {len(pop)} cavities, cap {cap} steps")
    grids = [_cavity_grid(L, u, "f16s") for L, u in pop]
    b = Batch(sum(g.nbytes for g, _ in grids) + (1 << 20), len(grids))
    slots = [b.admit(g, cap, tol) for g, _ in grids]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bursts = 0
    while len(b.poll()) < len(grids):
        b.run(burst)
        bursts += 1
        if bursts % 200 == 0:
            log(f"[cavities] batched: {bursts} bursts, {len(b.poll())} done")
    t_batch = time.perf_counter() - t0
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

    # ---- plain: one grid at a time, one launch per step
    log("[cavities] plain")
    be = GpuBackend(1 << 30, 1, prec="f16s")
    t0 = time.perf_counter()
    same = True
    for k, (L, u) in enumerate(pop):
        g, _ = _cavity_grid(L, u, "f16s")
        state, n, _ = be.run_alone(g, cap, tol, burst)
        same &= n == steps[k]
        if k in batched_fields:
            same &= all(np.array_equal(a, c) for a, c in zip(g.read_moments(), batched_fields[k]))
        g.close()
        if k % 32 == 31:
            log(f"[cavities] plain: {k + 1} grids, {time.perf_counter() - t0:.1f} s")
    t_plain = time.perf_counter() - t0
    be.close()
    mlups_plain = lups_total / t_plain / 1e6
    log(f"[cavities] plain: {t_plain:.2f} s, {mlups_plain:.0f} MLUPS, identical {same}")

    # ---- error of the FP16 storage against FP64 runs of the same steps (sample)
    errs = []
    for k in sample[:4]:
        L, u = pop[k]
        g, (flags, *_r) = _cavity_grid(L, u, "f64")
        g.step(steps[k])
        ref = g.read_moments()
        g.close()
        fl = flags == I.FLUID
        jscale = max(np.abs(ref[1][fl]).max(), np.abs(ref[2][fl]).max())
        ej = max(np.abs(batched_fields[k][1] - ref[1])[fl].max(), np.abs(batched_fields[k][2] - ref[2])[fl].max())
        errs.append(dict(L=L, steps=steps[k], max_abs_j=float(ej), rel_to_max_j=float(ej / jscale)))
    return {
        "metric": METRIC,
        "value": round(mlups_batch, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": int(sum(steps)),
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{len(pop)} lid-driven cavities, side log-uniform [32, 512], lid U[0.01, 0.1], "
                               f"seed 4, FP16 shifted storage, to residual <= 1e-8 or {cap} steps",
                   "cavities": len(pop), "fluid_lups": lups_total},
        "batched": {"seconds": round(t_batch, 3), "mlups": round(mlups_batch, 1)},
        "plain": {"seconds": round(t_plain, 3), "mlups": round(mlups_plain, 1)},
        "speedup": round(t_plain / t_batch, 2),
        "stop_reasons": {r: why.count(r) for r in set(why)},
        "alone_vs_mix_identical": bool(same),
        "error_vs_f64_sample": errs,
    }


def bench_serve(args, torch, log):
    from .serve import GpuBackend, PlainFifo, Server, requests_from_stream, summarize
    budget = int(getattr(args, "budget_mib", 1024)) << 20
    slots = 64

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
    rate = args.load * cap
    log(f"[serve] capacity {cap:.2f} req/s; offered load {args.load} -> {rate:.2f} req/s")
    reqs = requests_from_stream(I.request_stream(n=args.requests, seed=5, rate=rate))
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

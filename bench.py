#!/usr/bin/env python3
"""Benchmark of the LBMTau1 D2Q9 step on one MI355X.

Default workload: the 8192 x 8192 fully periodic random field (rho = 1 +
1e-3 N(0,1), u = 0.01 N(0,1), seed 0), FP32 moment storage, the roofline run.
A "step" is one LBMTau1 time step of the whole grid (gather of the nine
upwind neighbours' moments, equilibria, sums, store), with the FP64
mass / residual / non-finite reduction every 100 steps and the steps issued as
HIP-graph bursts.  Inputs are resident in HBM before the timed region.

The JSON line carries:
  value        fluid lattice updates per second (MLUPS), whole job
  roofline     the step kernel's algorithmic HBM bytes per launch (read and write
               3 moment planes once: 2 * 3 * c bytes per fluid node, for one step,
               or for two when the kernel fuses two steps per pass) over its
               average launch duration from HIP events on the grid's stream,
               against 8 TB/s
  cpu_baseline the FP64 CPU oracle on a bounded sample of the same workload
  variants     the same run with FP64, FP16 and BF16 shifted storage, each with its
               error against the FP64 run

Other workloads: --workload cavity (the 256^2 lid-driven cavity, 50,000 steps in
FP64 and FP32, cache-resident), --workload cavities (batched uneven cavities vs one grid per
launch), --workload serve (continuous-batching server vs FIFO), --workload
compare (LBMTau1 against the stored-population BGK method on the same field:
the paper's memory comparison measured, and the speed ratio), --workload
stability (largest stable Reynolds number of the lid-driven cavity against
grid size at tau = 1, 0.55, 0.7 and 1.5, with the power-law fits), --workload
drop (the paper's multiphase performance test: a liquid drop in periodic
vapour, L = 128..8192, multiphase LBMTau1 against the stored-population
multiphase method), --workload 3d (3-D LBMTau1 on D3Q19 / D3Q27 periodic
random fields of 256^3 and 512^3); each prints its own line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "MLUPS + % HBM roofline (LBMTau1 D2Q9); batched p50/p99 vs plain per-grid"
VALUE_BYTES = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1000)
    p.add_argument("--warmup", type=int, default=100)
    p.add_argument("--workload", default="periodic",
                   choices=["periodic", "cavity", "cavities", "serve", "compare", "stability", "drop", "3d"])
    p.add_argument("--n", type=int, default=8192, help="grid side of the periodic workload")
    p.add_argument("--storage", default="f32", choices=["f64", "f32", "f16s", "bf16s"])
    p.add_argument("--no-variants", action="store_true", help="skip the other storage variants")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-tune", action="store_true", help="skip the autotuner")
    p.add_argument("--kernel", default=None, help="fix the kernel: gather or strip:vec:rows:waves[:fuse]")
    p.add_argument("--planar", action="store_true", help="three separate moment planes instead of "
                   "the row-interleaved layout")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--n3", default="256,512", help="3d: grid sides (comma-separated)")
    p.add_argument("--q3", default="19,27", help="3d: lattices (comma-separated)")
    p.add_argument("--steps3", type=int, default=0, help="3d: timed steps (0: 200 at 256^3, 50 above)")
    p.add_argument("--cavity-steps", type=int, default=50000, help="cavity: steps of the lid-driven cavity")
    p.add_argument("--cavity-n", type=int, default=256, help="cavity: side of the lid-driven cavity")
    p.add_argument("--cavities", type=int, default=512)
    p.add_argument("--max-steps", type=int, default=200000)
    p.add_argument("--requests", type=int, default=200)
    p.add_argument("--budget-mib", type=int, default=1024, help="serve: HBM budget of the server")
    p.add_argument("--load", type=float, default=0.7)
    p.add_argument("--no-batched", action="store_true", help="periodic: skip the batched-cavities sub-record")
    p.add_argument("--no-serve", action="store_true", help="periodic: skip the serving sub-record")
    p.add_argument("--batched-steps", type=int, default=2000,
                   help="periodic: steps of every cavity in the batched sub-record")
    p.add_argument("--serve-requests", type=int, default=300, help="periodic: requests of the serving sub-record")
    p.add_argument("--batched-only", action="store_true",
                   help="cavities: time the batched form only (profiling runs)")
    p.add_argument("--batch-shape", default=None,
                   help="cavities: fix the batch tile shape (no autotuning), "
                        "fuse:rows0:rows1:rows2:rows3[:rows4[:lds[:vec_cap]]]")
    return p.parse_args()


# ------------------------------------------------------------------ periodic roofline run
def make_grid(n, storage, state, tune=True, kernel=None, planar=False):
    from paper_1912_09327_amd.grid import Grid
    g = Grid(n, n, prec=storage, periodic=3, planar=planar)
    g.set_geometry(None, *state)
    if kernel:
        if kernel == "gather":
            g.set_kernel("gather")
        else:
            parts = kernel.split(":")
            v, r, w = parts[1:4]
            f = parts[4] if len(parts) > 4 else 1
            g.set_kernel("strip", int(v), int(r), int(w), int(f))
    elif tune:
        g.autotune(steps=30, reps=3)
    return g


def reduction_block(per_launch):
    """Steps between two FP64 reductions: 100, or the whole number of launches of
    `per_launch` steps closest below it (99 for three-step launches)."""
    return max(per_launch, 100 // per_launch * per_launch)


def run_schedule(steps, warmup, per_launch):
    """The segments of a run of `warmup` untimed then `steps` timed steps: a list of
    (timed, steps of whole launches, remainder steps, reduce after).  The reduction
    runs every reduction_block() steps counted from the start of the run, warmup
    included, whatever the timed length; a segment ends at each reduction and at the
    end of the warmup, and its steps are split into whole launches and a remainder
    (shorter launches), so the kernel time per step comes from whole launches only."""
    block = reduction_block(per_launch)
    out = []
    t = 0
    for timed, n in ((False, warmup), (True, steps)):
        left = n
        while left > 0:
            k = min(left, block - t % block)
            whole = k - k % per_launch
            t += k
            left -= k
            out.append((timed, whole, k - whole, t % block == 0))
    return out


def timed_run(g, steps, warmup, torch, per_launch=1):
    """Warm up, then time exactly `steps` steps (the schedule of run_schedule), with
    HIP events on the grid's stream around the whole launches of every timed segment.
    Returns (wall seconds, kernel ms per step over whole launches, schedule info)."""
    s = g.stream
    sched = run_schedule(steps, warmup, per_launch)
    ev = []
    reductions = 0
    t0 = None
    for timed, whole, rem, red in sched:
        if timed and t0 is None:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        if timed and whole:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(s)
            g.step(whole)
            b.record(s)
            ev.append((a, b, whole))
        elif whole:
            g.step(whole)
        if rem:
            g.step(rem)
        if red:
            g.reduce()                       # FP64 mass / residual / non-finite, synchronises
            reductions += timed
    if t0 is None:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if ev:
        kern_ms = sum(a.elapsed_time(b) for a, b, _ in ev) / sum(k for _, _, k in ev)
    else:
        kern_ms = wall * 1e3 / max(steps, 1)
    info = dict(reduction_every=reduction_block(per_launch), reductions_timed=reductions,
                steps_in_whole_launches=sum(k for _, _, k in ev))
    return wall, kern_ms, info


def copy_ceiling(nbytes=2 << 30):
    """Achievable bandwidth of a plain streaming copy on this GPU (the library's probe:
    1 GiB read and 1 GiB written per launch, best launch shape)."""
    from paper_1912_09327_amd import _capi as C
    return C.probe_bandwidth(C.PROBE_COPY, nbytes, nontemporal=False, reps=3)


# Vector-ALU issue ceiling: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one wave64 VALU
# instruction per SIMD every 4 cycles), in T lane-operations/s.  Operations per update
# in the kernel expression: emission 29 and target sums 14; the 16-bit storage codec
# adds about 12.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
ALG_OPS_PER_LUP = {"f64": 43, "f32": 43, "f16s": 55, "bf16s": 55}


def kernel_source_hash():
    """Hash of the sources that define the step kernels' code (the kernel table
    that instantiates them is left out: adding an entry changes no kernel)."""
    h = hashlib.sha256()
    for f in ("lbt1_step.hpp", "lbt1_fused.hpp", "lbt1_device.hpp", "lbt1_args.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1912_09327_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def profile_record(name, storage, kernel_name):
    """The record of `kernel_name` for `storage` in a committed counter summary
    (one record, or a list of them for several strip shapes), if it was taken on
    these kernel sources; None otherwise."""
    try:
        recs = json.load(open(os.path.join(ROOT, "profiles", name)))[storage]
    except (OSError, KeyError, ValueError):
        return None
    for rec in recs if isinstance(recs, list) else [recs]:
        if rec.get("source_hash") == kernel_source_hash() and rec.get("kernel_bench") == kernel_name:
            return rec
    return None


def measured_valu(storage, kernel_name):
    """Vector-ALU lane operations per launch of the step kernel from the committed
    rocprofv3 summary (profiles/valu_periodic8192.json: SQ_INSTS_VALU per dispatch
    times 64 lanes), if it was taken on this kernel and these kernel sources."""
    rec = profile_record("valu_periodic8192.json", storage, kernel_name)
    return None if rec is None else rec["valu_per_dispatch"] * 64


def measured_traffic(storage, kernel_name, kernel_ms):
    """HBM traffic of the step kernel from the committed rocprofv3 counter summary
    (profiles/traffic_periodic8192.json: FETCH_SIZE and WRITE_SIZE per dispatch, each
    scaled by what the counter reads for a copy of known size), if it was taken on this
    kernel and these kernel sources; None otherwise."""
    rec = profile_record("traffic_periodic8192.json", storage, kernel_name)
    if rec is None:
        return None
    return dict(bytes_per_launch=rec["traffic_bytes"], ratio=rec["traffic_ratio"],
                GBps=rec["traffic_bytes"] / (kernel_ms * 1e-3) / 1e9)


def host_cpu():
    """CPU model, logical cores of the host and cores this process may use."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(model=model, host_logical_cores=os.cpu_count(), usable_cores=len(os.sched_getaffinity(0)))


def cpu_baseline(state, budget_s):
    """The FP64 oracle on a 2048 x 2048 window of the same random field, OpenMP over rows."""
    import oracle
    threads = len(os.sched_getaffinity(0))
    oracle.set_threads(threads)
    m = min(2048, state[0].shape[0])
    sub = [np.ascontiguousarray(a[:m, :m]) for a in state]
    oracle.run(*sub, 1, None, 3)                  # warm the thread pool
    t0 = time.perf_counter()
    oracle.run(*sub, 10, None, 3)
    one = (time.perf_counter() - t0) / 10
    n = max(1, int(budget_s / max(one, 1e-3)))
    t0 = time.perf_counter()
    oracle.run(*sub, n, None, 3)
    dt = time.perf_counter() - t0
    out = dict(value=round(m * m * n / dt / 1e6, 2), unit="MLUPS", cores=threads, kind="oracle", host=host_cpu(),
               sample=f"{m}x{m} periodic window of the same seed-0 random field, {n} steps, "
                      f"FP64, {threads} OpenMP threads, {dt:.1f} s")
    # the same oracle on one thread, a 512 x 512 window for about a third of the budget
    oracle.set_threads(1)
    s = 512
    sub1 = [np.ascontiguousarray(a[:s, :s]) for a in state]
    t0 = time.perf_counter()
    oracle.run(*sub1, 5, None, 3)
    one = (time.perf_counter() - t0) / 5
    n1 = max(1, int(budget_s / 3 / max(one, 1e-4)))
    t0 = time.perf_counter()
    oracle.run(*sub1, n1, None, 3)
    dt1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    out["single_thread"] = dict(value=round(s * s * n1 / dt1 / 1e6, 2), unit="MLUPS",
                                sample=f"{s}x{s} window, {n1} steps, FP64, 1 thread, {dt1:.1f} s")
    return out


def field_error(a, ref):
    """Max and rms difference of (rho, jx, jy) against the FP64 run, normalised by the
    FP64 field's rms (the random field decays, so absolute errors mislead)."""
    out = {}
    for name, x, r in zip(("rho", "jx", "jy"), a, ref):
        if name == "rho":
            x, r = x - 1.0, r - 1.0
        rms = float(np.sqrt(np.mean(r * r)))
        d = x - r
        out[name] = dict(max=float(np.abs(d).max() / rms), rms=float(np.sqrt(np.mean(d * d)) / rms))
    return out


ACC_STEPS = (1, 10, 100, 1000)
ACC_WINDOW = (3072, 3072, 2048, 2048)      # x0, y0, w, h of the sampled window


def accuracy(n, state, storages):
    """Error of each storage format against the FP64 run after 1, 10, 100 and 1000
    steps from the same start, on a 2048 x 2048 window of the grid (untimed)."""
    from paper_1912_09327_amd.grid import Grid
    x0, y0, w, h = ACC_WINDOW
    if n < x0 + w:
        x0 = y0 = 0
        w = h = n
    snaps = {}
    for storage in ["f64"] + [s for s in storages if s != "f64"]:
        g = Grid(n, n, prec=storage, periodic=3)
        try:
            g.set_geometry(None, *state)
            done = 0
            for k in ACC_STEPS:
                g.step(k - done)
                done = k
                snaps[(storage, k)] = g.read_window(x0, y0, w, h)
        finally:
            g.close()
    out = {}
    for storage in storages:
        if storage == "f64":
            continue
        out[storage] = {str(k): field_error(snaps[(storage, k)], snaps[("f64", k)]) for k in ACC_STEPS}
    return out, f"{w}x{h} window at ({x0}, {y0})"


def run_periodic(args, torch):
    from paper_1912_09327_amd import inputs as I
    n = args.n
    log(f"[bench] generating the {n}x{n} periodic field (seed 0)")
    state = I.random_periodic(n, n, seed=0)
    lups = float(n) * n
    results = {}
    order = [args.storage] + ([] if args.no_variants else
                              [s for s in ("f64", "f32", "f16s", "bf16s") if s != args.storage])
    for storage in order:
        log(f"[bench] {storage}: set_geometry + autotune")
        g = make_grid(n, storage, state, tune=not args.no_tune, kernel=args.kernel, planar=args.planar)
        cfg, kname = g.kernel()
        log(f"[bench] {storage}: kernel {kname} {cfg}")
        K = max(1, cfg.get("fuse", 1)) if cfg.get("kernel") == 2 else 1   # steps per launch
        wall, kms, sched = timed_run(g, args.steps, args.warmup, torch, K)
        c = VALUE_BYTES[storage]
        launch_ms = kms * K
        achieved = 2 * 3 * c * lups / (launch_ms * 1e-3) / 1e9
        results[storage] = dict(mlups=lups * args.steps / wall / 1e6, ms_per_step=wall * 1e3 / args.steps,
                                kernel_ms=launch_ms, steps_per_launch=K, achieved=achieved, kernel=kname,
                                config=cfg, schedule=sched)
        log(f"[bench] {storage}: {results[storage]['mlups']:.0f} MLUPS, launch {launch_ms:.4f} ms "
            f"({K} step(s)), "
            f"{achieved:.0f} GB/s")
        g.close()
        torch.cuda.empty_cache()
    head = results[args.storage]
    c = VALUE_BYTES[args.storage]
    line = {
        "metric": METRIC,
        "value": round(head["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.storage == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"periodic {n}x{n} random field (rho = 1 + 1e-3 N(0,1), "
                               f"u = 0.01 N(0,1), seed 0), {args.storage} moment storage",
                   "nx": n, "ny": n, "storage": args.storage, "fluid_nodes": int(lups),
                   "reduction_every": head["schedule"]["reduction_every"],
                   "reductions_timed": head["schedule"]["reductions_timed"],
                   "steps_in_whole_launches": head["schedule"]["steps_in_whole_launches"],
                   "kernel": head["kernel"], "kernel_config": head["config"]},
        "roofline": {"bound": "hbm", "achieved": round(head["achieved"], 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(head["achieved"] / HBM_PEAK_GBPS, 4), "traffic": None,
                     "bytes_per_launch": 2 * 3 * c * int(lups), "steps_per_launch": head["steps_per_launch"],
                     "bytes_per_lup": round(2 * 3 * c / head["steps_per_launch"], 3),
                     "kernel_ms": round(head["kernel_ms"], 5),
                     "single_step_equivalent_GBps": round(2 * 3 * c * head["mlups"] * 1e6 / 1e9, 1)},
    }
    tr = measured_traffic(args.storage, head["kernel"], head["kernel_ms"])
    if tr is not None:
        # same unit as `achieved`: counted HBM bytes per launch over the launch duration
        line["roofline"]["traffic"] = round(tr["GBps"], 1)
        line["roofline"]["traffic_bytes_per_launch"] = round(tr["bytes_per_launch"])
        line["roofline"]["traffic_over_algorithmic"] = round(tr["ratio"], 4)
    # the fused kernels are close to the vector-ALU issue ceiling as well: operations per
    # update from the kernel expression, and the VALU instructions rocprofv3 counted
    lups_launch = lups * head["steps_per_launch"]
    launch_s = head["kernel_ms"] * 1e-3
    ops = ALG_OPS_PER_LUP[args.storage]
    alu = {"achieved": round(ops * lups_launch / launch_s / 1e12, 2), "peak": round(VALU_PEAK_TOPS, 2),
           "unit": "T lane-op/s", "frac": round(ops * lups_launch / launch_s / 1e12 / VALU_PEAK_TOPS, 4),
           "ops_per_lup": ops, "counted": None}
    counted = measured_valu(args.storage, head["kernel"])
    if counted is not None:
        alu["counted"] = round(counted / launch_s / 1e12, 2)
        alu["counted_frac"] = round(counted / launch_s / 1e12 / VALU_PEAK_TOPS, 4)
        alu["counted_ops_per_lup"] = round(counted / lups_launch, 2)
    line["roofline"]["alu"] = alu
    try:
        cc = copy_ceiling()
        line["roofline"]["copy_ceiling_GBps"] = round(cc, 1)
        line["roofline"]["frac_of_copy"] = round(head["achieved"] / cc, 4)
    except Exception as e:  # pragma: no cover - measurement aid only
        log(f"[bench] copy ceiling failed: {e}")
    if not args.no_variants:
        log("[bench] accuracy of the storage formats against FP64 (untimed)")
        err, where = accuracy(n, state, list(results))
        torch.cuda.empty_cache()
        var = {}
        for s, r in results.items():
            v = dict(mlups=round(r["mlups"], 1), achieved_GBps=round(r["achieved"], 1),
                     frac=round(r["achieved"] / HBM_PEAK_GBPS, 4), kernel=r["kernel"])
            if s in err:
                v["error_vs_f64"] = dict(err[s], sample=where,
                                         normalised_by="rms of the FP64 field at the same step")
            var[s] = v
        line["variants"] = var
    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(state, args.cpu_seconds)
    del state
    torch.cuda.empty_cache()
    # the metric's second half: the batched and served forms against the plain
    # one-grid-at-a-time form, bounded samples of the uneven-cavity and request workloads
    from paper_1912_09327_amd import workloads as W
    if not args.no_batched:
        log(f"[bench] batched sub-record: {args.cavities} cavities x {args.batched_steps} steps")
        r = W.run_cavities(args.cavities, args.batched_steps, -1.0, torch, log)
        r["workload"] = (f"{r['cavities']} lid-driven cavities, side log-uniform [32, 512], lid U[0.01, 0.1], "
                         f"seed 4, FP16 shifted storage, FP32 arithmetic, {args.batched_steps} steps each, "
                         "residual check every 100 steps")
        line["batched"] = r
        torch.cuda.empty_cache()
    if not args.no_serve:
        budget = int(args.budget_mib) << 20
        log(f"[bench] serve sub-record: {args.serve_requests} requests at load {args.load}")
        cap, rate, reqs, served, s_srv, s_pl = W.run_serve(args.serve_requests, args.load, budget, torch, log)
        line["serve"] = dict(
            workload=f"{len(reqs)} Poisson requests (seed 5) at {rate:.3f}/s, load {args.load} of the measured "
                     f"capacity {cap:.3f}/s, half lid-driven cavities half porous channels, side 32..2048, "
                     f"budgets 1e3..1e5 steps, FP16 storage, {budget >> 20} MiB HBM budget, 64 slots",
            capacity_req_per_s=round(cap, 3), rate_per_s=round(rate, 3), server=s_srv, plain=s_pl,
            p99_speedup=round(s_pl["p99_s"] / s_srv["p99_s"], 2) if s_srv["p99_s"] else None,
            mlups_ratio=round(s_srv["mlups"] / s_pl["mlups"], 3) if s_pl["mlups"] else None)
    return line


def run_cavity(args, torch):
    """The 256 x 256 lid-driven cavity (walls x = 0, x = 255, y = 0; lid row y = 255,
    j = (0.1, 0)): 50,000 steps (--steps) in FP64 and FP32 storage with the autotuned
    kernel and the FP64 residual / mass reduction every 100 steps, as in section 3's
    convergence runs.  The grid (0.8-1.6 MB) stays in cache, so MLUPS here is no HBM
    claim.  Beside it, the FP64 oracle runs the same cavity on the host cores."""
    from paper_1912_09327_amd import inputs as I
    from paper_1912_09327_amd.grid import Grid
    n = args.cavity_n
    flags, rho, jx, jy, per = I.cavity(n, 0.1)
    fluid = int((flags == I.FLUID).sum())
    steps = args.cavity_steps
    res = {}
    for st in ("f64", "f32"):
        g = Grid(n, n, prec=st, periodic=per)
        g.set_geometry(flags, rho, jx, jy)
        if not args.no_tune:
            g.autotune(steps=30, reps=3)
        cfg, kname = g.kernel()
        g.step(200)
        g.reduce()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < steps:
            k = min(100, steps - done)
            g.step(k)
            done += k
            d = g.reduce()                   # synchronises
        wall = time.perf_counter() - t0
        res[st] = dict(kernel=kname, mlups=round(fluid * steps / wall / 1e6, 1), steps_per_s=round(steps / wall, 1),
                       us_per_step=round(wall / steps * 1e6, 2), final_residual=d["residual"],
                       mass_drift=d["mass"] - float(rho[flags == I.FLUID].sum()))
        log(f"[cavity] {st}: {kname}, {res[st]['mlups']:.0f} MLUPS, {res[st]['us_per_step']:.2f} us/step "
            f"(reduction every 100 steps), residual {d['residual']:.3e}")
        g.close()
    line = {
        "metric": METRIC, "value": res["f32"]["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": steps,
        "warmup": 200, "ms_per_step": round(res["f32"]["us_per_step"] / 1e3, 6), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{n}x{n} lid-driven cavity, lid j = (0.1, 0), {steps} steps, FP64 and FP32 "
                               "storage, reduction every 100 steps" + (" (cache-resident, no HBM claim)" if n <= 1024 else ""),
                   "fluid_nodes": fluid},
        "runs": res,
    }
    if not args.no_cpu:
        import oracle
        threads = len(os.sched_getaffinity(0))
        oracle.set_threads(threads)
        probe = max(1, min(1000, int(2e8 / (n * n))))      # about 0.5 s of oracle work
        oracle.run(rho, jx, jy, 1, flags, per)
        t0 = time.perf_counter()
        oracle.run(rho, jx, jy, probe, flags, per)
        one = (time.perf_counter() - t0) / probe
        m = max(1, min(steps, int(args.cpu_seconds / max(one, 1e-6))))
        t0 = time.perf_counter()
        oracle.run(rho, jx, jy, m, flags, per)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = dict(value=round(fluid * m / dt / 1e6, 2), unit="MLUPS", cores=threads, kind="oracle", host=host_cpu(),
                                    sample=f"the same {n}x{n} cavity, {m} steps, FP64, {threads} OpenMP threads, "
                                           f"{dt:.1f} s")
    return line


def run_compare(args, torch):
    """LBMTau1 (the autotuned default kernel, and one step per launch) against the
    stored-population BGK method (tau = 1 and tau = 0.6) on the periodic field:
    device bytes per node and MLUPS for each, in the storage format asked for."""
    from paper_1912_09327_amd import _capi as C
    from paper_1912_09327_amd import inputs as I
    from paper_1912_09327_amd.grid import Grid
    n, st = args.n, args.storage
    c = VALUE_BYTES[st]
    log(f"[compare] generating the {n}x{n} periodic field (seed 0)")
    state = I.random_periodic(n, n, seed=0)
    lups = float(n) * n
    rows = {}
    vec_fused = 4 if st == "f32" else 2
    variants = [
        ("lbmtau1_default", dict(populations=False), "tune"),
        ("lbmtau1_single", dict(populations=False), ("strip", 4 if st != "f64" else 2, 6, 0, 1)),
        ("bgk_tau1", dict(populations=True, tau=1.0), None),
        ("bgk_tau0.6", dict(populations=True, tau=0.6), None),
    ]
    for name, kw, kern in variants:
        g = Grid(n, n, prec=st, periodic=3, **kw)
        g.set_geometry(None, *state)
        if kern == "tune":
            g.autotune(steps=30, reps=3)      # the library's choice for this grid
        elif kern:
            g.set_kernel(*kern)
        cfg, kname = g.kernel()
        log(f"[compare] {name}: {kname}")
        K = cfg.get("fuse", 1) if cfg.get("kernel") == 2 else 1
        wall, kms, _ = timed_run(g, args.steps, args.warmup, torch, K)
        per_node = (2 * 9 * c) if kw["populations"] else (2 * 3 * c)     # state bytes per node
        alg = per_node * lups                                          # read + write per launch
        rows[name] = dict(kernel=kname, mlups=round(lups * args.steps / wall / 1e6, 1),
                          steps_per_launch=K, launch_ms=round(kms * K, 5),
                          achieved_GBps=round(alg / (kms * K * 1e-3) / 1e9, 1),
                          # without the residual snapshot (the paper's counts have none)
                          device_bytes_per_node=round(C.grid_bytes(n, n, C.PRECISIONS[st],
                                                                   g.options & ~C.OPT_SNAPSHOT) / lups, 3),
                          state_bytes_per_node=per_node)
        log(f"[compare] {name}: {rows[name]['mlups']:.0f} MLUPS, {rows[name]['achieved_GBps']:.0f} GB/s")
        g.close()
        torch.cuda.empty_cache()
    f, s1, b = rows["lbmtau1_default"], rows["lbmtau1_single"], rows["bgk_tau1"]
    return {
        "metric": METRIC,
        "value": f["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if st == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"LBMTau1 vs stored-population BGK, periodic {n}x{n} random field (seed 0), "
                               f"{st} storage", "nx": n, "ny": n, "storage": st},
        "methods": rows,
        "memory_ratio_bgk_over_lbmtau1": round(b["device_bytes_per_node"] / f["device_bytes_per_node"], 3),
        "speed_ratio_lbmtau1_over_bgk": round(f["mlups"] / b["mlups"], 2),
        "speed_ratio_single_step_over_bgk": round(s1["mlups"] / b["mlups"], 2),
        "paper_memory_per_node_float": {"standard_AB": 84, "lbmtau1": 24, "note": "section 4, formulas"},
    }


def run_stability(args, torch):
    """Re_max(L) of the lid-driven cavity: LBMTau1 at tau = 1 (every lid speed of a
    size as one batch), the stored-population BGK method at tau = 0.55, 0.7, 1.5
    (and 1 on the smaller sizes, as a cross-check); power-law fits beside the
    paper's."""
    from paper_1912_09327_amd import stability as S
    Ls = [50, 100, 200, 400, 700, 1000]
    speeds = S.lid_speeds(0.1, 1.6, 1.05)
    paper = {1.0: (12.0, 0.8), 1.5: (3.7, 0.89), 0.7: (19.0, 0.87), 0.55: (43.0, 0.93)}
    out = {}
    lups = 0.0
    t0 = time.perf_counter()
    runs = [("lbmtau1", 1.0)] + [("bgk", t) for t in (0.55, 0.7, 1.5)] + [("bgk", 1.0)]
    for method, tau in runs:
        rows = []
        for L in Ls:
            if method == "bgk" and tau == 1.0 and L > 200:
                continue
            if method == "lbmtau1":
                res = S.scan_batched(L, speeds, log=log)
            else:
                res = S.scan_populations(L, tau, speeds)
            lups += sum(((L - 2) * (L - 1)) * n for _, _, n in res)
            re = S.re_max_from_scan(L, tau, [(u, bad) for u, bad, _ in res])
            first_bad = next((u for u, bad, _ in res if bad), None)
            rows.append(dict(L=L, re_max=None if re is None else round(re, 1),
                             u0_max=None if re is None else round(re * S.viscosity(tau) / L, 4),
                             first_unstable_u0=None if first_bad is None else round(first_bad, 4),
                             paper_fit=round(paper[tau][0] * L ** paper[tau][1], 1)))
            log(f"[stability] {method} tau={tau} L={L}: Re_max {rows[-1]['re_max']} "
                f"(paper fit {rows[-1]['paper_fit']})")
        ok = [r for r in rows if r["re_max"]]
        fit = S.fit_power([r["L"] for r in ok], [r["re_max"] for r in ok]) if len(ok) >= 2 else (None, None)
        out[f"{method}_tau{tau}"] = dict(rows=rows, fit_a=fit[0] and round(fit[0], 3),
                                         fit_b=fit[1] and round(fit[1], 4), paper_a=paper[tau][0],
                                         paper_b=paper[tau][1])
    wall = time.perf_counter() - t0
    return {
        "metric": METRIC,
        "value": round(lups / wall / 1e6, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": None,
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "lid-driven cavity Re_max(L) sweep, L in 50..1000, lid speeds 0.1 * 1.05^k up to 1.6, "
                               "unstable = non-finite moments within max(1000, 4 L / u0) steps (at most 40000), "
                               "FP32 storage", "sizes": Ls},
        "seconds": round(wall, 2),
        "sweeps": out,
    }


def run_drop(args, torch):
    """The multiphase drop test of the paper's performance evaluation: a drop of
    radius L/4 in a periodic L x L box of vapour (Shan-Chen force, G = -5.5), run
    with multiphase LBMTau1 (no psi field, one kernel per step) and with the
    stored-population method (nine populations and a psi field, two kernels per
    step); iterations per second, MLUPS and device bytes per node against L."""
    from paper_1912_09327_amd import _capi as C
    from paper_1912_09327_amd.grid import Grid
    G = (-5.5, 1.0)
    st = args.storage
    rows = []
    for L in (128, 256, 512, 1024, 2048, 4096, 8192):
        y, x = np.mgrid[0:L, 0:L]
        d = np.hypot(x - L / 2 + 0.5, y - L / 2 + 0.5)
        rho = 0.104 + (2.307 - 0.104) * 0.5 * (1 - np.tanh((d - L / 4) / 2))
        z = np.zeros_like(rho)
        steps = max(200, min(5000, int(2e11 / (L * L) / 100) * 100))
        rec = dict(L=L, steps=steps)
        for name, kw in (("lbmtau1", {}), ("populations", dict(populations=True, tau=1.0))):
            g = Grid(L, L, prec=st, periodic=3, multiphase=G, **kw)
            g.set_geometry(None, rho, z, z)
            if not kw:
                g.autotune(steps=30, reps=3)
            wall, kms, _ = timed_run(g, steps, min(100, steps // 4), torch)
            dd = g.reduce()
            opts = g.options & ~C.OPT_SNAPSHOT
            rec[name] = dict(kernel=g.kernel()[1], it_per_s=round(steps / wall, 1),
                             mlups=round(L * L * steps / wall / 1e6, 1),
                             device_bytes_per_node=round(C.grid_bytes(L, L, C.PRECISIONS[st], opts) / (L * L), 3),
                             nonfinite=int(dd["nonfinite"]))
            g.close()
            torch.cuda.empty_cache()
        rec["speed_ratio"] = round(rec["lbmtau1"]["mlups"] / rec["populations"]["mlups"], 2)
        rec["memory_ratio"] = round(rec["populations"]["device_bytes_per_node"] /
                                    rec["lbmtau1"]["device_bytes_per_node"], 3)
        log(f"[drop] L={L}: LBMTau1 {rec['lbmtau1']['mlups']:.0f} MLUPS "
            f"({rec['lbmtau1']['it_per_s']:.0f} it/s), populations {rec['populations']['mlups']:.0f} MLUPS, "
            f"speed x{rec['speed_ratio']}, memory x{rec['memory_ratio']}")
        rows.append(rec)
    big = rows[-1]
    return {
        "metric": METRIC,
        "value": big["lbmtau1"]["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": big["steps"],
        "warmup": None,
        "ms_per_step": round(1e3 / big["lbmtau1"]["it_per_s"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if st == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": "multiphase drop test: drop of radius L/4 in periodic vapour, Shan-Chen force "
                               f"G = -5.5, psi = 1 - exp(-rho), tau = 1, {st} storage, L = 128..8192",
                   "storage": st},
        "sizes": rows,
    }


def run_3d(args, torch):
    """3-D LBMTau1 on periodic random fields (rho = 1 + 1e-3 N(0,1), u = 0.01 N(0,1),
    seed 0): MLUPS and algorithmic GB/s (2 * 4 * c bytes per LUP) for D3Q19 and D3Q27,
    with device bytes per node against the standard method's (2 Q + 4) c; and a
    lid-driven box of the same sides, D3Q19, with the tile and the gather kernel."""
    from paper_1912_09327_amd import _capi as C
    from paper_1912_09327_amd.grid3d import Grid3D
    st = args.storage
    c = VALUE_BYTES[st]
    rows = []
    for n in [int(v) for v in args.n3.split(",")]:
        g0 = np.random.default_rng(0).standard_normal((4, n, n, n), dtype=np.float32)
        rho = 1.0 + 1e-3 * g0[0].astype(np.float64)
        js = [rho * (0.01 * g0[k].astype(np.float64)) for k in (1, 2, 3)]
        del g0
        for q in [int(v) for v in args.q3.split(",")]:
            g = Grid3D(n, n, n, q=q, prec=st, periodic=7)
            g.set_geometry(None, rho, *js)
            steps = args.steps3 or (200 if n <= 256 else 50)
            g.step(10)
            g.sync()
            s = g.stream
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            a.record(s)
            g.step(steps)
            b.record(s)
            d = g.reduce()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            kms = a.elapsed_time(b) / steps
            lups = float(n) ** 3
            rec = dict(n=n, q=q, steps=steps, mlups=round(lups * steps / wall / 1e6, 1), kernel_ms=round(kms, 4),
                       achieved_GBps=round(2 * 4 * c * lups / (kms * 1e-3) / 1e9, 1),
                       device_bytes_per_node=round(C.lib.lbt1_grid3d_bytes(n, n, n, q, C.PRECISIONS[st], 0) / lups, 3),
                       standard_bytes_per_node=(2 * q + 4) * c, nonfinite=int(d["nonfinite"]))
            rec["memory_saving"] = round(1 - rec["device_bytes_per_node"] / rec["standard_bytes_per_node"], 4)
            log(f"[3d] {n}^3 D3Q{q}: {rec['mlups']:.0f} MLUPS, {rec['achieved_GBps']:.0f} GB/s, "
                f"{rec['device_bytes_per_node']:.1f} vs {rec['standard_bytes_per_node']} B/node")
            rows.append(rec)
            g.close()
            torch.cuda.empty_cache()
        del rho, js
    # walled: a lid-driven box (SOLID faces, the top plane FIXED at u = (0.05, 0, 0)),
    # D3Q19, the tile kernel (its wall-aware form) against one thread per node
    walled = []
    for n in [int(v) for v in args.n3.split(",")]:
        flags = np.zeros((n, n, n), np.uint8)
        flags[0] = flags[:, 0] = flags[:, -1] = flags[:, :, 0] = flags[:, :, -1] = 1
        flags[-1, 1:-1, 1:-1] = 2
        rho = np.ones((n, n, n))
        jx = np.where(flags == 2, 0.05, 0.0)
        zero = np.zeros((n, n, n))
        for kern in ("tile", "gather"):
            g = Grid3D(n, n, n, q=19, prec=st, periodic=0)
            g.set_kernel(kern)
            g.set_geometry(flags, rho, jx, zero, zero)
            steps = args.steps3 or (200 if n <= 256 else 50)
            g.step(10)
            g.sync()
            s = g.stream
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(s)
            g.step(steps)
            b.record(s)
            torch.cuda.synchronize()
            kms = a.elapsed_time(b) / steps
            fluid = float(((flags == 0).sum()))
            rec = dict(n=n, q=19, kernel=kern, steps=steps, kernel_ms=round(kms, 4),
                       mlups=round(fluid / (kms * 1e-3) / 1e6, 1),
                       achieved_GBps=round(2 * 4 * c * n ** 3 / (kms * 1e-3) / 1e9, 1))
            log(f"[3d] box {n}^3 D3Q19 {kern}: {rec['mlups']:.0f} MLUPS (fluid nodes), {rec['achieved_GBps']:.0f} GB/s")
            walled.append(rec)
            g.close()
            torch.cuda.empty_cache()
        del flags, rho, jx, zero
    head = max(rows, key=lambda r: (r["n"], r["q"] == 19))
    return {
        "metric": METRIC,
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": head["steps"],
        "warmup": 10,
        "ms_per_step": head["kernel_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if st == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"3-D LBMTau1, periodic random field (seed 0), {st} storage, 256^3 and 512^3, "
                               "D3Q19 and D3Q27", "storage": st},
        "roofline": {"bound": "hbm", "achieved": head["achieved_GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(head["achieved_GBps"] / HBM_PEAK_GBPS, 4), "traffic": None,
                     "bytes_per_lup": 2 * 4 * c},
        "runs": rows,
        "walled": walled,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent grids would shard across GPUs with no exchange; see the design notes)",
              file=sys.stderr)
        return 2
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    if args.workload == "periodic":
        line = run_periodic(args, torch)
    elif args.workload == "3d":
        line = run_3d(args, torch)
    elif args.workload == "drop":
        line = run_drop(args, torch)
    elif args.workload == "stability":
        line = run_stability(args, torch)
    elif args.workload == "cavity":
        line = run_cavity(args, torch)
    elif args.workload == "compare":
        line = run_compare(args, torch)
    elif args.workload == "cavities":
        from paper_1912_09327_amd.workloads import bench_cavities
        line = bench_cavities(args, torch, log)
    else:
        from paper_1912_09327_amd.workloads import bench_serve
        line = bench_serve(args, torch, log)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

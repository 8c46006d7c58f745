"""Continuous-batching server for LBMTau1 solves, and the plain FIFO baseline.

Requests (cavities, porous channels, ... of different sizes) arrive over time.
The server admits a request as soon as its grid fits the HBM budget and a slot
is free, keeps its moment fields resident, and steps all resident grids
together in bursts (one fused launch per time step for all of them, see
``lbt1_batch_run``); a grid finishes when its residual reaches the tolerance or
its step budget is used, and its slot and memory are handed to the next
request at once.  Latency is finish time minus arrival time, queueing
included.

Admission is in arrival order, except that a request that does not fit the
free HBM budget may be overtaken by later ones that do, at most
``max_overtakes`` times; after that nothing behind it is admitted until it is
(a reservation, so no request starves).

The plain baseline serves the same requests one at a time in arrival order,
each stepped alone with ``lbt1_step`` (the library's default kernel for the grid,
graph bursts) and the same residual checks at the same burst boundaries, so each
result is bit-for-bit the one the server produces for it.

The scheduling logic talks to a ``Backend`` (``GpuBackend`` here); the tests
drive it with a CPU stand-in.
"""
import collections
import concurrent.futures
import time
from dataclasses import dataclass, field

import numpy as np

from . import inputs as I


@dataclass
class Request:
    id: int
    arrival: float          # seconds after the start of the run
    kind: str               # "cavity" | "channel"
    L: int
    steps: int              # step budget
    u: float = 0.05
    porosity: float = 0.8
    seed: int = 0
    tol: float = -1.0       # residual tolerance (negative: run the whole budget)


@dataclass
class Result:
    id: int
    arrival: float
    admitted: float
    finished: float
    steps: int
    state: str              # "budget" | "converged" | "nonfinite" | "refused"
    residual: float
    lups: float             # fluid node updates done
    moments: tuple = field(default=None, repr=False)

    @property
    def latency(self):
        return self.finished - self.arrival


def requests_from_stream(dicts, tol=-1.0):
    return [Request(id=d["id"], arrival=d["arrival"], kind=d["kind"], L=d["L"], steps=d["steps"], u=d["u"],
                    porosity=d["porosity"], seed=d["seed"], tol=tol) for d in dicts]


def geometry(req):
    """(flags, rho, jx, jy, periodic, force) of a request (seeded, see ``inputs``)."""
    return I.build_request(dict(kind=req.kind, L=req.L, u=req.u, porosity=req.porosity, seed=req.seed))


# ------------------------------------------------------------------ backends
class Backend:
    """What the schedulers need from an engine."""

    def grid_bytes(self, req):          # device bytes the request's grid takes
        raise NotImplementedError

    def create(self, req, geo=None):    # the grid with geometry `geo` (built if None); a handle
        raise NotImplementedError

    def admit(self, handle, step_budget, tol):   # slot id, or None if the engine is full
        raise NotImplementedError

    def run(self, burst):               # one burst for every resident, running grid
        raise NotImplementedError

    def finished(self):                 # [(slot, state, steps, residual)] of finished slots
        raise NotImplementedError

    def evict(self, slot):              # returns the handle
        raise NotImplementedError

    def read(self, handle):             # (rho, jx, jy) of a grid
        raise NotImplementedError

    def release(self, handle):
        raise NotImplementedError

    def fluid_nodes(self, handle):
        raise NotImplementedError

    # plain path: one grid, one launch per step
    def run_alone(self, handle, step_budget, tol, burst):
        """Steps one grid by itself until the residual reaches tol (checked every
        `burst` steps) or the budget is used; returns (state, steps, residual)."""
        raise NotImplementedError


class GpuBackend(Backend):
    """The HIP library: grids in torch-owned device memory, a ``Batch`` for the server."""

    def __init__(self, hbm_budget_bytes, max_slots, prec="f16s", wall="paper", scale=(0.0, 0.0)):
        from . import _capi as C
        from .batch import Batch
        self.C = C
        self.prec = prec
        self.wall = wall
        self.scale = scale
        self.batch = Batch(hbm_budget_bytes, max_slots)
        self.slot_handle = {}

    def grid_bytes(self, req):
        return self.C.grid_bytes(req.L, req.L, self.C.PRECISIONS[self.prec], self.C.OPT_SNAPSHOT)

    def create(self, req, geo=None):
        from .grid import Grid
        flags, rho, jx, jy, periodic, force = geo if geo is not None else geometry(req)
        g = Grid(req.L, req.L, prec=self.prec, wall=self.wall, periodic=periodic, force=force,
                 scale=self.scale)
        g.set_geometry(flags, rho, jx, jy)
        g.fluid = int((flags == I.FLUID).sum())
        return g

    def admit(self, handle, step_budget, tol):
        slot = self.batch.admit(handle, step_budget, tol)
        if slot is not None:
            self.slot_handle[slot] = handle
        return slot

    def run(self, burst):
        self.batch.run(burst)

    def finished(self):
        C = self.C
        names = {C.SLOT_BUDGET: "budget", C.SLOT_CONVERGED: "converged", C.SLOT_NONFINITE: "nonfinite"}
        out = []
        for slot in self.batch.poll():
            st, steps, res = self.batch.slot_info(slot)
            out.append((slot, names[st], steps, res))
        return out

    def evict(self, slot):
        self.batch.evict(slot)
        return self.slot_handle.pop(slot)

    def read(self, handle):
        return handle.read_moments()

    def release(self, handle):
        handle.close()

    def fluid_nodes(self, handle):
        return handle.fluid

    def run_alone(self, handle, step_budget, tol, burst):
        steps, residual, state = 0, float("nan"), "budget"
        while steps < step_budget:
            k = min(burst, step_budget - steps)
            handle.step(k)
            steps += k
            d = handle.reduce(self.C.REDUCE_RESIDUAL | self.C.REDUCE_NONFINITE)
            residual = d["residual"]
            if d["nonfinite"] > 0:
                return "nonfinite", steps, residual
            if tol >= 0 and residual <= tol:
                return "converged", steps, residual
        return state, steps, residual

    def close(self):
        self.batch.close()


# ------------------------------------------------------------------ schedulers
class Server:
    """Continuous batching with admission by HBM budget and slot count."""

    def __init__(self, backend, hbm_budget_bytes, max_slots, burst=100, keep_results=False, clock=None,
                 sleep=None, progress=None, max_overtakes=16):
        self.b = backend
        self.budget = int(hbm_budget_bytes)
        self.max_slots = int(max_slots)
        self.burst = int(burst)
        self.max_overtakes = int(max_overtakes)
        self.overtaken = {}            # request id -> times a later request was admitted first
        self.keep = keep_results
        self.clock = clock or time.perf_counter
        self.sleep = sleep or time.sleep
        self.progress = progress       # optional callable(done_count, now)

    def serve(self, requests):
        """Serve `requests` (arrival times relative to the call); returns the Results
        in completion order."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue = collections.deque()
        active = {}                    # slot -> (request, handle, admitted, bytes)
        used = 0
        done = []
        # geometry of queued requests is built on a host thread while the GPU steps
        pool = concurrent.futures.ThreadPoolExecutor(max_workers=2)
        geo = {}
        t0 = self.clock()
        while pending or queue or active:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                req = pending.popleft()
                queue.append(req)
                geo[req.id] = pool.submit(geometry, req)
            # admit in arrival order; a request the free budget cannot hold yet may be
            # overtaken by later ones that fit, at most max_overtakes times, after which
            # nothing behind it is admitted before it (no starvation)
            i = 0
            blocked = []               # requests ahead of i that did not fit
            while i < len(queue) and len(active) < self.max_slots:
                req = queue[i]
                nbytes = self.b.grid_bytes(req)
                if nbytes > self.budget:
                    # can never fit: refused at once, the queue moves on
                    del queue[i]
                    geo.pop(req.id).cancel()
                    now = self.clock() - t0
                    done.append(Result(req.id, req.arrival, now, now, 0, "refused", float("nan"), 0.0))
                    if self.progress:
                        self.progress(len(done), now)
                    continue
                if used + nbytes > self.budget:
                    if self.overtaken.get(req.id, 0) >= self.max_overtakes:
                        break          # reserved: wait until it fits
                    blocked.append(req)
                    i += 1
                    continue
                handle = self.b.create(req, geo.pop(req.id).result())
                slot = self.b.admit(handle, req.steps, req.tol)
                if slot is None:       # the engine's own accounting disagrees: wait
                    self.b.release(handle)
                    geo[req.id] = pool.submit(geometry, req)   # built again for the next try
                    break
                del queue[i]
                for r in blocked:
                    self.overtaken[r.id] = self.overtaken.get(r.id, 0) + 1
                active[slot] = (req, handle, self.clock() - t0, nbytes)
                used += nbytes
            if active:
                self.b.run(self.burst)
                now = self.clock() - t0
                for slot, state, steps, res in self.b.finished():
                    req, handle, adm, nbytes = active.pop(slot)
                    self.b.evict(slot)
                    mom = self.b.read(handle) if self.keep else None
                    done.append(Result(req.id, req.arrival, adm, now, steps, state, res,
                                       float(steps) * self.b.fluid_nodes(handle), mom))
                    self.b.release(handle)
                    used -= nbytes
                    if self.progress:
                        self.progress(len(done), now)
            elif pending:
                wait = pending[0].arrival - (self.clock() - t0)
                if wait > 0:
                    self.sleep(min(wait, 0.05))
        pool.shutdown()
        return done


class PlainFifo:
    """One request at a time, in arrival order, one launch per step."""

    def __init__(self, backend, burst=100, keep_results=False, clock=None, sleep=None, progress=None,
                 budget=None):
        self.b = backend
        self.budget = budget           # requests larger than this are refused (None: no limit)
        self.burst = int(burst)
        self.keep = keep_results
        self.clock = clock or time.perf_counter
        self.sleep = sleep or time.sleep
        self.progress = progress

    def serve(self, requests):
        done = []
        order = sorted(requests, key=lambda r: r.arrival)
        pool = concurrent.futures.ThreadPoolExecutor(max_workers=1)
        nxt = pool.submit(geometry, order[0]) if order else None
        t0 = self.clock()
        for k, req in enumerate(order):
            now = self.clock() - t0
            if req.arrival > now:
                self.sleep(req.arrival - now)
            adm = self.clock() - t0
            g = nxt.result()
            # the next request's geometry is built while this one runs
            nxt = pool.submit(geometry, order[k + 1]) if k + 1 < len(order) else None
            if self.budget is not None and self.b.grid_bytes(req) > self.budget:
                done.append(Result(req.id, req.arrival, adm, adm, 0, "refused", float("nan"), 0.0))
                if self.progress:
                    self.progress(len(done), adm)
                continue
            handle = self.b.create(req, g)
            state, steps, res = self.b.run_alone(handle, req.steps, req.tol, self.burst)
            now = self.clock() - t0
            mom = self.b.read(handle) if self.keep else None
            done.append(Result(req.id, req.arrival, adm, now, steps, state, res,
                               float(steps) * self.b.fluid_nodes(handle), mom))
            self.b.release(handle)
            if self.progress:
                self.progress(len(done), now)
        pool.shutdown()
        return done


def summarize(results, wall_seconds=None):
    """p50 / p99 latency (over the requests served; refused ones are counted apart),
    aggregate MLUPS and counts of a finished run."""
    served = [r for r in results if r.state != "refused"]
    lat = np.array([r.latency for r in served]) if served else np.zeros(1)
    lups = sum(r.lups for r in served)
    if wall_seconds is None:
        wall_seconds = max(r.finished for r in results) - min(r.arrival for r in results)
    return dict(n=len(results), served=len(served), p50_s=float(np.percentile(lat, 50)),
                p99_s=float(np.percentile(lat, 99)), mean_s=float(lat.mean()),
                mlups=lups / max(wall_seconds, 1e-12) / 1e6, wall_s=wall_seconds,
                states=dict(collections.Counter(r.state for r in results)))

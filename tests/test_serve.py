"""Scheduler tests on the CPU: the server and the plain FIFO path driven by a
stand-in backend built on the CPU oracle (same Backend interface as the GPU
engine).  Admission by HBM budget and slots, continuous refill, latency
accounting, failure isolation and the alone-vs-mix identity."""
import numpy as np
import pytest

import oracle
from paper_1912_09327_amd import inputs as I
from paper_1912_09327_amd.serve import Backend, PlainFifo, Request, Server, geometry, summarize


class FakeClock:
    """Simulated time: each burst of the backend advances it by its modelled cost."""

    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class OracleBackend(Backend):
    BYTES_PER_NODE = 13

    def __init__(self, clock, slots, sec_per_lup=1e-9):
        self.clock = clock
        self.slots = [None] * slots
        self.sec_per_lup = sec_per_lup
        self.max_active = 0
        self.poison = set()        # request ids whose state is made non-finite at the first burst

    def grid_bytes(self, req):
        return req.L * req.L * self.BYTES_PER_NODE

    def create(self, req, geo=None):
        flags, rho, jx, jy, per, F = geo if geo is not None else geometry(req)
        n = req.L
        rho = np.ones((n, n)) if rho is None else rho
        jx = np.zeros((n, n)) if jx is None else jx
        jy = np.zeros((n, n)) if jy is None else jy
        return dict(req=req, flags=flags, per=per, F=F, state=[rho, jx, jy],
                    snap=[rho.copy(), jx.copy(), jy.copy()], fluid=int((flags == 0).sum()))

    def admit(self, h, budget, tol):
        for i, s in enumerate(self.slots):
            if s is None:
                self.slots[i] = dict(h=h, budget=budget, tol=tol, taken=0, state="running", res=np.nan)
                self.max_active = max(self.max_active, sum(x is not None for x in self.slots))
                return i
        return None

    def _advance(self, h, k):
        if h["req"].id in self.poison:
            h["state"][1][h["flags"] == 0] = np.nan
        h["state"] = list(oracle.run(*h["state"], k, h["flags"], h["per"], h["F"], 0))
        d = oracle.reduce(*h["state"], flags=h["flags"], snapshot=h["snap"])
        h["snap"] = [a.copy() for a in h["state"]]
        self.clock.t += k * h["fluid"] * self.sec_per_lup
        return d

    def run(self, burst):
        for s in self.slots:
            if s is None or s["state"] != "running":
                continue
            k = min(burst, s["budget"] - s["taken"])
            d = self._advance(s["h"], k)
            s["taken"] += k
            s["res"] = d["residual"]
            if d["nonfinite"]:
                s["state"] = "nonfinite"
            elif s["tol"] >= 0 and d["residual"] <= s["tol"]:
                s["state"] = "converged"
            elif s["taken"] >= s["budget"]:
                s["state"] = "budget"

    def finished(self):
        return [(i, s["state"], s["taken"], s["res"]) for i, s in enumerate(self.slots)
                if s is not None and s["state"] != "running"]

    def evict(self, slot):
        h = self.slots[slot]["h"]
        self.slots[slot] = None
        return h

    def read(self, h):
        return tuple(a.copy() for a in h["state"])

    def release(self, h):
        pass

    def fluid_nodes(self, h):
        return h["fluid"]

    def run_alone(self, h, budget, tol, burst):
        taken, res = 0, np.nan
        while taken < budget:
            k = min(burst, budget - taken)
            d = self._advance(h, k)
            taken += k
            res = d["residual"]
            if d["nonfinite"]:
                return "nonfinite", taken, res
            if tol >= 0 and res <= tol:
                return "converged", taken, res
        return "budget", taken, res


def _reqs(n, seed=0, rate=200.0):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    out = []
    for i in range(n):
        kind = "cavity" if i % 2 == 0 else "channel"
        out.append(Request(id=i, arrival=float(t[i]), kind=kind, L=int(rng.integers(12, 24)),
                           steps=int(rng.integers(100, 400)), u=0.05, porosity=0.85, seed=i, tol=-1.0))
    return out


def test_admission_respects_budget_and_slots():
    clock = FakeClock()
    be = OracleBackend(clock, slots=8)
    reqs = _reqs(12)
    budget = 2 * 24 * 24 * OracleBackend.BYTES_PER_NODE      # at most ~2 grids resident
    res = Server(be, budget, max_slots=8, burst=50, clock=clock, sleep=clock.sleep).serve(reqs)
    assert len(res) == len(reqs)
    assert 1 <= be.max_active <= 2
    burst_of_arrivals = _reqs(12)
    for r in burst_of_arrivals:
        r.arrival = 0.0
    be2 = OracleBackend(FakeClock(), slots=8)
    Server(be2, 10 ** 9, max_slots=3, burst=50, clock=be2.clock, sleep=be2.clock.sleep).serve(burst_of_arrivals)
    assert be2.max_active == 3


def test_continuous_refill_and_latency_accounting():
    clock = FakeClock()
    be = OracleBackend(clock, slots=4, sec_per_lup=1e-6)      # requests overlap in time
    reqs = _reqs(10)
    res = Server(be, 10 ** 9, max_slots=4, burst=50, clock=clock, sleep=clock.sleep).serve(reqs)
    by_id = {r.id: r for r in res}
    for q in reqs:
        r = by_id[q.id]
        assert r.admitted >= q.arrival - 1e-12
        assert r.finished >= r.admitted
        assert r.latency == pytest.approx(r.finished - q.arrival)
        assert r.steps == q.steps and r.state == "budget"
    # a slot freed by an early finisher is reused before the slowest resident grid ends
    order = sorted(res, key=lambda r: r.admitted)
    first_finish = min(r.finished for r in res)
    assert any(first_finish <= r.admitted < max(x.finished for x in order[:4]) for r in order[4:])
    s = summarize(res)
    assert s["n"] == 10 and s["p99_s"] >= s["p50_s"] > 0 and s["mlups"] > 0


def test_alone_and_in_the_mix_give_the_same_results():
    reqs = _reqs(8, seed=3)
    for r in reqs[::3]:
        r.tol = 1e-7                 # some stop early on their residual
    be = OracleBackend(FakeClock(), slots=3)
    mix = {r.id: r for r in Server(be, 10 ** 9, 3, burst=40, keep_results=True, clock=be.clock, sleep=be.clock.sleep).serve(reqs)}
    be2 = OracleBackend(FakeClock(), slots=1)
    alone = {r.id: r for r in PlainFifo(be2, burst=40, keep_results=True, clock=be2.clock, sleep=be2.clock.sleep).serve(reqs)}
    for i in mix:
        assert mix[i].steps == alone[i].steps and mix[i].state == alone[i].state
        for a, b in zip(mix[i].moments, alone[i].moments):
            assert np.array_equal(a, b)


def test_nonfinite_grid_is_reported_and_isolated():
    reqs = _reqs(6, seed=5)
    be = OracleBackend(FakeClock(), slots=6)
    be.poison = {2}
    res = {r.id: r for r in Server(be, 10 ** 9, 6, burst=50, keep_results=True, clock=be.clock, sleep=be.clock.sleep).serve(reqs)}
    assert res[2].state == "nonfinite" and res[2].steps == 50
    be2 = OracleBackend(FakeClock(), slots=1)
    alone = {r.id: r for r in PlainFifo(be2, burst=50, keep_results=True, clock=be2.clock, sleep=be2.clock.sleep).serve(reqs)}
    for i in res:
        if i != 2:
            assert res[i].state == "budget"
            for a, b in zip(res[i].moments, alone[i].moments):
                assert np.array_equal(a, b)


def test_request_larger_than_the_budget_is_refused():
    """A request that can never fit is refused at once; the others are served."""
    reqs = _reqs(4)
    reqs[1].L = 200                                   # 200^2 * 13 B > the budget below
    budget = 30 * 30 * OracleBackend.BYTES_PER_NODE
    be = OracleBackend(FakeClock(), slots=2)
    res = {r.id: r for r in Server(be, budget, 2, clock=be.clock, sleep=be.clock.sleep).serve(reqs)}
    assert res[1].state == "refused" and res[1].steps == 0
    assert all(res[i].state == "budget" for i in (0, 2, 3))
    be2 = OracleBackend(FakeClock(), slots=1)
    plain = {r.id: r for r in PlainFifo(be2, clock=be2.clock, sleep=be2.clock.sleep, budget=budget).serve(reqs)}
    assert plain[1].state == "refused" and all(plain[i].state == "budget" for i in (0, 2, 3))
    s = summarize(list(res.values()))
    assert s["served"] == 3 and s["states"]["refused"] == 1


def test_small_requests_overtake_a_blocked_head_within_a_bound():
    """A request the free budget cannot hold yet is overtaken by later ones that fit,
    at most max_overtakes times; then it is reserved and admitted before any later one."""
    big = Request(id=0, arrival=0.0, kind="cavity", L=20, steps=100, seed=0)
    long_ = Request(id=1, arrival=0.0, kind="cavity", L=20, steps=2000, seed=1)
    smalls = [Request(id=10 + k, arrival=0.001 * k, kind="cavity", L=10, steps=100, seed=k) for k in range(12)]
    budget = (20 * 20 + 12 * 12) * OracleBackend.BYTES_PER_NODE   # one 20^2 grid plus some small ones
    for cap, expect_before in ((16, 12), (3, 3)):
        be = OracleBackend(FakeClock(), slots=8, sec_per_lup=1e-6)   # the long grid holds its memory
        srv = Server(be, budget, 8, burst=50, clock=be.clock, sleep=be.clock.sleep, max_overtakes=cap)
        res = {r.id: r for r in srv.serve([long_, big] + smalls)}
        # the long grid holds the budget; the big one waits for it, small ones overtake it
        before = [r for r in res.values() if r.id >= 10 and r.admitted < res[0].admitted]
        assert len(before) == expect_before, (cap, len(before))
        assert srv.overtaken[0] == expect_before
        assert all(r.state == "budget" for r in res.values())


def test_request_stream_shapes():
    reqs = I.request_stream(200, seed=5, rate=2.0)
    assert len(reqs) == 200
    L = np.array([r["L"] for r in reqs])
    st = np.array([r["steps"] for r in reqs])
    assert L.min() >= 32 and L.max() <= 2048 and st.min() >= 1000 and st.max() <= 100000
    assert 0.35 < np.mean([r["kind"] == "cavity" for r in reqs]) < 0.65
    arr = np.array([r["arrival"] for r in reqs])
    assert np.all(np.diff(arr) > 0)
    assert np.mean(np.diff(arr)) == pytest.approx(0.5, rel=0.2)


def test_porous_channel_generator():
    rng = np.random.default_rng(7)
    for target in (0.6, 0.75, 0.9):
        flags, per, phi = I.porous_channel(128, rng, porosity=target)
        assert per == I.PERIODIC_X
        assert (flags[0] == I.SOLID).all() and (flags[-1] == I.SOLID).all()
        assert phi <= target + 1e-12 and phi > target - 0.1

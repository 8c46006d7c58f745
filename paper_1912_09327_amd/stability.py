"""Largest stable Reynolds number of the lid-driven cavity (the paper's
Discussion section and its Re_max figure).

Protocol, as the paper states it: for a cavity of side L the lid speed u0,
and with it Re = u0 L / nu (Eq. Reynolds, nu = (tau - 1/2)/3, 1/6 at tau = 1),
is raised until a run becomes unstable; the Re before the first unstable one
is Re_max(L).  A power law Re_max = a L^b is fitted by least squares in
log-log.  Readings where the paper is silent:

* the scan: u0 = u_lo * ratio^k (k = 0, 1, ...) up to u_hi;
* a run is unstable when its moments become non-finite (the FP64 non-finite
  count of the reduction, checked every 100 steps) within its horizon;
* the horizon: at least 1000 steps (the paper's "at least 1000 time steps")
  and at least `transits` lid transit times L / u0, at most `max_steps`.

At tau = 1 the cavities of one L are run together as one batch of LBMTau1
grids (every cavity of the scan resident, one fused launch per step).  At
other tau the stored-population BGK grids are run one at a time.
"""
import math

import numpy as np

from . import inputs as I


def viscosity(tau):
    """Eq. viscosity: nu = (tau - 1/2) / 3."""
    return (tau - 0.5) / 3.0


def reynolds(u0, L, tau=1.0):
    """Eq. Reynolds: Re = u0 L / nu."""
    return u0 * L / viscosity(tau)


def lid_speeds(u_lo=0.02, u_hi=1.5, ratio=1.06):
    n = int(math.floor(math.log(u_hi / u_lo) / math.log(ratio))) + 1
    return [u_lo * ratio ** k for k in range(n)]


def horizon(L, u0, transits=4.0, min_steps=1000, max_steps=40000):
    """Steps a run is given: at least min_steps and `transits` lid transit times."""
    return int(min(max_steps, max(min_steps, math.ceil(transits * L / u0 / 100.0) * 100)))


def re_max_from_scan(L, tau, results):
    """results: [(u0, unstable)] in increasing u0.  The Re of the last stable
    speed before the first unstable one (None if the first is unstable, the
    last speed's Re if none is)."""
    prev = None
    for u0, bad in results:
        if bad:
            return None if prev is None else reynolds(prev, L, tau)
        prev = u0
    return reynolds(prev, L, tau) if prev is not None else None


def fit_power(Ls, Re):
    """Least-squares fit of log Re = log a + b log L.  Returns (a, b)."""
    x = np.log(np.asarray(Ls, dtype=float))
    y = np.log(np.asarray(Re, dtype=float))
    b, loga = np.polyfit(x, y, 1)
    return float(math.exp(loga)), float(b)


def scan_batched(L, speeds, prec="f32", transits=4.0, max_steps=40000, burst=100, log=None):
    """tau = 1: every lid speed of the scan as one LBMTau1 cavity, all in one
    batch.  Returns [(u0, unstable, steps)]."""
    from . import _capi as C
    from .batch import Batch
    from .grid import Grid
    grids, slots = [], []
    for u0 in speeds:
        flags, rho, jx, jy, per = I.cavity(L, u0)
        g = Grid(L, L, prec=prec, periodic=per)
        g.set_geometry(flags, rho, jx, jy)
        grids.append(g)
    b = Batch(sum(g.nbytes for g in grids) + (1 << 20), len(grids))
    try:
        for g, u0 in zip(grids, speeds):
            s = b.admit(g, horizon(L, u0, transits, max_steps=max_steps), -1.0)
            assert s is not None
            slots.append(s)
        bursts = 0
        while len(b.poll()) < len(grids):
            b.run(burst)
            bursts += 1
            if log and bursts % 100 == 0:
                log(f"[stability] L={L}: {bursts * burst} steps, {len(b.poll())}/{len(grids)} done")
        out = []
        for u0, s in zip(speeds, slots):
            state, steps, _ = b.slot_info(s)
            out.append((u0, state == C.SLOT_NONFINITE, int(steps)))
            b.evict(s)
        return out
    finally:
        b.close()
        for g in grids:
            g.close()


def scan_populations(L, tau, speeds, prec="f32", transits=4.0, max_steps=40000, burst=100, stop_at_first=True):
    """Any tau: stored-population BGK cavities one after another (the scan stops
    at the first unstable speed).  Returns [(u0, unstable, steps)]."""
    from .grid import Grid
    out = []
    for u0 in speeds:
        flags, rho, jx, jy, per = I.cavity(L, u0)
        g = Grid(L, L, prec=prec, periodic=per, populations=True, tau=tau)
        try:
            g.set_geometry(flags, rho, jx, jy)
            h = horizon(L, u0, transits, max_steps=max_steps)
            done, bad = 0, False
            while done < h:
                k = min(burst, h - done)
                g.step(k)
                done += k
                if g.reduce(8)["nonfinite"] > 0:
                    bad = True
                    break
        finally:
            g.close()
        out.append((u0, bad, done))
        if bad and stop_at_first:
            break
    return out

"""Seeded synthetic workloads: node flags and initial moments.

These generators are shared by the GPU path, the benchmarks and the tests;
they hold none of the method's arithmetic (no equilibria, no update).  Every
array is numpy ``[ny, nx]`` with x fastest; flags use 0 FLUID, 1 SOLID,
2 FIXED.  Shapes follow the paper's workloads: the body-force channel of
section 3 (Poiseuille test), the lid-driven cavity of section 3 and
Appendix A, a random periodic field, and porous channels.
"""
import math

import numpy as np

FLUID, SOLID, FIXED = 0, 1, 2
PERIODIC_X, PERIODIC_Y = 1, 2
NU_TAU1 = 1.0 / 6.0   # lattice viscosity at tau = 1 (Eq. viscosity), used to size forces


def channel(nx, ny):
    """Channel of section 3: solid rows 0 and ny-1, periodic in x.  Returns (flags, periodic)."""
    flags = np.zeros((ny, nx), np.uint8)
    flags[0, :] = SOLID
    flags[-1, :] = SOLID
    return flags, PERIODIC_X


def cavity(L, u_lid, ny=None):
    """Lid-driven cavity (section 3, Appendix A): walls at x = 0, x = L-1 and y = 0,
    a FIXED lid row y = ny-1 moving at (u_lid, 0) with rho = 1, top corners solid.

    Returns (flags, rho, jx, jy, periodic=0).
    """
    nx = int(L)
    ny = nx if ny is None else int(ny)
    flags = np.zeros((ny, nx), np.uint8)
    flags[0, :] = SOLID
    flags[:, 0] = SOLID
    flags[:, -1] = SOLID
    flags[-1, 1:-1] = FIXED
    rho = np.ones((ny, nx))
    jx = np.zeros((ny, nx))
    jy = np.zeros((ny, nx))
    jx[-1, 1:-1] = u_lid          # rho = 1 on the lid, so momentum = velocity
    return flags, rho, jx, jy, 0


def random_periodic(nx, ny, seed=0, drho=1e-3, du=1e-2):
    """Random periodic field: g = default_rng(seed).standard_normal((3, ny, nx)) in the
    order (density deviation, ux, uy); rho = 1 + drho g0, u = du (g1, g2), j = rho u."""
    g = np.random.default_rng(seed).standard_normal((3, ny, nx))
    rho = 1.0 + drho * g[0]
    jx = rho * (du * g[1])
    jy = rho * (du * g[2])
    return rho, jx, jy


def random_state(nx, ny, rng, drho=1e-2, du=1e-2):
    """Small random perturbation of rest (for parity tests)."""
    rho = 1.0 + drho * rng.standard_normal((ny, nx))
    jx = rho * du * rng.standard_normal((ny, nx))
    jy = rho * du * rng.standard_normal((ny, nx))
    return rho, jx, jy


def random_obstacles(nx, ny, frac, rng):
    """Independent solid nodes with probability ``frac``."""
    return (rng.random((ny, nx)) < frac).astype(np.uint8)


def channel_force_for(u_max, ny):
    """Body force that gives a centre velocity u_max in an empty channel of height
    H = ny - 1 (Navier-Stokes channel: u_max = F H^2 / (8 nu))."""
    H = ny - 1
    return 8.0 * NU_TAU1 * u_max / (H * H)


def porous_channel(L, rng, r_lo=3.0, r_hi=12.0, porosity=0.8, max_tries=200000):
    """Channel with random non-overlapping disks (periodic in x), added one by one
    (random sequential addition) until the fluid fraction of the interior drops to
    ``porosity`` or below.

    Radii U[r_lo, r_hi], capped at L/8; disks keep one node of fluid between them.
    Returns (flags, periodic, achieved_porosity).
    """
    nx = ny = int(L)
    flags, periodic = channel(nx, ny)
    interior = (ny - 2) * nx
    r_hi = min(r_hi, L / 8.0)
    r_lo = min(r_lo, r_hi)
    cell = 2.0 * r_hi + 1.0                    # disks overlapping a candidate sit in adjacent cells
    ncx = max(1, int(nx // cell))
    cells = {}
    solid = 0
    tries = 0
    while solid < (1.0 - porosity) * interior and tries < max_tries:
        tries += 1
        r = rng.uniform(r_lo, r_hi)
        cx = rng.uniform(0, nx)
        cy = rng.uniform(1 + r, ny - 1 - r) if ny - 2 > 2 * r + 1 else (ny - 1) / 2.0
        gx, gy = int(cx / nx * ncx) % ncx, int(cy // cell)
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for (px, py, pr) in cells.get(((gx + dx) % ncx, gy + dy), ()):
                    ddx = abs(cx - px)
                    ddx = min(ddx, nx - ddx)   # periodic in x
                    if math.hypot(ddx, cy - py) < r + pr + 1.0:
                        ok = False
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            continue
        cells.setdefault((gx, gy), []).append((cx, cy, r))
        y0, y1 = max(1, int(math.floor(cy - r))), min(ny - 2, int(math.ceil(cy + r)))
        x0, x1 = int(math.floor(cx - r)), int(math.ceil(cx + r))
        yy, xx = np.mgrid[y0:y1 + 1, x0:x1 + 1]
        inside = (xx - cx) ** 2 + (yy - cy) ** 2 <= r * r
        xs = np.mod(xx[inside], nx)
        ys = yy[inside]
        newly = flags[ys, xs] != SOLID
        solid += int(newly.sum())
        flags[ys, xs] = SOLID
    return flags, periodic, 1.0 - solid / interior


def loguniform_int(rng, lo, hi, size=None):
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size))).astype(int)


def cavity_population(n=512, seed=4, lo=32, hi=512):
    """n cavities with side log-uniform on [lo, hi] and lid speed U[0.01, 0.1]."""
    rng = np.random.default_rng(seed)
    sizes = loguniform_int(rng, lo, hi, n)
    lids = rng.uniform(0.01, 0.1, n)
    return [(int(L), float(u)) for L, u in zip(sizes, lids)]


def request_stream(n=1000, seed=5, rate=1.0, lo=32, hi=2048, steps_lo=1e3, steps_hi=1e5):
    """Serving workload: Poisson arrivals (``rate`` per second), half cavities and half
    porous channels, square side log-uniform on [lo, hi], step budget log-uniform on
    [steps_lo, steps_hi].  Returns a list of dicts (geometry built lazily by ``build``)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    reqs = []
    for i in range(n):
        kind = "cavity" if rng.random() < 0.5 else "channel"
        L = int(loguniform_int(rng, lo, hi))
        steps = int(loguniform_int(rng, steps_lo, steps_hi))
        u = float(rng.uniform(0.01, 0.1))
        porosity = float(rng.uniform(0.6, 0.9))
        reqs.append(dict(id=i, arrival=float(t[i]), kind=kind, L=L, steps=steps, u=u,
                         porosity=porosity, seed=int(rng.integers(2 ** 31))))
    return reqs


def build_request(req):
    """(flags, rho, jx, jy, periodic, force) for a request of ``request_stream``."""
    L = req["L"]
    if req["kind"] == "cavity":
        flags, rho, jx, jy, periodic = cavity(L, req["u"])
        return flags, rho, jx, jy, periodic, (0.0, 0.0)
    flags, periodic, _ = porous_channel(L, np.random.default_rng(req["seed"]), porosity=req["porosity"])
    F = channel_force_for(req["u"], L)
    return flags, None, None, None, periodic, (F, 0.0)

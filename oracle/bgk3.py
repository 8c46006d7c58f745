"""Brute-force stored-population BGK on the 3-D lattices D3Q19 / D3Q27 --
TEST INFRASTRUCTURE ONLY.

The three-dimensional counterpart of ``bgk.BGK`` (section 2, Eq. lbm, with
the 3-D lattices of the memory analysis of section 4), written out with
Python loops for tiny grids: keep Q populations per node, relax them toward
the equilibrium with relaxation time tau, stream them; at tau = 1 its
moments must follow the moments-only 3-D step.  Conventions as ``bgk.BGK``:
flags 0 FLUID, 1 SOLID, 2 FIXED; velocity (j + tau F)/rho in the
equilibrium; wall "paper" returns w_k rho(x), "halfway" the relaxed
population reversed; a neighbour outside a non-periodic axis is a wall.
The lattice is built here from |e|^2 (its own enumeration, x outermost).
"""
import itertools

import numpy as np

FLUID, SOLID, FIXED = 0, 1, 2
WALL_PAPER, WALL_HALFWAY = 0, 1


def lattice(q):
    weights = {19: {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}, 27: {0: 8 / 27, 1: 2 / 27, 2: 1 / 54, 3: 1 / 216}}[q]
    e, w = [], []
    for v in itertools.product((-1, 0, 1), repeat=3):
        m = sum(c * c for c in v)
        if m in weights:
            e.append(v)
            w.append(weights[m])
    return e, w


class BGK3:
    def __init__(self, q, rho, jx, jy, jz, flags=None, periodic=0, force=(0.0, 0.0, 0.0),
                 wall=WALL_PAPER, tau=1.0):
        self.E, self.W = lattice(q)
        rho = np.array(rho, dtype=np.float64)
        self.nz, self.ny, self.nx = rho.shape
        self.flags = np.zeros(rho.shape, np.uint8) if flags is None else np.array(flags, np.uint8)
        self.periodic, self.F, self.wall, self.tau = int(periodic), tuple(map(float, force)), int(wall), float(tau)
        self.given = (rho.copy(), np.array(jx, float), np.array(jy, float), np.array(jz, float))
        self.f = self._feq(rho, self.given[1] / rho, self.given[2] / rho, self.given[3] / rho)

    def _feq(self, rho, ux, uy, uz):
        f = np.empty((len(self.E),) + rho.shape)
        usq = ux * ux + uy * uy + uz * uz
        for k, (a, b, c) in enumerate(self.E):
            eu = a * ux + b * uy + c * uz
            f[k] = self.W[k] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq)
        return f

    def _opposite(self, k):
        a, b, c = self.E[k]
        return self.E.index((-a, -b, -c))

    def _target(self, i, j, l, k):
        n = [i + self.E[k][0], j + self.E[k][1], l + self.E[k][2]]
        for ax, size in enumerate((self.nx, self.ny, self.nz)):
            if not 0 <= n[ax] < size:
                if not self.periodic & (1 << ax):
                    return None
                n[ax] %= size
        return n[2], n[1], n[0]

    def moments(self):
        rho = self.f.sum(axis=0)
        js = [sum(self.E[k][a] * self.f[k] for k in range(len(self.E))) for a in range(3)]
        keep = self.flags != FLUID
        out = [rho] + js
        for m, g in zip(out, self.given):
            m[keep] = g[keep]
        return tuple(out)

    def step(self):
        rho, jx, jy, jz = self.moments()
        safe = np.where(self.flags == SOLID, 1.0, rho)
        u = [(j + self.tau * F) / safe for j, F in zip((jx, jy, jz), self.F)]
        feq = self._feq(rho, *u)
        post = self.f - (self.f - feq) / self.tau
        fixed = self.flags == FIXED
        post[:, fixed] = feq[:, fixed]
        new = np.zeros_like(self.f)
        for l in range(self.nz):
            for j in range(self.ny):
                for i in range(self.nx):
                    if self.flags[l, j, i] == SOLID:
                        continue
                    for k in range(len(self.E)):
                        t = self._target(i, j, l, k)
                        if t is None or self.flags[t] == SOLID:
                            if self.flags[l, j, i] == FIXED:
                                continue
                            q = self._opposite(k)
                            new[q, l, j, i] = self.W[k] * rho[l, j, i] if self.wall == WALL_PAPER else post[k, l, j, i]
                        elif self.flags[t] == FIXED:
                            continue
                        else:
                            new[(k,) + t] = post[k, l, j, i]
        new[:, fixed] = feq[:, fixed]
        self.f = new

    def run(self, n):
        for _ in range(int(n)):
            self.step()
        return self.moments()

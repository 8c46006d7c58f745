"""Brute-force stored-population BGK lattice Boltzmann (D2Q9) -- TEST INFRASTRUCTURE ONLY.

This is the standard algorithm the paper starts from (section 2, Eq. lbm): keep
all nine populations f_k per node, relax them toward the equilibrium
(Eq. maxwellboltzmann) with relaxation time tau, then stream them to the
neighbours.  At tau = 1 the relaxed populations are exactly the equilibria
(Eq. LBMTau1), so this solver's density and momentum must follow the
moments-only step to rounding.  It is deliberately written without any of
the moments-only machinery, for tiny grids, with Python loops over links.

Conventions (the same problem statement as the moments-only oracle):
  * flags: 0 FLUID, 1 SOLID, 2 FIXED; a neighbour outside a non-periodic axis
    is a wall.
  * body force F: velocity used in the equilibrium is (j + tau F) / rho, which
    at tau = 1 is the momentum shift of the paper's algorithm.
  * wall "paper" (Eq. feqnoslip): the population that comes back to x from a
    wall link in direction k is the zero-velocity equilibrium w_k rho(x).
    (The paper states this rule for tau = 1 only; it is applied unchanged
    at other tau.)
  * wall "halfway": the relaxed population x sent into the wall comes back
    reversed (half-way bounce-back).
  * FIXED nodes hold their moments, emit the equilibrium of those moments
    every step and absorb whatever arrives.
"""
import numpy as np

# D2Q9 velocities, weights and inverse directions of section 2, written out here
# independently of the C oracle.
EX = (0, 1, 0, -1, 0, 1, -1, -1, 1)
EY = (0, 0, 1, 0, -1, 1, 1, -1, -1)
W = (4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36)
FLUID, SOLID, FIXED = 0, 1, 2
WALL_PAPER, WALL_HALFWAY = 0, 1


def opposite(k):
    """Direction with velocity -e_k, found by search (no table)."""
    for q in range(9):
        if EX[q] == -EX[k] and EY[q] == -EY[k]:
            return q
    raise AssertionError


def equilibrium(rho, ux, uy):
    """All nine equilibria, Eq. maxwellboltzmann, shape (9, ...)."""
    rho = np.asarray(rho, dtype=np.float64)
    f = np.empty((9,) + rho.shape)
    usq = ux * ux + uy * uy
    for k in range(9):
        eu = EX[k] * ux + EY[k] * uy
        f[k] = W[k] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq)
    return f


class BGK:
    """Stored-population D2Q9 BGK on an [ny, nx] grid."""

    def __init__(self, rho, jx, jy, flags=None, periodic=0, force=(0.0, 0.0),
                 wall=WALL_PAPER, tau=1.0):
        rho = np.array(rho, dtype=np.float64)
        self.ny, self.nx = rho.shape
        self.flags = (np.zeros(rho.shape, np.uint8) if flags is None
                      else np.array(flags, dtype=np.uint8))
        self.periodic = int(periodic)
        self.F = (float(force[0]), float(force[1]))
        self.wall = int(wall)
        self.tau = float(tau)
        jx = np.array(jx, dtype=np.float64)
        jy = np.array(jy, dtype=np.float64)
        # Any populations carrying these moments will do at tau = 1; the
        # equilibrium of the moments is used (at other tau this fixes the
        # non-equilibrium part to zero at t = 0).
        self.f = equilibrium(rho, jx / rho, jy / rho)
        fixed = self.flags == FIXED
        self.fixed_moments = (rho[fixed].copy(), jx[fixed].copy(), jy[fixed].copy())
        self._solid_rho = rho[self.flags == SOLID].copy()
        self._solid_j = (jx[self.flags == SOLID].copy(), jy[self.flags == SOLID].copy())

    def _target(self, i, j, k):
        ip, jp = i + EX[k], j + EY[k]
        if not 0 <= ip < self.nx:
            if not self.periodic & 1:
                return None
            ip %= self.nx
        if not 0 <= jp < self.ny:
            if not self.periodic & 2:
                return None
            jp %= self.ny
        return jp, ip

    def moments(self):
        """(rho, jx, jy) from the populations (Eq. rho1, Eq. u1); FIXED and SOLID
        nodes report the moments they were given."""
        rho = self.f.sum(axis=0)
        jx = sum(EX[k] * self.f[k] for k in range(9))
        jy = sum(EY[k] * self.f[k] for k in range(9))
        fixed = self.flags == FIXED
        rho[fixed], jx[fixed], jy[fixed] = self.fixed_moments
        solid = self.flags == SOLID
        rho[solid] = self._solid_rho
        jx[solid], jy[solid] = self._solid_j
        return rho, jx, jy

    def step(self):
        rho, jx, jy = self.moments()
        ux = (jx + self.tau * self.F[0]) / np.where(self.flags == SOLID, 1.0, rho)
        uy = (jy + self.tau * self.F[1]) / np.where(self.flags == SOLID, 1.0, rho)
        feq = equilibrium(rho, ux, uy)
        post = self.f - (self.f - feq) / self.tau          # Eq. lbm, collision
        fixed = self.flags == FIXED
        post[:, fixed] = feq[:, fixed]
        new = np.zeros_like(self.f)
        for j in range(self.ny):
            for i in range(self.nx):
                if self.flags[j, i] == SOLID:
                    continue
                for k in range(9):
                    t = self._target(i, j, k)
                    if t is None or self.flags[t] == SOLID:
                        if self.flags[j, i] == FIXED:
                            continue
                        q = opposite(k)
                        if self.wall == WALL_PAPER:
                            new[q, j, i] = W[k] * rho[j, i]
                        else:
                            new[q, j, i] = post[k, j, i]
                    elif self.flags[t] == FIXED:
                        continue
                    else:
                        new[k][t] = post[k, j, i]               # Eq. lbm, streaming
        new[:, fixed] = feq[:, fixed]
        self.f = new

    def run(self, nsteps):
        for _ in range(int(nsteps)):
            self.step()
        return self.moments()

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
  * multiphase (``sc=(G, rho0)``): the Shan-Chen force of the paper's
    Eq. f_sc, -G psi(x) sum_k w_k psi(x + e_k) e_k with psi(rho) =
    rho0 (1 - exp(-rho / rho0)), is added to F at every non-solid node; a
    solid neighbour contributes the psi of its given density, a neighbour
    outside a non-periodic axis that of the node itself.
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
                 wall=WALL_PAPER, tau=1.0, sc=None):
        rho = np.array(rho, dtype=np.float64)
        self.ny, self.nx = rho.shape
        self.flags = (np.zeros(rho.shape, np.uint8) if flags is None
                      else np.array(flags, dtype=np.uint8))
        self.periodic = int(periodic)
        self.F = (float(force[0]), float(force[1]))
        self.wall = int(wall)
        self.tau = float(tau)
        self.sc = None if sc is None else (float(sc[0]), float(sc[1]))
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

    def _psi(self, rho):
        G, rho0 = self.sc
        return rho0 * (1.0 - np.exp(-rho / rho0))

    def _sc_force_loops(self, rho):
        """Per-node Shan-Chen force, written with loops over nodes and links."""
        G, _ = self.sc
        psi = self._psi(rho)
        FX = np.zeros(rho.shape)
        FY = np.zeros(rho.shape)
        for j in range(self.ny):
            for i in range(self.nx):
                if self.flags[j, i] == SOLID:
                    continue
                sx = sy = 0.0
                for k in range(1, 9):
                    t = self._target(i, j, k)
                    p = psi[j, i] if t is None else psi[t]
                    sx += W[k] * p * EX[k]
                    sy += W[k] * p * EY[k]
                FX[j, i] = -G * psi[j, i] * sx
                FY[j, i] = -G * psi[j, i] * sy
        return FX, FY

    def _force(self, rho, arrays):
        """Uniform force plus, for multiphase runs, the Shan-Chen force."""
        fx = np.full(rho.shape, self.F[0])
        fy = np.full(rho.shape, self.F[1])
        if self.sc is not None:
            FX, FY = self._sc_force_arrays(rho) if arrays else self._sc_force_loops(rho)
            fx = fx + FX
            fy = fy + FY
        return fx, fy

    def step(self):
        rho, jx, jy = self.moments()
        fx, fy = self._force(rho, arrays=False)
        ux = (jx + self.tau * fx) / np.where(self.flags == SOLID, 1.0, rho)
        uy = (jy + self.tau * fy) / np.where(self.flags == SOLID, 1.0, rho)
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

    # ------------------------------------------------------------- array form
    # The same push step written with whole-array operations, for grids too
    # large for the loops above: the link lists are built once from the same
    # neighbour rule, and every population takes the same arithmetic, so the
    # two forms agree bit for bit (tested).
    def _link_lists(self):
        if getattr(self, "_links", None) is not None:
            return self._links
        ny, nx = self.ny, self.nx
        jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        src_ok = self.flags != SOLID
        links = []
        for k in range(9):
            ip, jp = ii + EX[k], jj + EY[k]
            inside = np.ones((ny, nx), bool)
            if self.periodic & 1:
                ip = ip % nx
            else:
                inside &= (ip >= 0) & (ip < nx)
            if self.periodic & 2:
                jp = jp % ny
            else:
                inside &= (jp >= 0) & (jp < ny)
            ipc, jpc = np.clip(ip, 0, nx - 1), np.clip(jp, 0, ny - 1)
            tflag = np.where(inside, self.flags[jpc, ipc], SOLID)
            stream = src_ok & (tflag != SOLID) & (tflag != FIXED)
            bounce = (self.flags == FLUID) & (tflag == SOLID)
            s_idx = (jj * nx + ii)[stream]
            t_idx = (jpc * nx + ipc)[stream]
            b_idx = (jj * nx + ii)[bounce]
            links.append((s_idx, t_idx, b_idx))
        self._links = links
        return links

    def _sc_force_arrays(self, rho):
        G, _ = self.sc
        psi = self._psi(rho)
        ny, nx = self.ny, self.nx
        jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        sx = np.zeros(rho.shape)
        sy = np.zeros(rho.shape)
        for k in range(1, 9):
            ip, jp = ii + EX[k], jj + EY[k]
            inside = np.ones((ny, nx), bool)
            if self.periodic & 1:
                ip = ip % nx
            else:
                inside &= (ip >= 0) & (ip < nx)
            if self.periodic & 2:
                jp = jp % ny
            else:
                inside &= (jp >= 0) & (jp < ny)
            p = np.where(inside, psi[np.clip(jp, 0, ny - 1), np.clip(ip, 0, nx - 1)], psi)
            sx = sx + W[k] * p * EX[k]
            sy = sy + W[k] * p * EY[k]
        solid = self.flags == SOLID
        FX = np.where(solid, 0.0, -G * psi * sx)
        FY = np.where(solid, 0.0, -G * psi * sy)
        return FX, FY

    def step_arrays(self):
        rho, jx, jy = self.moments()
        fx, fy = self._force(rho, arrays=True)
        ux = (jx + self.tau * fx) / np.where(self.flags == SOLID, 1.0, rho)
        uy = (jy + self.tau * fy) / np.where(self.flags == SOLID, 1.0, rho)
        feq = equilibrium(rho, ux, uy)
        post = self.f - (self.f - feq) / self.tau
        fixed = self.flags == FIXED
        post[:, fixed] = feq[:, fixed]
        new = np.zeros_like(self.f)
        rflat = rho.reshape(-1)
        for k, (s_idx, t_idx, b_idx) in enumerate(self._link_lists()):
            pk = post[k].reshape(-1)
            new[k].reshape(-1)[t_idx] = pk[s_idx]
            q = opposite(k)
            if self.wall == WALL_PAPER:
                new[q].reshape(-1)[b_idx] = W[k] * rflat[b_idx]
            else:
                new[q].reshape(-1)[b_idx] = pk[b_idx]
        new[:, fixed] = feq[:, fixed]
        self.f = new

    def run(self, nsteps, arrays=False):
        for _ in range(int(nsteps)):
            if arrays:
                self.step_arrays()
            else:
                self.step()
        return self.moments()


def shear_mode(tau, kappa):
    """Linear theory of the BGK step around rest (rho = 1, u = 0) for a wave
    exp(i kappa y): the one-step operator is streaming S = diag(exp(-i kappa e_y))
    after the linearised collision I - (I - E) / tau, with E the linearised
    equilibrium (E f)_k = w_k (sum f + 3 e_k . sum e f).  Returns the eigenvalue
    and eigenvector of the shear mode (the one carrying x-momentum), the
    eigenvector scaled to unit x-momentum.  Test infrastructure: pins the BGK
    oracle at tau != 1 and, as kappa -> 0, the viscosity (tau - 1/2) / 3 of
    section 2 (Eq. viscosity)."""
    E = np.array([[W[k] * (1.0 + 3.0 * (EX[k] * EX[q] + EY[k] * EY[q])) for q in range(9)] for k in range(9)])
    Cop = np.eye(9) - (np.eye(9) - E) / tau
    S = np.diag([np.exp(-1j * kappa * EY[k]) for k in range(9)])
    lam, vec = np.linalg.eig(S @ Cop)
    ex = np.array(EX, dtype=float)
    jx = ex @ vec
    best = int(np.argmax(np.abs(jx) / np.linalg.norm(vec, axis=0)))
    v = vec[:, best] / jx[best]
    return lam[best], v

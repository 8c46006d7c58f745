"""Closed forms that pin the oracle -- TEST INFRASTRUCTURE ONLY.

Derived from the paper's rules, not from the oracle's code.

One-dimensional reduction (x-independent flow, v = 0, rho = 1): group the nine
D2Q9 directions by their y velocity.  Each group's share of density and
x momentum follows from Eq. maxwellboltzmann with the |u|^2 terms cancelling
inside the group:
    e_y =  0 : density 2/3 rho, x momentum 2/3 J
    e_y = +1 : density 1/6 rho, x momentum 1/6 J, y momentum +1/6 rho
    e_y = -1 : density 1/6 rho, x momentum 1/6 J, y momentum -1/6 rho
where J = j + F is the forced momentum of the emitting row (Algorithm 1).
So a fluid row updates as j'(y) = 2/3 J(y) + 1/6 J(y-1) + 1/6 J(y+1).  A wall
row next to y supplies, through Eq. feqnoslip, density rho(y)/6 and no x
momentum; under half-way bounce-back it returns the row's own group,
x momentum -J(y)/6.

Steady channel flow then satisfies a three-point recurrence whose solution is a
parabola: with the paper's wall rule the forced momentum vanishes exactly on
the solid rows (walls on rows 0 and H = ny - 1); with half-way bounce-back the
walls sit half a node outside the last fluid rows.  The viscosity is 1/6
(Eq. viscosity at tau = 1), so the analytic profile F y (H - y) / (2 nu) is
3 F y (H - y).
"""
import math

import numpy as np


def poiseuille_ueq_paper(ny, F):
    """Steady equilibrium velocity u_eq = (j + F) / rho on rows 0..ny-1, paper wall rule.

    Walls on rows 0 and ny-1; u_eq(y) = 3 F y (H - y), H = ny - 1 (zero on the walls).
    """
    H = ny - 1
    y = np.arange(ny, dtype=np.float64)
    return 3.0 * F * y * (H - y)


def poiseuille_ueq_halfway(ny, F):
    """Steady u_eq on rows 0..ny-1 under half-way bounce-back (wall rows returned as 0).

    N = ny - 2 fluid rows; u_eq(y) = 3 F [(y - 1/2)(N + 1/2 - y) + 1/4] for y = 1..N.
    """
    N = ny - 2
    y = np.arange(ny, dtype=np.float64)
    u = 3.0 * F * ((y - 0.5) * (N + 0.5 - y) + 0.25)
    u[0] = 0.0
    u[-1] = 0.0
    return u


def poiseuille_analytic(ny, F):
    """Navier-Stokes channel profile with walls on rows 0 and ny-1, nu = 1/6."""
    H = ny - 1
    y = np.arange(ny, dtype=np.float64)
    nu = 1.0 / 6.0
    return F * y * (H - y) / (2.0 * nu)


def centre_error_percent_paper(ny):
    """Percent error of the measured centre velocity j/rho under the paper's wall rule.

    Measured velocity is u_eq - F (rho = 1), the analytic centre value 3 F H^2 / 4,
    so e = 100 F / (3 F H^2 / 4) = 400 / (3 H^2): the L^-2 law of section 3.
    """
    H = ny - 1
    return 100.0 * 4.0 / (3.0 * H * H)


def shear_wave_factor(kwave):
    """Per-step amplitude factor of a periodic shear wave jx ~ sin(k y): (2 + cos k) / 3."""
    return (2.0 + math.cos(kwave)) / 3.0


def channel_1d(ny, F, wall, nsteps, j0=None):
    """Exact one-dimensional recurrence for x-independent channel flow (rho = 1, v = 0).

    Rows 0 and ny-1 are walls; ``wall`` 0 = paper rule, 1 = half-way bounce-back.
    Returns j_x on rows 0..ny-1 after ``nsteps`` (wall rows 0).
    """
    j = np.zeros(ny) if j0 is None else np.array(j0, dtype=np.float64)
    j[0] = j[-1] = 0.0
    for _ in range(int(nsteps)):
        J = j + F
        new = np.zeros(ny)
        for y in range(1, ny - 1):
            below = J[y - 1] if y - 1 > 0 else (0.0 if wall == 0 else -J[y])
            above = J[y + 1] if y + 1 < ny - 1 else (0.0 if wall == 0 else -J[y])
            new[y] = (2.0 / 3.0) * J[y] + (1.0 / 6.0) * below + (1.0 / 6.0) * above
        j = new
    return j


def memory_standard(Q, Nf, c):
    """Eq. lbmmemory: bytes per node of the two-lattice (AB) standard LBM."""
    return (2 * Q + Nf) * c


def memory_lbmtau1(Nf, c):
    """Eq. LBMTau1memory: bytes per node of LBMTau1 (two copies of the moments)."""
    return 2 * Nf * c


def reynolds_max_tau1(L):
    """Empirical stability fit at tau = 1 (caption of the Re_max figure): 12 L^0.8."""
    return 12.0 * L ** 0.8

"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test names the passage it follows.  None of them re-types the oracle's
update: the expected values come from exact rational arithmetic, closed-form
solutions, conservation laws, the independent brute-force BGK solver, or the
paper's worked example and printed numbers (``tests/golden``).

P1  equilibrium and lattice tables    -- exact moment identities (section 2)
P2  uniform state / force             -- fixed point, j_n = j_0 + n F
P3  shear wave                        -- exact decay (2 + cos k)/3 per step
P4  full 2-D step                     -- brute-force BGK at tau = 1 (Eq. lbm vs Eq. LBMTau1)
P5  channel flow                      -- steady parabola, L^-2 error law, 1-D recurrence
P6  paper wall rule mass budget       -- exact leak identity
P7  periodic conservation             -- mass, momentum + N F
P8  north-wall worked example         -- tests/golden/north_wall.txt
P9  memory formulas                   -- tests/golden/memory_example.txt
P10 stored-population BGK, any tau    -- array form = loop form; linear theory of the
                                         shear mode (9 x 9 eigenproblem); viscosity
                                         (tau - 1/2)/3; exact steady parabola; conservation
P11 multiphase (Shan-Chen force)       -- brute-force BGK with the force at tau = 1; pair
                                         antisymmetry (momentum conserved); flat-interface
                                         coexistence against the mechanical-stability
                                         integral; Laplace law; G = 0 is the plain step
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import bgk
from oracle import closed_forms as cf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EPS = np.finfo(np.float64).eps


def _rng(seed):
    return np.random.default_rng(seed)


def _random_state(rng, ny, nx, drho=1e-2, du=1e-2):
    rho = 1.0 + drho * rng.standard_normal((ny, nx))
    jx = rho * du * rng.standard_normal((ny, nx))
    jy = rho * du * rng.standard_normal((ny, nx))
    return rho, jx, jy


# ----------------------------------------------------------------- P1 tables, f^eq
def test_p1_tables_are_d2q9():
    ex, ey, inv, w = oracle.tables()
    # velocity set printed in section 2, k = 0..8
    assert list(zip(ex, ey)) == [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1),
                                 (1, 1), (-1, 1), (-1, -1), (1, -1)]
    exact = [Fraction(w_).limit_denominator(100) for w_ in w]
    assert exact == [Fraction(4, 9)] + [Fraction(1, 9)] * 4 + [Fraction(1, 36)] * 4
    assert sum(exact) == 1
    for k in range(9):
        assert (ex[inv[k]], ey[inv[k]]) == (-ex[k], -ey[k])
        assert w[inv[k]] == w[k]
        assert inv[inv[k]] == k
    # lattice isotropy: sum w e_a e_b = delta_ab / 3 (c_s^2 = 1/3, Eq. viscosity)
    assert sum(e * e * q for e, q in zip(ex, exact)) == Fraction(1, 3)
    assert sum(a * b * q for a, b, q in zip(ex, ey, exact)) == 0


def test_p1_equilibrium_moments_exact_rational():
    """sum f = rho, sum e f = rho u, sum e e f = rho/3 I + rho u u, in exact arithmetic."""
    ex, ey, _, w = oracle.tables()
    wq = [Fraction(x).limit_denominator(100) for x in w]
    rho, u, v = Fraction(7, 5), Fraction(3, 50), Fraction(-2, 25)

    def feq(k):
        eu = ex[k] * u + ey[k] * v
        return wq[k] * rho * (1 - Fraction(3, 2) * (u * u + v * v) + 3 * eu + Fraction(9, 2) * eu * eu)

    f = [feq(k) for k in range(9)]
    assert sum(f) == rho
    assert sum(ex[k] * f[k] for k in range(9)) == rho * u
    assert sum(ey[k] * f[k] for k in range(9)) == rho * v
    assert sum(ex[k] ** 2 * f[k] for k in range(9)) == rho / 3 + rho * u * u
    assert sum(ey[k] ** 2 * f[k] for k in range(9)) == rho / 3 + rho * v * v
    assert sum(ex[k] * ey[k] * f[k] for k in range(9)) == rho * u * v
    # and the oracle's floating-point f^eq is the same function
    for k in range(9):
        assert oracle.feq(k, float(rho), float(u), float(v)) == pytest.approx(float(f[k]), rel=4 * EPS, abs=0)


# ----------------------------------------------------------------- P2 uniform state
@pytest.mark.parametrize("wall", [0, 1])
def test_p2_uniform_state_fixed_point_and_force(wall):
    ny, nx = 6, 5
    rho = np.full((ny, nx), 1.25)
    jx = np.full((ny, nx), 0.03)
    jy = np.full((ny, nx), -0.02)
    r, u, v = oracle.run(rho, jx, jy, 10, periodic=3, wall=wall)
    assert np.allclose(r, rho, rtol=20 * EPS, atol=0)
    assert np.allclose(u, jx, rtol=0, atol=40 * EPS)
    assert np.allclose(v, jy, rtol=0, atol=40 * EPS)
    F = (2.5e-5, -1e-5)
    r, u, v = oracle.run(rho, jx, jy, 10, periodic=3, force=F, wall=wall)
    assert np.abs(r - rho).max() < 1e-15
    assert np.abs(u - (jx + 10 * F[0])).max() < 1e-16
    assert np.abs(v - (jy + 10 * F[1])).max() < 1e-16


# ----------------------------------------------------------------- P3 shear wave
@pytest.mark.parametrize("A", [1e-3, 0.1])
@pytest.mark.parametrize("m", [1, 3])
def test_p3_shear_wave_exact_decay(A, m):
    """x-independent jx = A sin(k y): all |u|^2 terms cancel, so it decays by (2 + cos k)/3."""
    ny, nx, n = 24, 4, 50
    kwave = 2 * math.pi * m / ny
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    rho = np.ones((ny, nx))
    jx = A * np.sin(kwave * y)
    r, u, v = oracle.run(rho, jx, np.zeros((ny, nx)), n, periodic=3)
    lam = cf.shear_wave_factor(kwave)
    assert np.abs(u - A * lam ** n * np.sin(kwave * y)).max() < 1e-15 * max(1.0, A * 10)
    assert np.abs(r - 1).max() < 1e-14
    assert np.abs(v).max() < 1e-15
    # the transposed wave tests the other axis
    r, u, v = oracle.run(rho.T.copy(), np.zeros((nx, ny)), jx.T.copy(), n, periodic=3)
    assert np.abs(v - A * lam ** n * np.sin(kwave * y.T)).max() < 1e-15 * max(1.0, A * 10)
    assert np.abs(u).max() < 1e-15


def test_p3_small_k_viscosity_is_one_sixth():
    """(2 + cos k)/3 = 1 - k^2/6 + O(k^4): diffusion with nu = c_s^2 (tau - 1/2) = 1/6."""
    ny, nx, n = 256, 3, 20
    kwave = 2 * math.pi / ny
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    _, u, _ = oracle.run(np.ones((ny, nx)), 1e-4 * np.sin(kwave * y), np.zeros((ny, nx)), n, periodic=3)
    lam = (np.abs(u).max() / 1e-4) ** (1.0 / n)
    nu = (1 - lam) / kwave ** 2
    assert nu == pytest.approx(1.0 / 6.0, rel=1e-3)


# ----------------------------------------------------------------- P4 brute-force BGK
def _cavity_flags(ny, nx, obstacle=True):
    flags = np.zeros((ny, nx), np.uint8)
    flags[0, :] = oracle.SOLID
    flags[:, 0] = oracle.SOLID
    flags[:, -1] = oracle.SOLID
    flags[-1, 1:-1] = oracle.FIXED
    if obstacle:
        flags[ny // 2, nx // 2] = oracle.SOLID
    return flags


@pytest.mark.parametrize("wall", [0, 1])
def test_p4_bgk_tau1_equals_moments_only(wall):
    rng = _rng(4)
    ny, nx = 7, 9
    flags = _cavity_flags(ny, nx)
    rho, jx, jy = _random_state(rng, ny, nx)
    F = (1e-3, -2e-3)
    ref = bgk.BGK(rho, jx, jy, flags, periodic=0, force=F, wall=wall)
    r, u, v = rho, jx, jy
    worst = 0.0
    for _ in range(200):
        ref.step()
        r, u, v = oracle.step(r, u, v, flags, 0, F, wall)
        br, bu, bv = ref.moments()
        worst = max(worst, np.abs(br - r).max(), np.abs(bu - u).max(), np.abs(bv - v).max())
    assert worst < 5e-15


@pytest.mark.parametrize("periodic", [1, 2, 3])
@pytest.mark.parametrize("wall", [0, 1])
def test_p4_bgk_tau1_periodic_axes_and_obstacles(periodic, wall):
    rng = _rng(10 + periodic)
    ny, nx = 6, 7
    flags = (rng.random((ny, nx)) < 0.2).astype(np.uint8)
    rho, jx, jy = _random_state(rng, ny, nx)
    F = (3e-4, 1e-4)
    ref = bgk.BGK(rho, jx, jy, flags, periodic=periodic, force=F, wall=wall)
    br, bu, bv = ref.run(60)
    r, u, v = oracle.run(rho, jx, jy, 60, flags, periodic, F, wall)
    assert max(np.abs(br - r).max(), np.abs(bu - u).max(), np.abs(bv - v).max()) < 5e-15


def test_p4_wall_rules_differ():
    """The two wall readings are different operators (guards against a rule being ignored)."""
    rng = _rng(5)
    flags = _cavity_flags(7, 9)
    rho, jx, jy = _random_state(rng, 7, 9)
    a = oracle.step(rho, jx, jy, flags, 0, (0, 0), 0)
    b = oracle.step(rho, jx, jy, flags, 0, (0, 0), 1)
    assert np.abs(a[1] - b[1]).max() > 1e-4


# ----------------------------------------------------------------- P5 channel flow
@pytest.mark.parametrize("ny", [5, 8, 16, 33])
@pytest.mark.parametrize("wall", [0, 1])
def test_p5_poiseuille_closed_form_is_fixed_point(ny, wall):
    nx, F = 4, 2.5e-5
    flags = np.zeros((ny, nx), np.uint8)
    flags[0] = flags[-1] = oracle.SOLID
    ueq = cf.poiseuille_ueq_paper(ny, F) if wall == 0 else cf.poiseuille_ueq_halfway(ny, F)
    jx = np.repeat((ueq - F)[:, None], nx, axis=1)
    jx[0] = jx[-1] = 0.0
    rho = np.ones((ny, nx))
    r, u, v = oracle.step(rho, jx, np.zeros((ny, nx)), flags, 1, (F, 0), wall)
    assert np.abs(u - jx)[1:-1].max() < 1e-12 * ueq.max()
    assert np.abs(r - 1).max() < 4 * EPS
    assert np.abs(v).max() < 4 * EPS      # rho/6 - rho/6 up to rounding


@pytest.mark.parametrize("wall", [0, 1])
def test_p5_channel_from_rest_matches_1d_recurrence_and_converges(wall):
    """The 64 x 32 channel (periodic x, walls on rows 0 and 31, F = 1e-6) run 10,000 steps."""
    ny, nx, F, n = 32, 64, 1e-6, 10000
    flags = np.zeros((ny, nx), np.uint8)
    flags[0] = flags[-1] = oracle.SOLID
    r, u, v = oracle.run(np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)), n, flags, 1, (F, 0), wall)
    j1 = cf.channel_1d(ny, F, wall, n)
    assert np.abs(u - j1[:, None])[1:-1].max() < 1e-12 * np.abs(j1).max()
    assert np.abs(u - u[:, :1]).max() < 1e-18                      # x-independent
    ueq = cf.poiseuille_ueq_paper(ny, F) if wall == 0 else cf.poiseuille_ueq_halfway(ny, F)
    # slowest mode decays as ((2 + cos(pi/31))/3)^n; after 10,000 steps ~3.7e-8 of u_max remains
    assert np.abs((u + F) - ueq[:, None])[1:-1].max() < 1e-7 * ueq.max()


def test_p5_error_scales_as_inverse_square_of_size():
    """Section 3: the centre-velocity error falls as L^-2; here with the exact prefactor 400/(3 H^2)."""
    F = 2.5e-5
    errs = []
    for ny in (17, 25, 33, 49):
        H = ny - 1
        flags = np.zeros((ny, 3), np.uint8)
        flags[0] = flags[-1] = oracle.SOLID
        ueq = cf.poiseuille_ueq_paper(ny, F)
        # start near the steady state and relax the remaining rounding with a few steps
        jx = np.repeat((ueq - F)[:, None], 3, axis=1)
        jx[0] = jx[-1] = 0.0
        r, u, _ = oracle.run(np.ones((ny, 3)), jx, np.zeros((ny, 3)), 200, flags, 1, (F, 0), 0)
        c = H // 2
        measured = u[c, 0] / r[c, 0]
        exact = cf.poiseuille_analytic(ny, F)[c]
        e = 100 * abs(measured - exact) / abs(exact)
        assert e == pytest.approx(cf.centre_error_percent_paper(ny), rel=1e-8)
        errs.append((H, e))
    slope = np.polyfit(np.log([h for h, _ in errs]), np.log([e for _, e in errs]), 1)[0]
    assert slope == pytest.approx(-2.0, abs=1e-6)
    # the 200 x 100 channel of section 3: 400 / (3 * 99^2) percent
    assert cf.centre_error_percent_paper(100) == pytest.approx(0.0136041, rel=1e-5)


# ----------------------------------------------------------------- P6 paper wall rule mass budget
def test_p6_paper_wall_mass_leak_identity():
    """Under Eq. feqnoslip a wall link returns w_k rho(x) instead of the f^eq_k(x) it received,
    so the mass changes by sum over wall links of (w_k rho(x) - f^eq_k(x)); half-way keeps it."""
    rng = _rng(6)
    ny, nx = 8, 10
    flags = np.zeros((ny, nx), np.uint8)
    flags[0] = flags[-1] = oracle.SOLID
    flags[:, 0] = flags[:, -1] = oracle.SOLID
    flags[3, 4] = flags[4, 6] = oracle.SOLID
    rho, jx, jy = _random_state(rng, ny, nx, 1e-2, 3e-2)
    F = (1e-4, 2e-4)
    fluid = flags == oracle.FLUID
    for _ in range(30):
        leak = 0.0
        feq = bgk.equilibrium(rho, (jx + F[0]) / rho, (jy + F[1]) / rho)
        for j in range(ny):
            for i in range(nx):
                if not fluid[j, i]:
                    continue
                for k in range(1, 9):
                    if flags[j + bgk.EY[k], i + bgk.EX[k]] == oracle.SOLID:
                        leak += bgk.W[k] * rho[j, i] - feq[k, j, i]
        m0 = rho[fluid].sum()
        rho, jx, jy = oracle.step(rho, jx, jy, flags, 0, F, 0)
        assert rho[fluid].sum() - m0 == pytest.approx(leak, abs=1e-13)   # leak itself ~1e-4
    rho, jx, jy = _random_state(rng, ny, nx, 1e-2, 3e-2)
    m0 = rho[fluid].sum()
    r, _, _ = oracle.run(rho, jx, jy, 30, flags, 0, F, 1)
    assert abs(r[fluid].sum() - m0) / m0 < 8 * EPS * 30


# ----------------------------------------------------------------- P7 periodic conservation
@pytest.mark.parametrize("wall", [0, 1])
def test_p7_periodic_conservation(wall):
    rng = _rng(7)
    ny, nx, n = 12, 10, 40
    rho, jx, jy = _random_state(rng, ny, nx)
    F = (2e-5, -3e-5)
    r, u, v = oracle.run(rho, jx, jy, n, None, 3, F, wall)
    N = ny * nx
    m0 = rho.sum()
    assert abs(r.sum() - m0) / m0 < 8 * EPS * n
    assert u.sum() == pytest.approx(jx.sum() + n * N * F[0], abs=1e-12)
    assert v.sum() == pytest.approx(jy.sum() + n * N * F[1], abs=1e-12)


def test_p7_halfway_obstacles_conserve_mass():
    rng = _rng(8)
    ny, nx, n = 12, 10, 40
    flags = (rng.random((ny, nx)) < 0.25).astype(np.uint8)
    rho, jx, jy = _random_state(rng, ny, nx)
    fluid = flags == 0
    r, _, _ = oracle.run(rho, jx, jy, n, flags, 3, (1e-4, 0), 1)
    assert abs(r[fluid].sum() - rho[fluid].sum()) / rho[fluid].sum() < 8 * EPS * n


# ----------------------------------------------------------------- P8 north-wall worked example
def _read_north_wall():
    terms = []
    with open(os.path.join(GOLDEN, "north_wall.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                kind, dx, dy, k = line.split()[:4]
                terms.append((kind, int(dx), int(dy), int(k)))
    return terms


@pytest.mark.parametrize("F", [(0.0, 0.0), (1e-3, 2e-3)])
def test_p8_north_wall_worked_example(F):
    terms = _read_north_wall()
    assert len(terms) == 9
    rng = _rng(9)
    ny, nx = 4, 5
    flags = np.zeros((ny, nx), np.uint8)
    flags[3, :] = oracle.SOLID          # the north wall
    flags[0, :] = oracle.SOLID
    rho, jx, jy = _random_state(rng, ny, nx, 5e-2, 5e-2)
    X, Y = 2, 2
    r, u, v = oracle.step(rho, jx, jy, flags, 1, F, 0)

    def q(x):
        return Fraction(float(x))

    def feq(k, j, i):
        rr = q(rho[j, i])
        ux = (q(jx[j, i]) + q(F[0])) / rr
        uy = (q(jy[j, i]) + q(F[1])) / rr
        eu = bgk.EX[k] * ux + bgk.EY[k] * uy
        w = Fraction(bgk.W[k]).limit_denominator(100)
        return w * rr * (1 - Fraction(3, 2) * (ux * ux + uy * uy) + 3 * eu + Fraction(9, 2) * eu * eu)

    R = Jx = Jy = Fraction(0)
    for kind, dx, dy, k in terms:
        if kind == "wall":
            val = Fraction(bgk.W[k]).limit_denominator(100) * q(rho[Y, X])
            arrive = bgk.opposite(k)
        else:
            val = feq(k, Y + dy, X + dx)
            arrive = k
        R += val
        Jx += bgk.EX[arrive] * val
        Jy += bgk.EY[arrive] * val
    assert r[Y, X] == pytest.approx(float(R), rel=1e-15, abs=1e-15)
    assert u[Y, X] == pytest.approx(float(Jx), abs=1e-15)
    assert v[Y, X] == pytest.approx(float(Jy), abs=1e-15)


# ----------------------------------------------------------------- P9 memory formulas
def test_p9_memory_example_of_the_paper():
    vals = {}
    with open(os.path.join(GOLDEN, "memory_example.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                key, val = line.split()
                vals[key] = float(val)
    n = int(vals["nodes"])
    assert cf.memory_standard(9, 3, 4) == 21 * 4
    assert cf.memory_lbmtau1(3, 4) == 6 * 4
    assert n * cf.memory_standard(9, 3, 4) == vals["bytes_standard"]
    assert n * cf.memory_lbmtau1(3, 4) == vals["bytes_lbmtau1"]
    assert 1 - cf.memory_lbmtau1(3, 4) / cf.memory_standard(9, 3, 4) == pytest.approx(
        vals["saving_d2q9_from_counts"], rel=1e-15)
    # D3Q27: N_f = 4
    assert 1 - cf.memory_lbmtau1(4, 4) / cf.memory_standard(27, 4, 4) == pytest.approx(
        vals["saving_d3q27_approx"], abs=0.005)


# ----------------------------------------------------------------- reductions
# The diagnostics of section 3 (velocity change between two times, mass) are
# pinned by states whose sums and velocity changes are known in closed form,
# not by re-deriving the sums.
@pytest.mark.parametrize("rho0", [1.0, 1.75])
@pytest.mark.parametrize("axis", ["x", "y"])
def test_reduce_residual_of_the_shear_wave(rho0, axis):
    """A shear wave j = rho0 A sin(k y) e_x on a uniform density rho0 decays exactly
    by (2 + cos k)/3 per step (P3; the group shares of Appendix A.1 do not depend on
    rho).  So the velocity u = j / rho changes between steps t - 100 and t by
    A lam^(t - 100) (1 - lam^100) sin(k y), and the residual is that amplitude times
    max_y |sin(k y)|.  rho0 != 1 separates u = j / rho from j; the transposed wave
    (a y momentum varying along x) pins the second component."""
    ny, nx, A, m, t0 = 12, 5, 0.05, 2, 7
    kwave = 2 * math.pi * m / ny
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    rho = np.full((ny, nx), rho0)
    jw = rho0 * A * np.sin(kwave * y)
    zero = np.zeros((ny, nx))
    state = (rho, jw, zero) if axis == "x" else (rho.T.copy(), zero.T.copy(), jw.T.copy())
    snap = oracle.run(*state, t0, None, 3)
    cur = oracle.run(*snap, 100, None, 3)
    lam = cf.shear_wave_factor(kwave)
    smax = max(abs(math.sin(kwave * yy)) for yy in range(ny))       # sin(pi/3) here
    expect = A * lam ** t0 * (1 - lam ** 100) * smax
    d = oracle.reduce(*cur, None, snap)
    assert d["residual"] == pytest.approx(expect, rel=1e-12)
    assert d["fluid"] == ny * nx and d["nonfinite"] == 0
    # momentum of a sine over whole periods is zero; periodic mass is rho0 N exactly
    assert d["mass"] == pytest.approx(rho0 * ny * nx, rel=1e-14)
    assert abs(d["mom_x"]) < 1e-13 and abs(d["mom_y"]) < 1e-13     # N eps rounding of the sums
    # against itself the residual is exactly zero
    assert oracle.reduce(*cur, None, cur)["residual"] == 0.0


def test_reduce_residual_against_a_snapshot_of_another_density():
    """Uniform periodic flow under a force (P2): rho stays rho0 and j_n = j_0 + n F, so
    u_n = (j_0 + n F) / rho0.  Against a uniform snapshot of density 1.5 and velocity
    u_s (momentum 1.5 u_s) the residual is max(|u_n - u_s|) over both components."""
    ny, nx, n, rho0 = 6, 5, 10, 1.25
    j0, F, us = (0.03, -0.02), (2.5e-5, -1e-5), (0.01, 0.004)
    state = (np.full((ny, nx), rho0), np.full((ny, nx), j0[0]), np.full((ny, nx), j0[1]))
    cur = oracle.run(*state, n, None, 3, F)
    snap = (np.full((ny, nx), 1.5), np.full((ny, nx), 1.5 * us[0]), np.full((ny, nx), 1.5 * us[1]))
    expect = max(abs((j0[0] + n * F[0]) / rho0 - us[0]), abs((j0[1] + n * F[1]) / rho0 - us[1]))
    assert oracle.reduce(*cur, None, snap)["residual"] == pytest.approx(expect, rel=1e-12)


def _steady_channel(ny, nx, F, solid_rho=3.0, solid_j=0.3):
    """The steady Poiseuille state of the paper's wall rule (P5): walls on rows 0 and
    H = ny - 1, u_eq(y) = 3 F y (H - y), rho = 1, j = u_eq - F; the wall rows hold
    values that no FLUID diagnostic may see."""
    flags = np.zeros((ny, nx), np.uint8)
    flags[0] = flags[-1] = oracle.SOLID
    ueq = cf.poiseuille_ueq_paper(ny, F)
    rho = np.ones((ny, nx))
    jx = np.repeat((ueq - F)[:, None], nx, axis=1)
    rho[0] = rho[-1] = solid_rho
    jx[0] = jx[-1] = solid_j
    return flags, rho, jx, np.zeros((ny, nx))


@pytest.mark.parametrize("wall", [0, 1])
def test_reduce_sums_over_fluid_nodes_of_the_steady_channel(wall):
    """Over the N = ny - 2 fluid rows of the steady channel: mass = N nx (rho = 1), x
    momentum = nx sum_y (3 F y (H - y) - F) = nx F ((H - 1) H (H + 1) / 2 - (H - 1)),
    y momentum 0, FLUID count N nx; a fixed point (P5), so the residual after 100 more
    steps is at rounding level.  The wall rows carry rho = 3 and j = 0.3 (and a
    snapshot with j = -0.3), which count nowhere."""
    ny, nx, F = 17, 6, 2.5e-5
    H = ny - 1
    flags, rho, jx, jy = _steady_channel(ny, nx, F)
    if wall == 1:
        ueq = cf.poiseuille_ueq_halfway(ny, F)
        jx[1:-1] = (ueq - F)[1:-1, None]
    snap = (rho.copy(), jx.copy(), jy.copy())
    snap[1][0] = snap[1][-1] = -0.3
    cur = oracle.run(rho, jx, jy, 100, flags, 1, (F, 0.0), wall)
    d = oracle.reduce(*cur, flags, snap)
    N = ny - 2
    assert d["fluid"] == N * nx
    assert d["mass"] == pytest.approx(N * nx, rel=1e-14)
    if wall == 0:
        assert d["mom_x"] == pytest.approx(nx * F * ((H - 1) * H * (H + 1) / 2 - (H - 1)), rel=1e-11)
    else:
        # half-way walls at 1/2 and N + 1/2: u_eq = 3 F [(y - 1/2)(N + 1/2 - y) + 1/4]
        s = sum((yy - 0.5) * (N + 0.5 - yy) + 0.25 for yy in range(1, N + 1))
        assert d["mom_x"] == pytest.approx(nx * F * (3 * s - N), rel=1e-11)
    assert abs(d["mom_y"]) < 1e-13     # rho/6 - rho/6 per node, rounded, summed
    assert d["residual"] < 1e-14       # a fixed point up to rounding; the wall rows would give 0.6
    assert d["nonfinite"] == 0


def test_reduce_counts_non_finite_fluid_nodes():
    """Three FLUID nodes made non-finite, one through each field, and two wall nodes:
    the count is 3."""
    ny, nx, F = 9, 7, 1e-5
    flags, rho, jx, jy = _steady_channel(ny, nx, F)
    rho[2, 1] = np.nan
    jx[4, 3] = np.inf
    jy[6, 5] = -np.inf
    rho[0, 2] = np.nan
    jx[-1, 4] = np.inf
    d = oracle.reduce(rho, jx, jy, flags)
    assert d["nonfinite"] == 3 and d["fluid"] == (ny - 2) * nx


def test_lid_cavity_mass_is_not_conserved_but_fixed_row_is_held():
    """The lid (FIXED row, Appendix A) is a density reservoir and is never updated."""
    ny = nx = 12
    flags = _cavity_flags(ny, nx, obstacle=False)
    rho = np.ones((ny, nx))
    jx = np.zeros((ny, nx))
    jx[-1, 1:-1] = 0.1
    r, u, v = oracle.run(rho, jx, np.zeros((ny, nx)), 200, flags, 0, (0, 0), 0)
    assert np.array_equal(u[-1], jx[-1]) and np.array_equal(r[-1], rho[-1])
    assert u[-2, nx // 2] > 0.01        # the lid drags the top fluid row along


# ----------------------------------------------------------------- P10 BGK at any tau
@pytest.mark.parametrize("periodic", [0, 1, 3])
@pytest.mark.parametrize("wall", [bgk.WALL_PAPER, bgk.WALL_HALFWAY])
def test_p10_bgk_array_form_equals_loop_form(periodic, wall):
    rng = _rng(40 + periodic)
    ny, nx = 9, 11
    rho, jx, jy = _random_state(rng, ny, nx)
    flags = (rng.random((ny, nx)) < 0.15).astype(np.uint8)
    flags[-1, 2:6] = oracle.FIXED
    for tau in (0.6, 1.0, 1.7):
        a = bgk.BGK(rho, jx, jy, flags, periodic, (1e-4, -2e-5), wall, tau)
        b = bgk.BGK(rho, jx, jy, flags, periodic, (1e-4, -2e-5), wall, tau)
        for _ in range(15):
            a.step()
            b.step_arrays()
        assert np.array_equal(a.f, b.f), tau


@pytest.mark.parametrize("tau", [0.55, 0.8, 1.0, 1.7])
@pytest.mark.parametrize("m", [1, 3])
def test_p10_bgk_shear_mode_follows_linear_theory(tau, m):
    """Section 2, Eq. lbm: a small shear wave set on the shear eigenvector of the
    linearised one-step operator decays by its eigenvalue each step."""
    ny, nx, A, n = 32, 4, 1e-8, 12
    kap = 2 * np.pi * m / ny
    lam, v = bgk.shear_mode(tau, kap)
    y = np.arange(ny)
    g = bgk.BGK(np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)), None, 3, (0.0, 0.0), 0, tau)
    w = np.array(bgk.W)[:, None, None]
    wave = lambda t: np.real(A * lam ** t * v[:, None, None] * np.exp(1j * kap * y)[None, :, None])
    g.f = w + wave(0) * np.ones((1, 1, nx))
    g.run(n, arrays=True)
    err = np.abs(g.f - (w + wave(n))).max() / (A * abs(lam) ** n)
    assert err < 1e-6, err
    if tau == 1.0:      # the moments-only closed form of P3
        assert lam.real == pytest.approx(cf.shear_wave_factor(kap), abs=1e-14)


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.3])
def test_p10_bgk_viscosity(tau):
    """Eq. viscosity: the shear mode decays as 1 - nu kappa^2 with nu = (tau - 1/2)/3."""
    kap = 2 * np.pi / 4096
    lam, _ = bgk.shear_mode(tau, kap)
    assert (1 - lam.real) / kap ** 2 == pytest.approx((tau - 0.5) / 3, rel=1e-5)


@pytest.mark.parametrize("tau", [0.7, 1.3])
@pytest.mark.parametrize("wall", [bgk.WALL_PAPER, bgk.WALL_HALFWAY])
def test_p10_bgk_steady_channel_is_exact_parabola(tau, wall):
    """A body-force channel at steady state: the velocity profile has constant
    second difference -F / nu, nu = (tau - 1/2)/3 (Eq. viscosity), under both wall
    rules; the density stays 1."""
    ny, nx, F = 12, 3, 1e-6
    flags = np.zeros((ny, nx), np.uint8)
    flags[0] = flags[-1] = oracle.SOLID
    g = bgk.BGK(np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)), flags, 1, (F, 0.0), wall, tau)
    nu = (tau - 0.5) / 3
    g.run(int(45 / (nu * (np.pi / (ny - 2)) ** 2)), arrays=True)
    rho, jx, _ = g.moments()
    u = (jx / rho)[1:-1, 1]
    d2 = u[2:] - 2 * u[1:-1] + u[:-2]
    assert np.abs(d2 / (-F / nu) - 1).max() < 1e-8
    assert np.abs(rho[1:-1] - 1).max() < 1e-11


@pytest.mark.parametrize("tau", [0.6, 1.4])
def test_p10_bgk_periodic_conservation(tau):
    """Collision keeps mass and adds F to the momentum of every node (velocity-shift
    force); streaming moves populations: over n steps mass is unchanged and the total
    momentum grows by n N F."""
    rng = _rng(77)
    ny, nx, n, F = 13, 17, 30, (3e-5, -1e-5)
    rho, jx, jy = _random_state(rng, ny, nx)
    g = bgk.BGK(rho, jx, jy, None, 3, F, 0, tau)
    M0, X0, Y0 = rho.sum(), jx.sum(), jy.sum()
    r, x, y = g.run(n, arrays=True)
    assert abs(r.sum() - M0) <= 8 * EPS * n * M0
    assert x.sum() == pytest.approx(X0 + n * nx * ny * F[0], abs=1e-12)
    assert y.sum() == pytest.approx(Y0 + n * nx * ny * F[1], abs=1e-12)


# ----------------------------------------------------------------- P11 multiphase
def _sc_state(rng, ny, nx):
    rho = 1.0 + 0.4 * rng.random((ny, nx))
    return rho, 0.01 * rng.standard_normal((ny, nx)), 0.01 * rng.standard_normal((ny, nx))


@pytest.mark.parametrize("periodic", [0, 3])
@pytest.mark.parametrize("wall", [oracle.WALL_PAPER, oracle.WALL_HALFWAY])
def test_p11_bgk_tau1_with_shan_chen_force_equals_moments_only(periodic, wall):
    """Section "Moments-only multirelaxation time LBMTau1": at tau = 1 the populations
    leaving a node are the equilibria of its moments and its Shan-Chen force, so the
    stored-population solver (written independently, loops) and the moments-only
    oracle agree to rounding."""
    rng = _rng(90 + periodic)
    ny, nx = 9, 11
    rho, jx, jy = _sc_state(rng, ny, nx)
    flags = (rng.random((ny, nx)) < 0.1).astype(np.uint8)
    ref = bgk.BGK(rho, jx, jy, flags, periodic, (1e-4, 0.0), wall, 1.0, sc=(-5.0, 1.0))
    for _ in range(12):
        ref.step()
    got = oracle.run(rho, jx, jy, 12, flags, periodic, (1e-4, 0.0), wall, sc=(-5.0, 1.0))
    fl = flags == oracle.FLUID
    for a, b in zip(got, ref.moments()):
        assert np.abs(a - b)[fl].max() < 5e-15


def test_p11_shan_chen_pair_forces_cancel():
    """Eq. f_sc: the force between x and x + e_k is -G w_k psi(x) psi(x + e_k) e_k and
    its reverse, so in a periodic domain the forces sum to zero and the total momentum
    of a run is conserved (mass too)."""
    rng = _rng(93)
    ny, nx = 17, 23
    rho, jx, jy = _sc_state(rng, ny, nx)
    FX, FY = oracle.sc_force(rho, None, 3, -5.5, 1.0)
    scale = np.abs(FX).sum() + np.abs(FY).sum()
    assert abs(FX.sum()) < 1e-14 * scale and abs(FY.sum()) < 1e-14 * scale
    r, u, v = oracle.run(rho, jx, jy, 150, None, 3, (0.0, 0.0), 0, sc=(-5.5, 1.0))
    assert abs(r.sum() - rho.sum()) <= 8 * EPS * 150 * rho.sum()
    assert abs(u.sum() - jx.sum()) < 1e-12 and abs(v.sum() - jy.sum()) < 1e-12
    # G = 0: the plain step, bit for bit
    a = oracle.run(rho, jx, jy, 7, None, 3, (1e-5, 0.0), 0, sc=(0.0, 1.0))
    b = oracle.run(rho, jx, jy, 7, None, 3, (1e-5, 0.0), 0)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))


def _coexistence_theory(G, rho0=1.0):
    """Shan-Chen coexistence densities: p(rho_g) = p(rho_l) and the mechanical-stability
    integral of (p0 - p) psi' / psi^2 from rho_g to rho_l vanishes, with the pressure
    p = rho/3 + G psi^2 / 6 of the D2Q9 force weights (scipy quadrature and root)."""
    from scipy.integrate import quad
    from scipy.optimize import fsolve
    psi = lambda r: rho0 * (1 - np.exp(-r / rho0))
    dpsi = lambda r: np.exp(-r / rho0)
    p = lambda r: r / 3 + G * psi(r) ** 2 / 6

    def eqs(v):
        g, l = v
        return [p(g) - p(l), quad(lambda r: (p(g) - p(r)) * dpsi(r) / psi(r) ** 2, g, l, limit=200)[0]]
    return fsolve(eqs, [0.1, 2.0], xtol=1e-13)


@pytest.mark.parametrize("G", [-5.0, -6.0])
def test_p11_flat_interface_coexistence(G):
    """A liquid slab in vapour (periodic, x-independent) separates into the coexistence
    densities of the model's mechanical-stability condition (liquid within 0.2 %, vapour
    within 1.5 %: the lattice gradients differ from the continuum ones at that level)."""
    oracle.set_threads(4)
    g0, l0 = _coexistence_theory(G)
    ny, nx = 120, 3
    y = np.arange(ny)
    prof = g0 + (l0 - g0) * 0.5 * (np.tanh((y - 30) / 3) - np.tanh((y - 90) / 3))
    rho = np.repeat(prof[:, None], nx, 1)
    z = np.zeros_like(rho)
    r, _, _ = oracle.run(rho, z, z, 40000, None, 3, (0.0, 0.0), 0, sc=(G, 1.0))
    assert abs(r.max() / l0 - 1) < 2e-3
    assert abs(r.min() / g0 - 1) < 1.5e-2


def test_p11_laplace_law():
    """Static drops: the pressure jump times the radius (the surface tension) is the
    same for radii 12, 16 and 20 within 2 %, with p = rho/3 + G psi^2 / 6."""
    oracle.set_threads(4)
    G, L = -5.5, 72
    p = lambda r: r / 3 + G * (1 - np.exp(-r)) ** 2 / 6
    sig = []
    for R0 in (12, 16, 20):
        y, x = np.mgrid[0:L, 0:L]
        d = np.hypot(x - L / 2 + 0.5, y - L / 2 + 0.5)
        rho = 0.104 + (2.307 - 0.104) * 0.5 * (1 - np.tanh((d - R0) / 2))
        z = np.zeros_like(rho)
        r, _, _ = oracle.run(rho, z, z, 8000, None, 3, (0.0, 0.0), 0, sc=(G, 1.0))
        radius = np.sqrt((r > (r.max() + r.min()) / 2).sum() / np.pi)
        sig.append((p(r[L // 2, L // 2]) - p(r[0, 0])) * radius)
    assert max(sig) / min(sig) - 1 < 0.02, sig
    assert 0.08 < np.mean(sig) < 0.11


# ----------------------------------------------------------------- P12 3-D lattices
from oracle import bgk3  # noqa: E402


@pytest.mark.parametrize("q", [19, 27])
def test_p12_3d_lattice_is_isotropic(q):
    """Section 4's D3Q19 / D3Q27: weights sum to 1, first and third moments vanish,
    sum w e_a e_b = delta_ab / 3 and the fourth moment is isotropic (1/9 of the
    symmetrised delta product): exact rational arithmetic."""
    e, w = oracle.tables3(q)
    assert len(e) == q
    W = [Fraction(x).limit_denominator(1000) for x in w]
    assert sum(W) == 1
    for a in range(3):
        assert sum(Wk * ek[a] for Wk, ek in zip(W, e)) == 0
        for b in range(3):
            assert sum(Wk * ek[a] * ek[b] for Wk, ek in zip(W, e)) == (Fraction(1, 3) if a == b else 0)
            for c in range(3):
                assert sum(Wk * ek[a] * ek[b] * ek[c] for Wk, ek in zip(W, e)) == 0
                for d in range(3):
                    iso = Fraction(1, 9) * ((a == b) * (c == d) + (a == c) * (b == d) + (a == d) * (b == c))
                    assert sum(Wk * ek[a] * ek[b] * ek[c] * ek[d] for Wk, ek in zip(W, e)) == iso
    inv = {tuple(x) for x in e}
    assert all(tuple(-x) in inv for x in e)


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("wall", [oracle.WALL_PAPER, oracle.WALL_HALFWAY])
def test_p12_3d_collapses_to_2d(q, wall):
    """One periodic layer in z with no z-momentum: the populations with e_z != 0 come
    back to the same layer and the weights grouped over e_z are those of D2Q9 (4/9,
    1/9, 1/36), so the 3-D step is the (pinned) 2-D step, walls included."""
    rng = _rng(120 + q)
    ny, nx = 9, 11
    rho, jx, jy = _random_state(rng, ny, nx)
    flags = (rng.random((ny, nx)) < 0.15).astype(np.uint8)
    flags[-1, 2:6] = oracle.FIXED
    F = (1e-4, -3e-5)
    ref = oracle.run(rho, jx, jy, 20, flags, 1, F, wall)
    got = oracle.run3(rho[None], jx[None], jy[None], np.zeros((1, ny, nx)), 20, q, flags[None], 1 | 4,
                      (F[0], F[1], 0.0), wall)
    for a, b in zip(got[:3], ref):
        assert np.abs(a[0] - b).max() < 5e-15
    assert np.abs(got[3]).max() < 1e-16


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("periodic", [0, 7])
def test_p12_3d_brute_force_bgk_at_tau1(q, periodic):
    """Eq. lbm vs Eq. LBMTau1 in 3-D: the loop-form stored-population solver at tau = 1
    and the moments-only 3-D oracle agree to rounding (walls, obstacles, a fixed
    plane, force, all three momentum components)."""
    rng = _rng(130 + q + periodic)
    nz, ny, nx = 4, 5, 6
    shape = (nz, ny, nx)
    rho = 1.0 + 1e-2 * rng.standard_normal(shape)
    js = [rho * 1e-2 * rng.standard_normal(shape) for _ in range(3)]
    flags = (rng.random(shape) < 0.12).astype(np.uint8)
    flags[-1, 1:4, 1:4] = oracle.FIXED
    F = (1e-4, -2e-5, 3e-5)
    for wall in (oracle.WALL_PAPER, oracle.WALL_HALFWAY):
        ref = bgk3.BGK3(q, rho, *js, flags, periodic, F, wall, 1.0).run(6)
        got = oracle.run3(rho, *js, 6, q, flags, periodic, F, wall)
        fl = flags == oracle.FLUID
        for a, b in zip(got, ref):
            assert np.abs(a - b)[fl].max() < 5e-15


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_p12_3d_shear_wave_exact(q, axis):
    """A shear wave along each axis decays exactly by (2 + cos k)/3 per step: the
    weights grouped by the wave-direction component are 2/3, 1/6, 1/6 on both
    lattices."""
    n, m, steps, A = 16, 2, 30, 3e-3
    k = 2 * np.pi * m / n
    shape = (n, n, n)
    coord = np.indices(shape)[2 - axis]          # position along the wave axis (x = index 2)
    rho = np.ones(shape)
    js = [np.zeros(shape) for _ in range(3)]
    js[(axis + 1) % 3] = A * np.sin(k * coord)   # momentum transverse to the wave
    got = oracle.run3(rho, *js, steps, q, None, 7)
    lam = cf.shear_wave_factor(k)
    assert np.abs(got[1 + (axis + 1) % 3] - A * lam ** steps * np.sin(k * coord)).max() < 1e-15
    assert np.abs(got[0] - 1).max() <= 8 * EPS * steps     # weights sum to 1 up to rounding


@pytest.mark.parametrize("q", [19, 27])
def test_p12_3d_plate_channel_and_conservation(q):
    """Plates at z = 0 and z = nz - 1, force along x: x- and y-invariant flow follows
    the exact 1-D channel recurrence of the 2-D channel (same grouped weights);
    periodic mass and momentum + n N F are conserved."""
    nz, F = 12, 1e-5
    flags = np.zeros((nz, 3, 3), np.uint8)
    flags[0] = flags[-1] = oracle.SOLID
    one, zero = np.ones((nz, 3, 3)), np.zeros((nz, 3, 3))
    got = oracle.run3(one, zero, zero, zero, 400, q, flags, 3, (F, 0.0, 0.0), oracle.WALL_PAPER)
    ref = cf.channel_1d(nz, F, 0, 400)
    assert np.abs(got[1][1:-1, 1, 1] - ref[1:-1]).max() < 1e-15
    rng = _rng(150)
    shape = (5, 6, 7)
    rho = 1.0 + 1e-2 * rng.standard_normal(shape)
    js = [1e-2 * rng.standard_normal(shape) for _ in range(3)]
    Fv = (2e-5, -1e-5, 3e-5)
    r = oracle.run3(rho, *js, 25, q, None, 7, Fv)
    assert abs(r[0].sum() - rho.sum()) <= 8 * EPS * 25 * rho.sum()
    for a in range(3):
        assert r[1 + a].sum() == pytest.approx(js[a].sum() + 25 * rho.size * Fv[a], abs=1e-13)

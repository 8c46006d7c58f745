"""The section-3 stopping rules on the CPU: driven by stand-in grids with a
known probe history, and by the oracle on a small channel and cavity."""
import math

import numpy as np
import pytest

import oracle
from oracle import closed_forms as CF
from paper_1912_09327_amd import inputs as I
from paper_1912_09327_amd.stopping import centre_velocity, mid_section_flux, section_flux


class ScriptedGrid:
    """Grid whose probed node follows u_n = U (1 - lam^n) (rho = 1)."""

    def __init__(self, U=0.05, lam=0.99, nx=9, ny=7):
        self.nx, self.ny, self.U, self.lam, self.n = nx, ny, U, lam, 0

    def step(self, k):
        self.n += k

    def u(self, n):
        return self.U * (1.0 - self.lam ** n)

    def read_window(self, x0, y0, w, h):
        jx = np.full((h, w), self.u(self.n))
        return np.ones((h, w)), jx, np.zeros((h, w))


def test_centre_rule_fires_at_the_first_step_below_eps():
    for lam, eps in ((0.99, 1e-7), (0.9, 1e-5), (0.999, 1e-9)):
        g = ScriptedGrid(lam=lam)
        out = centre_velocity(g, eps=eps, max_steps=10 ** 6)
        # first n with |u_{n-1} - u_n| / |u_n| < eps, by direct search
        n = 1
        while abs(g.u(n - 1) - g.u(n)) / abs(g.u(n)) >= eps:
            n += 1
        assert out.fired and out.steps == n
        assert out.value == g.u(n)


def test_centre_rule_reports_the_cap():
    out = centre_velocity(ScriptedGrid(lam=0.999), eps=1e-12, max_steps=50)
    assert not out.fired and out.steps == 50


def test_flux_rule_checks_every_interval():
    g = ScriptedGrid(lam=0.999)
    out = mid_section_flux(g, tol=0.01, interval=1000, max_steps=10 ** 6)
    assert out.fired and out.steps % 1000 == 0
    q = lambda n: (g.ny - 2) * g.u(n)
    n = 1000
    while abs(q(n) - q(n - 1000)) / q(n) >= 0.01:
        n += 1000
    assert out.steps == n


class OracleGrid:
    """The oracle behind the grid interface the rules use."""

    def __init__(self, flags, per, F, state):
        self.flags, self.per, self.F = flags, per, F
        self.state = list(state)
        self.ny, self.nx = flags.shape

    def step(self, k):
        self.state = list(oracle.run(*self.state, k, self.flags, self.per, self.F, oracle.WALL_PAPER))

    def read_window(self, x0, y0, w, h):
        return tuple(a[y0:y0 + h, x0:x0 + w].copy() for a in self.state)


def test_centre_rule_on_the_oracle_channel():
    """A 12 x 17 channel: the rule fires while the centre velocity is still short of
    the steady value by about eps / (1 - lam) (lam the slowest mode's factor)."""
    nx, ny, F = 12, 17, 1e-5
    flags, per = I.channel(nx, ny)
    g = OracleGrid(flags, per, (F, 0.0), (np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx))))
    eps = 1e-7
    out = centre_velocity(g, eps=eps, max_steps=100000)
    assert out.fired
    steady = CF.poiseuille_ueq_paper(ny, F)[ny // 2] - F
    lam = CF.shear_wave_factor(math.pi / (ny - 1))
    deficit = (steady - out.value) / steady
    assert 0 < deficit < 2 * eps / (1 - lam)
    assert deficit > 0.5 * eps * lam / (1 - lam)


def test_flux_rule_on_the_oracle_cavity():
    flags, rho, jx, jy, per = I.cavity(24, 0.05)
    g = OracleGrid(flags, per, (0.0, 0.0), (rho, jx, jy))
    out = mid_section_flux(g, tol=0.01, interval=200, max_steps=20000)
    assert out.fired and out.steps % 200 == 0
    q = section_flux(g)
    u = g.state[1] / g.state[0]
    assert q == pytest.approx(np.abs(u[1:-1, 12]).sum())
    # a second check interval later the flux has moved by less than the tolerance
    g.step(200)
    assert abs(section_flux(g) - q) / q < 0.01

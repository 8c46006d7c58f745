"""Host logic of the Re_max sweep (the paper's Discussion section): the
Reynolds number, the horizon rule, the scan reading and the power-law fit."""
import math

import pytest

from paper_1912_09327_amd import stability as S


def test_reynolds_and_viscosity():
    assert S.viscosity(1.0) == pytest.approx(1.0 / 6.0)
    assert S.reynolds(0.1, 256) == pytest.approx(153.6)          # the 256^2 cavity at u_lid 0.1
    assert S.reynolds(0.1, 100, tau=0.55) == pytest.approx(0.1 * 100 / (0.05 / 3))


def test_horizon_rule():
    assert S.horizon(50, 1.0) == 1000                             # at least 1000 steps
    assert S.horizon(1000, 0.5) == 8000                           # four lid transits
    assert S.horizon(1000, 0.01) == 40000                         # capped
    assert S.horizon(333, 0.37) % 100 == 0


def test_scan_reading():
    L, tau = 100, 1.0
    scan = [(0.1, False), (0.2, False), (0.3, True), (0.4, False), (0.5, True)]
    assert S.re_max_from_scan(L, tau, scan) == pytest.approx(S.reynolds(0.2, L))
    assert S.re_max_from_scan(L, tau, [(0.1, True)]) is None
    assert S.re_max_from_scan(L, tau, [(0.1, False), (0.2, False)]) == pytest.approx(S.reynolds(0.2, L))


def test_lid_speeds_are_geometric():
    u = S.lid_speeds(0.1, 1.6, 1.05)
    assert u[0] == 0.1 and u[-1] <= 1.6 and u[-1] * 1.05 > 1.6
    assert all(b / a == pytest.approx(1.05) for a, b in zip(u, u[1:]))


def test_power_law_fit_recovers_the_paper_form():
    Ls = [50, 100, 200, 400, 1000]
    a, b = S.fit_power(Ls, [12.0 * L ** 0.8 for L in Ls])
    assert a == pytest.approx(12.0) and b == pytest.approx(0.8)

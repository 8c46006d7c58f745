"""The two steady-state stopping rules of the paper's section 3.

Both probe a few nodes of a grid through ``read_window`` (no full read-back),
so they work on grids of any size.  A grid here is any object with
``step(n)``, ``read_window(x0, y0, w, h)`` and ``nx``/``ny`` attributes
(``Grid`` is one).

centre_velocity: the channel test.  The velocity u_n at the middle of the
    channel is read after every step and the run stops once
    |u_{n-1} - u_n| / |u_n| < eps (eps = 1e-7 in the paper).
mid_section_flux: the cavity test.  Every ``interval`` steps (1000 in the
    paper) the volumetric flux through the vertical cross-section at half of
    the system is formed and the run stops once its relative change since the
    previous check is below ``tol`` (1 %).  In a closed cavity the net flux
    through that section is zero, so the flux is read as the total exchange
    sum_y |u_x(x_mid, y)| over the interior rows (the lid row and the bottom
    wall left out).

u is the velocity j / rho of the stored moments.
"""
import math

import numpy as np


class Outcome:
    """Result of a stopping-rule run: steps taken, whether the rule fired, the
    last probe value and the last relative change."""

    def __init__(self, steps, fired, value, change):
        self.steps, self.fired, self.value, self.change = int(steps), bool(fired), float(value), float(change)

    def __repr__(self):
        return f"Outcome(steps={self.steps}, fired={self.fired}, value={self.value:.9g}, change={self.change:.3g})"


def _u_at(grid, x, y):
    rho, jx, _ = grid.read_window(x, y, 1, 1)
    return float(jx[0, 0] / rho[0, 0])


def centre_velocity(grid, eps=1e-7, max_steps=10 ** 7, x=None, y=None):
    """Step one at a time until the relative change of u_x at (x, y) (default the
    middle of the grid) between two consecutive steps drops below ``eps``."""
    x = grid.nx // 2 if x is None else int(x)
    y = grid.ny // 2 if y is None else int(y)
    prev = _u_at(grid, x, y)
    change = math.inf
    for n in range(1, int(max_steps) + 1):
        grid.step(1)
        u = _u_at(grid, x, y)
        change = abs(prev - u) / abs(u) if u != 0.0 else math.inf
        if change < eps:
            return Outcome(n, True, u, change)
        prev = u
    return Outcome(max_steps, False, prev, change)


def section_flux(grid, x=None, y0=1, y1=None):
    """sum over y0 <= y < y1 of |jx / rho| at column x (default the middle column)."""
    x = grid.nx // 2 if x is None else int(x)
    y1 = grid.ny - 1 if y1 is None else int(y1)
    rho, jx, _ = grid.read_window(x, y0, 1, y1 - y0)
    return float(np.abs(jx / rho).sum())


def mid_section_flux(grid, tol=0.01, interval=1000, max_steps=10 ** 7, x=None, y0=1, y1=None):
    """Step in blocks of ``interval`` until the section flux changes by less than
    ``tol`` relative to its current value between two consecutive checks."""
    prev = section_flux(grid, x, y0, y1)
    change = math.inf
    n = 0
    while n < max_steps:
        k = min(int(interval), int(max_steps) - n)
        grid.step(k)
        n += k
        q = section_flux(grid, x, y0, y1)
        change = abs(q - prev) / abs(q) if q != 0.0 else math.inf
        if change < tol:
            return Outcome(n, True, q, change)
        prev = q
    return Outcome(n, False, prev, change)

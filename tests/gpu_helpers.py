"""Shared helpers for the GPU tests: run the HIP path through the C ABI and
compare with the CPU oracle."""
import json
import os
import sys

import numpy as np

import oracle
from paper_1912_09327_amd import inputs as I

# FP64 and FP32 bars on the state x = (rho, jx, jy) over FLUID nodes, normwise:
# max |x_gpu - x_oracle| / max |x_oracle| (the density, ~1, sets the scale, so
# this is in effect the bar on the density).
TOL = {"f64": 1e-12, "f32": 1e-5}
# Momentum alone, relative to the largest momentum of the oracle's result:
# max |j_gpu - j_oracle| <= JTOL * max |j_oracle|.
JTOL = {"f64": 1e-12, "f32": 1e-5}
# The looser momentum bar of the named long runs only (the 64 x 32 channel over
# 10,000 steps, the 256^2 cavity over 3,000 and 50,000 steps, the 200 x 100 channel
# to convergence).  The summands of the step are populations of size ~rho/9, so the
# rounding floor of either side in momentum is ~eps * (rho/9) per operation,
# whatever the momentum's size, and errors persist for ~1/(1 - lambda_1) steps of
# the slowest mode.  In the 64 x 32 channel (u_max ~ 7e-4, lambda_1 = (2 +
# cos(pi/31))/3) the FP64 oracle itself sits ~5e-12 of max |j| away from the exact
# 1-D recurrence after 10,000 steps, so a bar of 1e-12 there would test the
# oracle's rounding, not the GPU.
LONG_JTOL = {"f64": 1e-10, "f32": 1e-4}
# Reduced-precision storage: one rounding to 11 (binary16) or 8 (bfloat16)
# significand bits per stored value and step; the averaging stencil damps
# earlier roundings, so the drift from the FP64 trajectory stays within a few
# units in the last place of the field's largest value.  Stated bar: 8 ulp of
# the field's largest magnitude (2^-11 or 2^-8 relative per ulp).
ULP = {"f16s": 2.0 ** -11, "bf16s": 2.0 ** -8}


def gpu_run(flags, rho, jx, jy, n, prec="f64", wall="paper", periodic=0, force=(0.0, 0.0),
            kernel=None, scale=(0.0, 0.0)):
    from paper_1912_09327_amd.grid import Grid
    ny, nx = np.shape(rho) if rho is not None else np.shape(flags)
    g = Grid(nx, ny, prec=prec, wall=wall, periodic=periodic, force=force, scale=scale)
    try:
        if kernel:
            g.set_kernel(**kernel)
        g.set_geometry(flags, rho, jx, jy)
        g.step(n)
        return g.read_moments()
    finally:
        g.close()


def field_errors(got, ref, flags=None, init=None):
    """(normwise state error, momentum error) over FLUID nodes.

    state error: max |x - x_ref| / max |x_ref| with x = (rho, jx, jy);
    momentum error: max |j - j_ref| / max(max |j_ref|, 1e-3).  The floor of 1e-3:
    the FP64 oracle sums populations of size rho/9 in the paper's rho form, so its
    rounding floor in momentum is a few eps absolute (~1e-15), which is 1e-12 of a
    momentum of 1e-3; runs whose momentum decays below that (a 3 x 3 box drained
    by its walls) are held to that absolute floor.  ``init`` is accepted for the
    callers' convenience and not used (the bar is relative to the result).
    Every measurement is printed, and appended to the JSON-lines file named by
    LBT1_PARITY_LOG when that is set, so each test's error can be stated beside
    its bar.
    """
    r, u, v = got
    R, U, V = ref
    m = np.ones(R.shape, bool) if flags is None else (np.asarray(flags) == I.FLUID)
    if not m.any():   # nothing is updated: the state must come back unchanged
        same = all(np.array_equal(a, b) for a, b in zip(got, ref))
        return (0.0, 0.0) if same else (np.inf, np.inf)
    xscale = max(np.abs(R[m]).max(), np.abs(U[m]).max(), np.abs(V[m]).max())
    jscale = max(np.abs(U[m]).max(), np.abs(V[m]).max(), 1e-3)
    dj = max(np.abs(u - U)[m].max(), np.abs(v - V)[m].max())
    ex = max(np.abs(r - R)[m].max(), dj) / xscale
    _record(dict(state=float(ex), momentum=float(dj / jscale), jmax=float(jscale)))
    return ex, dj / jscale


def _record(rec):
    test = os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0]
    rec = dict(test=test, **rec)
    print(f"[parity] {test}: state {rec['state']:.2e}, momentum {rec['momentum']:.2e} of max|j| "
          f"{rec['jmax']:.2e}", file=sys.stderr, flush=True)
    path = os.environ.get("LBT1_PARITY_LOG")
    if path:
        with open(path, "a") as fh:
            fh.write(json.dumps(rec) + "\n")


def reduced_bar(prec, ref, flags=None):
    """Stated bar for reduced-precision storage, 8 ulp of the largest stored magnitude:
    (absolute density bar = 8 ulp * max |rho - 1|, momentum bar relative to max |j|)."""
    R, U, V = ref
    m = np.ones(R.shape, bool) if flags is None else (np.asarray(flags) == I.FLUID)
    dmax = np.abs(R[m] - 1).max()
    return 8 * ULP[prec] * max(dmax, 1e-300), 8 * ULP[prec]


def oracle_run(flags, rho, jx, jy, n, wall="paper", periodic=0, force=(0.0, 0.0)):
    w = oracle.WALL_PAPER if wall == "paper" else oracle.WALL_HALFWAY
    return oracle.run(rho, jx, jy, n, flags, periodic, force, w)

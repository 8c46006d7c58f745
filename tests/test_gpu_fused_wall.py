"""GPU tests of the two-steps-per-launch strip kernel on grids with walls, fixed
(lid) nodes and non-periodic axes (through the C ABI).

Every configuration must give the bits of single steps of the gather kernel:
both wall rules, four storage formats, cavities with a lid, channels, random
obstacles, open grids whose edges are walls, widths that leave a partial last
chunk, odd step counts (a single-step launch finishes them), graph bursts and
split calls; FP64 is also held to the oracle.
"""
import numpy as np
import pytest

from gpu_helpers import JTOL, TOL, field_errors, gpu_run, oracle_run
from paper_1912_09327_amd import inputs as I

pytestmark = pytest.mark.gpu

GATHER = dict(kernel="gather")
# strip heights built for two fused steps with walls (30 rows not in FP64)
ROWS = {"f64": (2, 6, 14), "f32": (2, 6, 14, 30), "f16s": (2, 6, 14, 30), "bf16s": (2, 6, 14, 30)}


def _case(kind, nx, ny, seed):
    rng = np.random.default_rng(seed)
    rho, jx, jy = I.random_state(nx, ny, rng)
    if kind == "cavity":
        flags, r0, x0, y0, _ = I.cavity(nx, 0.08, ny)
        flags[ny // 2, nx // 3] = I.SOLID
        lid = flags == I.FIXED
        rho[lid], jx[lid], jy[lid] = r0[lid], x0[lid], y0[lid]
        return flags, rho, jx, jy, 0
    if kind == "channel":
        flags, per = I.channel(nx, ny)
        return flags, rho, jx, jy, per
    if kind == "obstacles":            # periodic in both axes, solid nodes inside
        return I.random_obstacles(nx, ny, 0.15, rng), rho, jx, jy, 3
    if kind == "obstacles_walls":      # periodic in y only: walls at x = -1 and x = nx
        return I.random_obstacles(nx, ny, 0.1, rng), rho, jx, jy, 2
    if kind == "open":                 # no flags, no periodicity
        return None, rho, jx, jy, 0
    raise ValueError(kind)


KINDS = ["cavity", "channel", "obstacles", "obstacles_walls", "open"]


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s", "bf16s"])
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("wall", ["paper", "halfway"])
def test_fused_wall_bitwise_equals_single_steps(prec, kind, wall):
    shapes = [(130, 45), (64, 20)] + ([] if kind in ("channel", "obstacles") else [(131, 33)])
    for nx, ny in shapes:
        flags, rho, jx, jy, per = _case(kind, nx, ny, nx * 7 + ny)
        F = (1e-5, -2e-6)
        base = gpu_run(flags, rho, jx, jy, 25, prec, wall, per, F, kernel=GATHER)
        for rows in ROWS[prec]:
            for waves in (0, 8):
                cfg = dict(kernel="strip", vec=2, rows=rows, waves=waves, fuse=2)
                got = gpu_run(flags, rho, jx, jy, 25, prec, wall, per, F, kernel=cfg)
                for a, b in zip(base, got):
                    assert np.array_equal(a, b), (nx, ny, rows, waves)


@pytest.mark.parametrize("prec", ["f32", "f16s"])
@pytest.mark.parametrize("wall", ["paper", "halfway"])
def test_fused_wall_bursts_and_splitting(prec, wall):
    """Graph bursts of 32 two-step launches, odd remainders and split calls."""
    from paper_1912_09327_amd.grid import Grid
    nx, ny = 200, 90
    flags, rho, jx, jy, per = _case("cavity", nx, ny, 3)
    ref = gpu_run(flags, rho, jx, jy, 231, prec, wall, per, kernel=GATHER)
    g = Grid(nx, ny, prec=prec, periodic=per, wall=wall)
    try:
        g.set_geometry(flags, rho, jx, jy)
        g.set_kernel("strip", vec=2, rows=14, waves=0, fuse=2)
        for n in (1, 64, 3, 128, 21, 2, 4, 5, 1, 2):
            g.step(n)
        got = g.read_moments()
    finally:
        g.close()
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("wall", ["paper", "halfway"])
def test_fused_wall_f64_matches_oracle(wall):
    nx, ny = 150, 70
    flags, rho, jx, jy, per = _case("cavity", nx, ny, 8)
    F = (2e-5, 1e-5)
    ref = oracle_run(flags, rho, jx, jy, 40, wall, per, F)
    got = gpu_run(flags, rho, jx, jy, 40, "f64", wall, per, F,
                  kernel=dict(kernel="strip", vec=2, rows=6, waves=0, fuse=2))
    ex, ej = field_errors(got, ref, flags, (rho, jx, jy))
    assert ex <= TOL["f64"] and ej <= JTOL["f64"], (ex, ej)


def test_fused_wall_refusals():
    from paper_1912_09327_amd import _capi as C
    from paper_1912_09327_amd.grid import Grid
    flags, rho, jx, jy, per = _case("cavity", 64, 32, 1)
    g = Grid(64, 32, prec="f32", periodic=per)
    try:
        g.set_geometry(flags, rho, jx, jy)
        for cfg in (dict(vec=4, rows=14, fuse=3),     # three steps need a periodic grid without walls
                    dict(vec=1, rows=14, fuse=2),     # fuse > vec
                    dict(vec=4, rows=14, fuse=2)):    # not built
            with pytest.raises(C.Lbt1Error) as e:
                g.set_kernel("strip", **cfg)
            assert e.value.status == C.EINVAL, cfg
        g.set_kernel("strip", vec=2, rows=14, fuse=2)
        cfg, name = g.kernel()
        assert cfg["fuse"] == 2 and "fused_wall" in name
        g.step(3)
    finally:
        g.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("shape", [(130, 3), (131, 4), (64, 5), (6, 9)])
@pytest.mark.parametrize("kind", ["open", "channel", "obstacles_walls"])
def test_fused_wall_thin_grids(prec, shape, kind):
    """Grids of 3 to 9 rows or 6 columns: every strip row is a halo or wrapped row."""
    nx, ny = shape
    if kind == "channel" and nx % 2:
        pytest.skip("periodic in x: 2 columns per lane need an even width")
    if kind == "channel":
        flags, per = I.channel(nx, ny)
        rho, jx, jy = I.random_state(nx, ny, np.random.default_rng(nx + ny))
    else:
        flags, rho, jx, jy, per = _case(kind, nx, ny, nx + 3 * ny)
    F = (1e-5, 3e-6)
    base = gpu_run(flags, rho, jx, jy, 13, prec, "halfway", per, F, kernel=GATHER)
    for rows in ROWS[prec]:
        got = gpu_run(flags, rho, jx, jy, 13, prec, "halfway", per, F,
                      kernel=dict(kernel="strip", vec=2, rows=rows, waves=0, fuse=2))
        for a, b in zip(base, got):
            assert np.array_equal(a, b), rows

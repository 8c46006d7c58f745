"""GPU tests of the fused two-step strip kernel (through the C ABI).

Two steps per launch on grids periodic in both axes with no wall or fixed
nodes.  Every configuration must give the bits of single steps (the gather
kernel), for odd step counts (a single-step launch finishes them), across
graph bursts, on grids smaller than a strip and with ragged strips; FP64 is
also held to the oracle.
"""
import numpy as np
import pytest

from gpu_helpers import JTOL, TOL, field_errors, gpu_run, oracle_run
from paper_1912_09327_amd import inputs as I

pytestmark = pytest.mark.gpu

BUILT = {"f64": (2,), "f32": (2, 4), "f16s": (2, 4), "bf16s": (2, 4)}


def _state(nx, ny, seed):
    return I.random_state(nx, ny, np.random.default_rng(seed))


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s", "bf16s"])
@pytest.mark.parametrize("shape", [(512, 77), (248, 64), (130, 33), (8, 5), (4, 3)])
def test_fused_bitwise_equals_single_steps(prec, shape):
    nx, ny = shape
    rho, jx, jy = _state(nx, ny, 31)
    F = (1e-5, -2e-6)
    base = gpu_run(None, rho, jx, jy, 25, prec, "paper", 3, F, kernel=dict(kernel="gather"))
    for vec in BUILT[prec]:
        if nx % vec:
            continue
        for rows in (6, 14):
            for waves in (0, 8):
                cfg = dict(kernel="strip", vec=vec, rows=rows, waves=waves, fuse=2)
                got = gpu_run(None, rho, jx, jy, 25, prec, "paper", 3, F, kernel=cfg)
                for a, b in zip(base, got):
                    assert np.array_equal(a, b), (vec, rows, waves)


@pytest.mark.parametrize("prec,vec,fuse,rows", [("f32", 2, 2, 14), ("f16s", 2, 2, 14), ("f32", 4, 3, 14),
                                                ("f32", 4, 3, 22), ("f32", 4, 3, 28), ("f32", 4, 3, 6)])
def test_fused_graph_bursts_and_splitting(prec, vec, fuse, rows):
    """Bursts (32 launches of two steps; 21 launches of three, which flip the parity),
    remainders (two-step launches after three-step ones, single steps) and split calls."""
    from paper_1912_09327_amd.grid import Grid
    nx, ny = 372, 90
    rho, jx, jy = _state(nx, ny, 5)
    ref = gpu_run(None, rho, jx, jy, 231, prec, "paper", 3, kernel=dict(kernel="gather"))
    g = Grid(nx, ny, prec=prec, periodic=3)
    try:
        g.set_geometry(None, rho, jx, jy)
        g.set_kernel("strip", vec=vec, rows=rows, waves=0, fuse=fuse)
        for n in (1, 64, 3, 128, 21, 2, 4, 5, 1, 2):
            g.step(n)
        got = g.read_moments()
    finally:
        g.close()
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["f32"])
@pytest.mark.parametrize("shape", [(512, 77), (248, 64), (8, 5)])
def test_three_fused_steps_bitwise(prec, shape):
    nx, ny = shape
    rho, jx, jy = _state(nx, ny, 33)
    F = (1e-5, -2e-6)
    base = gpu_run(None, rho, jx, jy, 26, prec, "paper", 3, F, kernel=dict(kernel="gather"))
    for rows in (6, 14):
        for waves in (0, 8):
            cfg = dict(kernel="strip", vec=4, rows=rows, waves=waves, fuse=3)
            got = gpu_run(None, rho, jx, jy, 26, prec, "paper", 3, F, kernel=cfg)
            for a, b in zip(base, got):
                assert np.array_equal(a, b), (rows, waves)


def test_fused_f64_matches_oracle():
    nx, ny = 260, 70
    rho, jx, jy = _state(nx, ny, 8)
    F = (2e-5, 1e-5)
    ref = oracle_run(None, rho, jx, jy, 40, "paper", 3, F)
    got = gpu_run(None, rho, jx, jy, 40, "f64", "paper", 3, F,
                  kernel=dict(kernel="strip", vec=2, rows=6, waves=0, fuse=2))
    ex, ej = field_errors(got, ref)
    assert ex <= TOL["f64"] and ej <= JTOL["f64"], (ex, ej)


def test_fused_refused_where_it_does_not_apply():
    from paper_1912_09327_amd import _capi as C
    from paper_1912_09327_amd.grid import Grid
    flags, per = I.channel(64, 32)
    g = Grid(64, 32, prec="f32", periodic=per)
    try:
        g.set_geometry(flags)
        with pytest.raises(C.Lbt1Error) as e:            # three steps need a grid without walls
            g.set_kernel("strip", vec=4, rows=14, fuse=3)
        assert e.value.status == C.EINVAL
    finally:
        g.close()
    g = Grid(64, 32, prec="f32", periodic=3)
    try:
        g.set_geometry(None)
        with pytest.raises(C.Lbt1Error) as e:            # fuse > vec
            g.set_kernel("strip", vec=1, rows=6, fuse=2)
        assert e.value.status == C.EINVAL
        with pytest.raises(C.Lbt1Error) as e:            # not built
            g.set_kernel("strip", vec=2, rows=6, fuse=4)
        assert e.value.status == C.EINVAL
        g.set_kernel("strip", vec=2, rows=6, fuse=2)
        cfg, name = g.kernel()
        assert cfg["fuse"] == 2 and "fused" in name
        g.step(3)
    finally:
        g.close()


@pytest.mark.parametrize("prec,vec,rows,fuse", [("f32", 4, 22, 2), ("f16s", 2, 22, 2), ("f16s", 2, 30, 2),
                                                ("bf16s", 2, 30, 2), ("f32", 4, 22, 3), ("f32", 4, 28, 2),
                                                ("f32", 4, 28, 3)])
@pytest.mark.parametrize("shape", [(512, 77), (248, 33)])
def test_tall_fused_strips_bitwise(prec, vec, rows, fuse, shape):
    """Strips taller than the single-step kernels: the remainder of 25 steps goes to
    the gather kernel (after two-step launches) or to two two-step launches (after
    three-step launches)."""
    nx, ny = shape
    rho, jx, jy = _state(nx, ny, 41)
    base = gpu_run(None, rho, jx, jy, 25, prec, "paper", 3, (1e-5, 0.0), kernel=dict(kernel="gather"))
    for waves in (0, 8):
        got = gpu_run(None, rho, jx, jy, 25, prec, "paper", 3, (1e-5, 0.0),
                      kernel=dict(kernel="strip", vec=vec, rows=rows, waves=waves, fuse=fuse))
        for a, b in zip(base, got):
            assert np.array_equal(a, b), waves


@pytest.mark.parametrize("prec,kind", [("f32", "periodic"), ("f16s", "periodic"), ("f64", "cavity")])
def test_autotune_leaves_the_state_and_the_trajectory_unchanged(prec, kind):
    """The autotuner times its candidates on the grid's own memory: the state it
    saved is restored bit for bit, and the steps after it give the bits of a grid
    that was never tuned (every kernel family gives the same bits)."""
    from paper_1912_09327_amd.grid import Grid
    nx, ny = 520, 66
    if kind == "periodic":
        flags, per = None, 3
        rho, jx, jy = _state(nx, ny, 71)
    else:
        flags, rho, jx, jy = I.cavity(nx, 0.05)[:4]
        ny, per = nx, 0
    ref = gpu_run(flags, rho, jx, jy, 37, prec, "paper", per, kernel=dict(kernel="gather"))
    g = Grid(nx, ny, prec=prec, periodic=per)
    try:
        g.set_geometry(flags, rho, jx, jy)
        before = g.read_moments()
        g.step(5)
        mid = g.read_moments()
        cfg, _ = g.autotune(steps=12, reps=2)
        after = g.read_moments()
        for a, b in zip(mid, after):
            assert np.array_equal(a, b)
        g.step(32)
        got = g.read_moments()
    finally:
        g.close()
    assert cfg["kernel"] in (1, 2)
    assert not all(np.array_equal(a, b) for a, b in zip(before, mid))
    for a, b in zip(ref, got):
        assert np.array_equal(a, b), cfg


def test_tuned_shape_of_a_walled_grid_is_not_reused_on_a_periodic_one():
    """The autotuner's choice is remembered per grid kind.  A walled grid of odd width
    may tune to strips whose chunks do not divide the width (its last chunk is padded
    with solid columns); a channel of the same size, precision and wall rule that is
    periodic in x cannot take that shape.  The channel must bind its own default shape
    and match the oracle."""
    from paper_1912_09327_amd.grid import Grid
    L = 263
    flags, rho, jx, jy, per = I.cavity(L, 0.05)
    g = Grid(L, L, prec="f64", periodic=per)
    try:
        g.set_geometry(flags, rho, jx, jy)
        cfg, _ = g.autotune(steps=12, reps=2)
    finally:
        g.close()
    cflags, cper = I.channel(L, L)
    crho, cjx, cjy = _state(L, L, 17)
    F = (2e-6, 0.0)
    got = gpu_run(cflags, crho, cjx, cjy, 20, "f64", "paper", cper, F)
    ref = oracle_run(cflags, crho, cjx, cjy, 20, "paper", cper, F)
    ex, ej = field_errors(got, ref, cflags)
    assert ex <= TOL["f64"] and ej <= JTOL["f64"], (cfg, ex, ej)

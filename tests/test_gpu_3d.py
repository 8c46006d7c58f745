"""GPU parity of the 3-D LBMTau1 grids (D3Q19, D3Q27) through the C ABI,
against the 3-D FP64 oracle."""
import numpy as np
import pytest

import oracle
from gpu_helpers import JTOL, TOL, ULP
from paper_1912_09327_amd import inputs as I

pytestmark = pytest.mark.gpu


def _case(kind, shape, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    rho = 1.0 + 1e-2 * rng.standard_normal(shape)
    js = [rho * 1e-2 * rng.standard_normal(shape) for _ in range(3)]
    if kind == "periodic":
        return None, rho, js, 7
    if kind == "box":         # closed box, lid plane on top moving in x, obstacles
        flags = (rng.random(shape) < 0.08).astype(np.uint8)
        flags[0] = flags[:, 0] = flags[:, -1] = flags[:, :, 0] = flags[:, :, -1] = I.SOLID
        flags[-1, 1:-1, 1:-1] = I.FIXED
        lid = flags == I.FIXED
        rho[lid] = 1.0
        js[0][lid], js[1][lid], js[2][lid] = 0.05, 0.0, 0.0
        return flags, rho, js, 0
    if kind == "plates":      # plates at z = 0 and nz - 1, periodic in x and y
        flags = np.zeros(shape, np.uint8)
        flags[0] = flags[-1] = I.SOLID
        return flags, rho, js, 3
    if kind == "open":
        return None, rho, js, 0
    raise ValueError(kind)


def _gpu(flags, rho, js, n, q, prec, wall, per, F):
    from paper_1912_09327_amd.grid3d import Grid3D
    nz, ny, nx = rho.shape
    g = Grid3D(nx, ny, nz, q=q, prec=prec, wall=wall, periodic=per, force=F)
    try:
        g.set_geometry(flags, rho, *js)
        g.step(n)
        return g.read_moments(), g.reduce()
    finally:
        g.close()


def _errors(got, ref, flags):
    m = np.ones(ref[0].shape, bool) if flags is None else flags == I.FLUID
    xscale = max(np.abs(a[m]).max() for a in ref)
    jscale = max(np.abs(a[m]).max() for a in ref[1:])
    dj = max(np.abs(a - b)[m].max() for a, b in zip(got[1:], ref[1:]))
    ex = max(np.abs(got[0] - ref[0])[m].max(), dj) / xscale
    return ex, dj / jscale


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("wall", ["paper", "halfway"])
@pytest.mark.parametrize("kind", ["periodic", "box", "plates", "open"])
def test_3d_f64_matches_oracle(kind, wall, q):
    shape = (9, 21, 70)
    flags, rho, js, per = _case(kind, shape, 3)
    F = (1e-5, -2e-6, 3e-6)
    (got, _) = _gpu(flags, rho, js, 20, q, "f64", wall, per, F)
    w = oracle.WALL_PAPER if wall == "paper" else oracle.WALL_HALFWAY
    ref = oracle.run3(rho, *js, 20, q, flags, per, F, w)
    ex, ej = _errors(got, ref, flags)
    assert ex <= TOL["f64"] and ej <= JTOL["f64"], (ex, ej)


@pytest.mark.parametrize("q", [19, 27])
def test_3d_f32_matches_oracle(q):
    shape = (24, 33, 130)
    flags, rho, js, per = _case("box", shape, 4)
    (got, _) = _gpu(flags, rho, js, 60, q, "f32", "paper", per, (0.0, 0.0, 0.0))
    oracle.set_threads(16)
    ref = oracle.run3(rho, *js, 60, q, flags, per)
    ex, ej = _errors(got, ref, flags)
    assert ex <= TOL["f32"] and ej <= JTOL["f32"], (ex, ej)


@pytest.mark.parametrize("prec", ["f16s", "bf16s"])
def test_3d_reduced_precision_bar(prec):
    shape = (16, 16, 64)
    flags, rho, js, per = _case("periodic", shape, 5)
    (got, _) = _gpu(flags, rho, js, 20, 19, prec, "paper", per, (0.0, 0.0, 0.0))
    ref = oracle.run3(rho, *js, 20, 19, flags, per)
    dr = np.abs(got[0] - ref[0]).max() / np.abs(ref[0] - 1).max()
    dj = max(np.abs(a - b).max() for a, b in zip(got[1:], ref[1:])) / max(np.abs(a).max() for a in ref[1:])
    assert dr <= 8 * ULP[prec] and dj <= 8 * ULP[prec], (dr, dj)


@pytest.mark.parametrize("q", [19, 27])
def test_3d_periodic_conservation_and_reductions(q):
    shape = (32, 40, 64)
    flags, rho, js, per = _case("periodic", shape, 6)
    F = (2e-6, 0.0, -1e-6)
    (got, d) = _gpu(flags, rho, js, 100, q, "f64", "paper", per, F)
    n = rho.size
    assert d["fluid"] == n and d["nonfinite"] == 0
    assert d["mass"] == pytest.approx(rho.sum(), rel=1e-13)
    for a in range(3):
        assert d["mom"][a] == pytest.approx(js[a].sum() + 100 * n * F[a], abs=1e-9)
        assert d["mom"][a] == pytest.approx(got[1 + a].sum(), abs=1e-9)


def test_3d_errors():
    from paper_1912_09327_amd import _capi as C
    from paper_1912_09327_amd.grid3d import Grid3D
    with pytest.raises(C.Lbt1Error):
        Grid3D(16, 16, 16, q=15)
    g = Grid3D(16, 16, 8, q=19)
    try:
        with pytest.raises(C.Lbt1Error) as e:
            g.step(1)
        assert e.value.status == C.ESTATE
        bad = np.zeros((8, 16, 16), np.uint8)
        bad[1, 2, 3] = 9
        with pytest.raises(C.Lbt1Error) as e:
            g.set_geometry(bad)
        assert e.value.status == C.EINVAL
        g.set_geometry(None)
        g.step(2)
    finally:
        g.close()


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("shape", [(9, 21, 70), (16, 4, 64), (20, 7, 130), (1, 3, 5), (40, 9, 124)])
@pytest.mark.parametrize("kind,wall", [("periodic", "paper"), ("box", "paper"), ("box", "halfway"),
                                       ("plates", "paper"), ("plates", "halfway"), ("open", "halfway")])
def test_3d_tile_bitwise_equals_gather(kind, wall, shape, prec, q):
    """The tile kernels (lane exchange on periodic grids; walls, fixed nodes and
    non-periodic axes as well) give the bits of one thread per node."""
    from paper_1912_09327_amd.grid3d import Grid3D
    if kind == "box" and min(shape) < 3:
        pytest.skip("a box needs three nodes along every axis")
    flags, rho, js, per = _case(kind, shape, 7)
    nz, ny, nx = shape
    F = (1e-5, 2e-6, -3e-6)
    out = {}
    for kern in ("gather", "tile"):
        g = Grid3D(nx, ny, nz, q=q, prec=prec, wall=wall, periodic=per, force=F)
        try:
            g.set_kernel(kern)
            g.set_geometry(flags, rho, *js)
            assert g.kernel() == kern
            g.step(11)
            out[kern] = g.read_moments()
        finally:
            g.close()
    for a, b in zip(out["gather"], out["tile"]):
        assert np.array_equal(a, b)


def test_3d_tile_is_the_default_with_walls():
    from paper_1912_09327_amd.grid3d import Grid3D
    flags, rho, js, per = _case("plates", (8, 8, 64), 8)
    g = Grid3D(64, 8, 8, q=19, periodic=per)
    try:
        g.set_geometry(flags, rho, *js)
        assert g.kernel() == "tile"
        g.set_kernel("gather")
        assert g.kernel() == "gather"
        g.step(2)
    finally:
        g.close()

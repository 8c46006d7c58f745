"""GPU parity of the stored-population BGK grids (LBT1_OPT_POPULATIONS)
through the C ABI, against the brute-force BGK oracle (array form) at
several relaxation times, and against the LBMTau1 path at tau = 1."""
import sys

import numpy as np
import pytest

from gpu_helpers import JTOL, TOL, ULP, field_errors
from oracle import bgk
from paper_1912_09327_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _case(kind, nx, ny, seed):
    rng = np.random.default_rng(seed)
    rho, jx, jy = I.random_state(nx, ny, rng)
    if kind == "periodic":
        return None, rho, jx, jy, 3
    if kind == "cavity":
        flags, r0, x0, y0, _ = I.cavity(nx, 0.08, ny)
        flags[ny // 2, nx // 3] = I.SOLID
        lid = flags == I.FIXED
        rho[lid], jx[lid], jy[lid] = r0[lid], x0[lid], y0[lid]
        return flags, rho, jx, jy, 0
    if kind == "channel":
        flags = I.random_obstacles(nx, ny, 0.1, rng)
        flags[0] = flags[-1] = I.SOLID
        return flags, rho, jx, jy, I.PERIODIC_X
    if kind == "open":
        return None, rho, jx, jy, 0
    raise ValueError(kind)


def _gpu(flags, rho, jx, jy, n, prec, wall, per, F, tau, split=None):
    from paper_1912_09327_amd.grid import Grid
    ny, nx = rho.shape
    g = Grid(nx, ny, prec=prec, wall=wall, periodic=per, force=F, populations=True, tau=tau)
    try:
        g.set_geometry(flags, rho, jx, jy)
        for k in (split or [n]):
            g.step(k)
        return g.read_moments(), g.read_populations()
    finally:
        g.close()


def _oracle(flags, rho, jx, jy, n, wall, per, F, tau):
    w = bgk.WALL_PAPER if wall == "paper" else bgk.WALL_HALFWAY
    o = bgk.BGK(rho, jx, jy, flags, per, F, w, tau)
    mom = o.run(n, arrays=True)
    return mom, o.f


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
@pytest.mark.parametrize("wall", ["paper", "halfway"])
@pytest.mark.parametrize("kind", ["periodic", "cavity", "channel", "open"])
def test_bgk_f64_matches_oracle(kind, wall, tau):
    nx, ny, n = 70, 45, 40
    flags, rho, jx, jy, per = _case(kind, nx, ny, 3)
    F = (2e-5, -1e-5)
    (got, fg) = _gpu(flags, rho, jx, jy, n, "f64", wall, per, F, tau)
    ref, fo = _oracle(flags, rho, jx, jy, n, wall, per, F, tau)
    ex, ej = field_errors(got, ref, flags)
    assert ex <= TOL["f64"] and ej <= JTOL["f64"], (ex, ej)
    live = np.ones((ny, nx), bool) if flags is None else flags != I.SOLID
    assert np.abs(fg - fo)[:, live].max() <= 1e-12 * np.abs(fo[:, live]).max()


@pytest.mark.parametrize("tau", [0.6, 1.3])
@pytest.mark.parametrize("kind", ["periodic", "cavity"])
def test_bgk_f32_matches_oracle(kind, tau):
    nx, ny, n = 130, 33, 60
    flags, rho, jx, jy, per = _case(kind, nx, ny, 4)
    (got, _) = _gpu(flags, rho, jx, jy, n, "f32", "halfway", per, (1e-5, 0.0), tau)
    ref, _ = _oracle(flags, rho, jx, jy, n, "halfway", per, (1e-5, 0.0), tau)
    ex, ej = field_errors(got, ref, flags)
    assert ex <= TOL["f32"] and ej <= JTOL["f32"], (ex, ej)


@pytest.mark.parametrize("prec", ["f16s", "bf16s"])
def test_bgk_reduced_precision_bar(prec):
    """Nine populations stored as 16-bit deviations, 20 steps: the moments stay within
    16 ulp of the largest magnitude of each moment field (each moment sums nine
    rounded populations; stated bar, parity unpinned beyond it)."""
    nx, ny, n = 96, 40, 20
    flags, rho, jx, jy, per = _case("periodic", nx, ny, 6)
    (got, _) = _gpu(flags, rho, jx, jy, n, prec, "paper", per, (0.0, 0.0), 0.8)
    ref, _ = _oracle(flags, rho, jx, jy, n, "paper", per, (0.0, 0.0), 0.8)
    dr = np.abs(got[0] - ref[0]).max() / np.abs(ref[0] - 1).max()
    dj = max(np.abs(got[1] - ref[1]).max(), np.abs(got[2] - ref[2]).max()) / max(
        np.abs(ref[1]).max(), np.abs(ref[2]).max())
    _say(f"[bgk] {prec}: density {dr:.3g}, momentum {dj:.3g} (ulp {ULP[prec]:.3g})")
    assert dr <= 16 * ULP[prec] and dj <= 16 * ULP[prec], (dr, dj)


def test_bgk_tau1_matches_lbmtau1():
    """At tau = 1 the relaxed populations are the equilibria (Eq. LBMTau1): the
    stored-population grid and the moments-only grid give the same moments."""
    from gpu_helpers import gpu_run
    nx, ny, n = 200, 77, 300
    flags, rho, jx, jy, per = _case("cavity", nx, ny, 8)
    for wall in ("paper", "halfway"):
        (pop, _) = _gpu(flags, rho, jx, jy, n, "f64", wall, per, (1e-5, 0.0), 1.0)
        mom = gpu_run(flags, rho, jx, jy, n, "f64", wall, per, (1e-5, 0.0))
        ex, ej = field_errors(pop, mom, flags)
        assert ex <= TOL["f64"] and ej <= JTOL["f64"], (wall, ex, ej)


def test_bgk_bursts_splitting_and_reductions():
    from paper_1912_09327_amd.grid import Grid
    nx, ny = 150, 64
    flags, rho, jx, jy, per = _case("channel", nx, ny, 9)
    F = (1e-5, 0.0)
    (a, fa) = _gpu(flags, rho, jx, jy, 150, "f32", "paper", per, F, 0.7)
    (b, fb) = _gpu(flags, rho, jx, jy, 150, "f32", "paper", per, F, 0.7, split=[1, 64, 5, 80])
    assert np.array_equal(fa, fb) and all(np.array_equal(x, y) for x, y in zip(a, b))
    g = Grid(nx, ny, prec="f64", periodic=per, force=F, populations=True, tau=0.7)
    try:
        g.set_geometry(flags, rho, jx, jy)
        g.step(100)
        d = g.reduce()
        r, x, y = g.read_moments()
        m = flags == I.FLUID
        assert d["fluid"] == int(m.sum()) and d["nonfinite"] == 0
        assert d["mass"] == pytest.approx(r[m].sum(), rel=1e-13)
        assert d["mom_x"] == pytest.approx(x[m].sum(), rel=1e-12, abs=1e-15)
        ref = np.abs(x / r - jx / rho)[m].max()
        ref = max(ref, np.abs(y / r - jy / rho)[m].max())
        assert d["residual"] == pytest.approx(ref, rel=1e-9)
    finally:
        g.close()


def test_bgk_refusals():
    from paper_1912_09327_amd import _capi as C
    from paper_1912_09327_amd.batch import Batch
    from paper_1912_09327_amd.grid import Grid
    g = Grid(32, 32, prec="f32", periodic=3, populations=True, tau=0.9)
    h = Grid(32, 32, prec="f32", periodic=3)
    b = Batch(1 << 26, 2)
    try:
        g.set_geometry(None)
        h.set_geometry(None)
        for call in (lambda: g.set_kernel("strip", vec=2), lambda: g.autotune(),
                     lambda: h.read_populations(), lambda: b.admit(g, 10, -1.0)):
            with pytest.raises(C.Lbt1Error) as e:
                call()
            assert e.value.status == C.EINVAL
        cfg, name = g.kernel()
        assert "bgk" in name
        g.step(3)
    finally:
        b.close()
        g.close()
        h.close()


def test_stability_scan_detects_blow_up():
    """The Re_max sweep's two runners agree at tau = 1 and flag a lid far beyond the
    stable range as unstable (non-finite moments) while a slow lid runs its horizon."""
    from paper_1912_09327_amd import stability as S
    speeds = [0.1, 0.6, 4.0]
    a = S.scan_batched(50, speeds)
    b = S.scan_populations(50, 1.0, speeds, stop_at_first=False)
    assert [bad for _, bad, _ in a] == [bad for _, bad, _ in b]
    assert not a[0][1] and a[0][2] == S.horizon(50, 0.1)
    assert a[-1][1] and b[-1][1]
    c = S.scan_populations(50, 0.7, speeds)
    assert not c[0][1] and c[-1][1]

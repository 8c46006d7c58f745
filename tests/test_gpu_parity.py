"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bars (see gpu_helpers): the state (rho, jx, jy) within 1e-12 (FP64) and 1e-5
(FP32) normwise relative, momentum alone within 1e-12 / 1e-5 of the oracle's
largest momentum (1e-10 / 1e-4 for the named long runs only); FP16/BF16 shifted
storage within 8 ulp of the field's largest magnitude.  Kernel families and launch shapes agree bit for bit.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import JTOL, LONG_JTOL, TOL, field_errors, gpu_run, oracle_run, reduced_bar
from paper_1912_09327_amd import inputs as I

pytestmark = pytest.mark.gpu

GATHER = dict(kernel="gather")


def strip(vec, rows=14, waves=0):
    return dict(kernel="strip", vec=vec, rows=rows, waves=waves)


def _case(kind, nx, ny, seed):
    rng = np.random.default_rng(seed)
    rho, jx, jy = I.random_state(nx, ny, rng)
    if kind == "periodic":
        return None, rho, jx, jy, 3
    if kind == "obstacles":
        return I.random_obstacles(nx, ny, 0.15, rng), rho, jx, jy, 3
    if kind == "cavity":
        flags, r0, x0, y0, _ = I.cavity(nx, 0.08, ny)
        flags[ny // 2, nx // 3] = I.SOLID
        lid = flags == I.FIXED
        rho[lid], jx[lid], jy[lid] = r0[lid], x0[lid], y0[lid]
        return flags, rho, jx, jy, 0
    if kind == "channel":
        flags, per = I.channel(nx, ny)
        return flags, rho, jx, jy, per
    if kind == "open":  # no flags, no periodicity: the domain edge is the wall
        return None, rho, jx, jy, 0
    raise ValueError(kind)


SHAPES = [(3, 3), (17, 9), (64, 32), (70, 45), (130, 33), (256, 31)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kind", ["periodic", "obstacles", "cavity", "channel", "open"])
@pytest.mark.parametrize("wall", ["paper", "halfway"])
def test_f64_gather_matches_oracle(shape, kind, wall):
    nx, ny = shape
    flags, rho, jx, jy, per = _case(kind, nx, ny, nx * 1000 + ny)
    F = (2e-4, -1e-4)
    ref = oracle_run(flags, rho, jx, jy, 40, wall, per, F)
    got = gpu_run(flags, rho, jx, jy, 40, "f64", wall, per, F, kernel=GATHER)
    ex, ej = field_errors(got, ref, flags, (rho, jx, jy))
    assert ex <= TOL["f64"] and ej <= JTOL["f64"], (ex, ej)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind", ["periodic", "obstacles", "cavity", "channel", "open"])
@pytest.mark.parametrize("wall", ["paper", "halfway"])
def test_strip_matches_oracle(prec, kind, wall):
    nx, ny = 264, 61   # several strips in x and y, ragged in both
    flags, rho, jx, jy, per = _case(kind, nx, ny, 7)
    F = (1e-4, 5e-5)
    ref = oracle_run(flags, rho, jx, jy, 30, wall, per, F)
    for vec in (1, 2):
        got = gpu_run(flags, rho, jx, jy, 30, prec, wall, per, F, kernel=strip(vec))
        ex, ej = field_errors(got, ref, flags, (rho, jx, jy))
        assert ex <= TOL[prec] and ej <= JTOL[prec], (vec, ex, ej)


# The FP16 cavity case faulted the GPU once while the (since removed) wall-aware
# strip kernels with 8 columns per lane were built; those variants spilled
# registers to scratch.  Its cause was not shown, so the case stays off the GPU.
FAULTED_REASON = ("faulted the GPU once (suspected: spilling wall-aware 8-column variants, no longer "
                  "built); not re-run until a cause is shown")


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s", "bf16s"])
@pytest.mark.parametrize("kind", ["periodic", "cavity", "channel"])
def test_kernel_families_are_bitwise_identical(prec, kind):
    if (prec, kind) == ("f16s", "cavity"):
        pytest.skip(FAULTED_REASON)
    nx, ny = 512, 77
    flags, rho, jx, jy, per = _case(kind, nx, ny, 11)
    F = (1e-5, 0.0)
    # 8 columns per lane exists for 16-bit storage without walls only
    vecs = {"f64": (1, 2), "f32": (1, 2, 4), "f16s": (1, 2, 4, 8), "bf16s": (1, 2, 4, 8)}[prec]
    if kind != "periodic":
        vecs = tuple(v for v in vecs if v <= 4)
    base = gpu_run(flags, rho, jx, jy, 25, prec, "halfway", per, F, kernel=GATHER)
    for vec in vecs:
        for rows in (6, 14):
            for waves in (0, 8):
                got = gpu_run(flags, rho, jx, jy, 25, prec, "halfway", per, F, kernel=strip(vec, rows, waves))
                for a, b in zip(base, got):
                    assert np.array_equal(a, b), (vec, rows, waves)


# Widths no wider chunk divides (131, 517), or 2 divides but 4 does not (250): on grids
# not periodic in x the last chunk of a row runs into the row padding, whose flags
# are SOLID, so strips of 2 and 4 columns per lane still apply.
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16s"])
@pytest.mark.parametrize("kind", ["cavity", "open", "obstacles_walls"])
@pytest.mark.parametrize("shape", [(131, 45), (517, 33), (250, 20)])
def test_padded_last_chunk_bitwise(prec, kind, shape):
    nx, ny = shape
    if kind == "obstacles_walls":
        rng = np.random.default_rng(nx + ny)
        rho, jx, jy = I.random_state(nx, ny, rng)
        flags, per = I.random_obstacles(nx, ny, 0.15, rng), 2      # walls at x = -1 and x = nx
    else:
        flags, rho, jx, jy, per = _case(kind, nx, ny, nx + ny)
    F = (1e-5, -2e-5)
    base = gpu_run(flags, rho, jx, jy, 21, prec, "halfway", per, F, kernel=GATHER)
    for vec in ((2,) if prec == "f64" else (2, 4)):
        for rows in (6, 14):
            got = gpu_run(flags, rho, jx, jy, 21, prec, "halfway", per, F, kernel=strip(vec, rows))
            for a, b in zip(base, got):
                assert np.array_equal(a, b), (vec, rows)
    if prec == "f64":
        ref = oracle_run(flags, rho, jx, jy, 21, "halfway", per, F)
        ex, ej = field_errors(base, ref, flags, (rho, jx, jy))
        assert ex <= TOL["f64"] and ej <= JTOL["f64"], (ex, ej)


def test_padded_chunk_refused_when_x_is_periodic():
    from paper_1912_09327_amd import _capi as C
    from paper_1912_09327_amd.grid import Grid
    flags, per = I.channel(131, 20)                 # periodic in x, odd width
    g = Grid(131, 20, prec="f32", periodic=per)
    try:
        g.set_geometry(flags)
        for vec in (2, 4):
            with pytest.raises(C.Lbt1Error) as e:
                g.set_kernel("strip", vec=vec, rows=14)
            assert e.value.status == C.EINVAL
        g.set_kernel("strip", vec=1, rows=14)
        g.step(2)
    finally:
        g.close()


@pytest.mark.parametrize("prec", ["f16s", "bf16s"])
@pytest.mark.parametrize("kind", ["periodic", "cavity"])
def test_reduced_precision_within_stated_bar(prec, kind):
    nx, ny = 256, 64
    flags, rho, jx, jy, per = _case(kind, nx, ny, 13)
    ref = oracle_run(flags, rho, jx, jy, 20, "paper", per)
    got = gpu_run(flags, rho, jx, jy, 20, prec, "paper", per, kernel=strip(4))
    m = np.ones(rho.shape, bool) if flags is None else flags == I.FLUID
    er = np.abs(got[0] - ref[0])[m].max()
    ej = max(np.abs(got[1] - ref[1])[m].max(), np.abs(got[2] - ref[2])[m].max())
    bar_d, bar_j = reduced_bar(prec, ref, flags)
    jmax = max(np.abs(ref[1][m]).max(), np.abs(ref[2][m]).max())
    assert er <= bar_d and ej <= bar_j * jmax, (er, bar_d, ej / jmax, bar_j)


@pytest.mark.parametrize("wall", ["paper", "halfway"])
def test_channel_64x32_f64_10000_steps(wall):
    """64 x 32 channel, periodic x, walls on rows 0 and 31, F = 1e-6, 10,000 steps."""
    flags, per = I.channel(64, 32)
    one = np.ones((32, 64))
    zero = np.zeros((32, 64))
    ref = oracle_run(flags, one, zero, zero, 10000, wall, per, (1e-6, 0.0))
    got = gpu_run(flags, one, zero, zero, 10000, "f64", wall, per, (1e-6, 0.0))
    ex, ej = field_errors(got, ref, flags)
    # a named long run: the oracle's own rounding drift over 10,000 steps (measured
    # 6.8e-13 paper, 5.5e-12 half-way) is above the 1e-12 bar of short runs
    assert ex <= TOL["f64"] and ej <= LONG_JTOL["f64"], (ex, ej)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cavity_256_matches_oracle(prec):
    """256 x 256 lid-driven cavity, u_lid = 0.1 (shortened to 3,000 steps here; the full
    50,000-step run is compared in test_gpu_full)."""
    flags, rho, jx, jy, per = I.cavity(256, 0.1)
    ref = oracle_run(flags, rho, jx, jy, 3000, "paper", per)
    got = gpu_run(flags, rho, jx, jy, 3000, prec, "paper", per)
    ex, ej = field_errors(got, ref, flags)
    # a named long run (measured: FP32 1.7e-5 of max |j| after 3,000 steps)
    assert ex <= TOL[prec] and ej <= LONG_JTOL[prec], (ex, ej)


def test_codec_round_trip_and_rounding():
    """set_geometry then read_moments returns the stored (rounded) values; binary16 and
    bfloat16 round to nearest even."""
    rng = np.random.default_rng(3)
    nx, ny = 67, 5
    rho = 1 + 1e-2 * rng.standard_normal((ny, nx))
    jx = 1e-2 * rng.standard_normal((ny, nx))
    jy = 1e-2 * rng.standard_normal((ny, nx))
    got = gpu_run(None, rho, jx, jy, 0, "f64", periodic=3)
    assert all(np.array_equal(a, b) for a, b in zip(got, (1 + (rho - 1), jx, jy)))
    got = gpu_run(None, rho, jx, jy, 0, "f32", periodic=3)
    assert np.array_equal(got[1], jx.astype(np.float32).astype(np.float64))
    assert np.array_equal(got[0], (rho - 1).astype(np.float32).astype(np.float64) + 1)
    got = gpu_run(None, rho, jx, jy, 0, "f16s", periodic=3)
    assert np.array_equal(got[1], jx.astype(np.float16).astype(np.float64))
    got = gpu_run(None, rho, jx, jy, 0, "f16s", periodic=3, scale=(2.0 ** -8, 2.0 ** -6))
    assert np.array_equal(got[1], (jx * 2.0 ** 6).astype(np.float16).astype(np.float64) * 2.0 ** -6)
    got = gpu_run(None, rho, jx, jy, 0, "bf16s", periodic=3)
    b = jx.astype(np.float32).view(np.uint32).astype(np.uint64)
    # round half to even on the upper 16 bits (the float32 intermediate is exact enough
    # here: these values are not within 2^-24 of a bfloat16 tie)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    assert np.array_equal(got[1], r.astype(np.uint32).view(np.float32).astype(np.float64))


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
def test_reductions_match_oracle(prec):
    flags, rho, jx, jy, per = _case("cavity", 200, 150, 5)
    from paper_1912_09327_amd.grid import Grid
    g = Grid(200, 150, prec=prec, periodic=per)
    g.set_geometry(flags, rho, jx, jy)
    snap = g.read_moments()
    g.step(7)
    d = g.reduce()
    cur = g.read_moments()
    g.close()
    ref = oracle.reduce(*cur, flags=flags, snapshot=snap)
    assert d["fluid"] == ref["fluid"]
    assert d["nonfinite"] == 0
    assert d["mass"] == pytest.approx(ref["mass"], rel=1e-14)
    assert d["mom_x"] == pytest.approx(ref["mom_x"], rel=1e-12, abs=1e-14)
    assert d["mom_y"] == pytest.approx(ref["mom_y"], rel=1e-12, abs=1e-14)
    assert d["residual"] == pytest.approx(ref["residual"], rel=1e-12)


def test_residual_snapshot_cadence():
    """The residual compares with the state at the previous residual call."""
    flags, rho, jx, jy, per = I.cavity(96, 0.1)
    from paper_1912_09327_amd.grid import Grid
    g = Grid(96, 96, prec="f64")
    g.set_geometry(flags, rho, jx, jy)
    g.step(100)
    r1 = g.reduce(4)["residual"]
    s1 = g.read_moments()
    g.step(100)
    r2 = g.reduce(4)["residual"]
    cur = g.read_moments()
    g.close()
    assert r1 > 0
    assert r2 == pytest.approx(oracle.reduce(*cur, flags=flags, snapshot=s1)["residual"], rel=1e-12)


def test_error_paths():
    from paper_1912_09327_amd import _capi as C
    from paper_1912_09327_amd.grid import Grid
    g = Grid(16, 16, prec="f32")
    with pytest.raises(C.Lbt1Error) as e:
        g.step(1)
    assert e.value.status == C.ESTATE
    bad = np.zeros((16, 16), np.uint8)
    bad[3, 3] = 7
    with pytest.raises(C.Lbt1Error) as e:
        g.set_geometry(bad)
    assert e.value.status == C.EINVAL
    with pytest.raises(C.Lbt1Error) as e:
        g.set_geometry(None, -np.ones((16, 16)))
    assert e.value.status == C.EINVAL
    lid = np.zeros((16, 16), np.uint8)
    lid[-1] = C.FIXED
    with pytest.raises(C.Lbt1Error) as e:
        g.set_geometry(lid)
    assert e.value.status == C.EINVAL
    g.set_geometry(None)
    with pytest.raises(C.Lbt1Error) as e:
        g.set_kernel("strip", vec=3)
    assert e.value.status == C.EINVAL
    g.step(3)
    g.close()


def test_deterministic_and_step_splitting():
    """Repeat runs agree bit for bit; n steps at once equal n split across calls and graph bursts."""
    flags, rho, jx, jy, per = _case("cavity", 300, 100, 17)
    a = gpu_run(flags, rho, jx, jy, 150, "f32", "paper", per)
    b = gpu_run(flags, rho, jx, jy, 150, "f32", "paper", per)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    from paper_1912_09327_amd.grid import Grid
    g = Grid(300, 100, prec="f32", periodic=per)
    g.set_geometry(flags, rho, jx, jy)
    for n in (1, 64, 5, 80):
        g.step(n)
    c = g.read_moments()
    g.close()
    assert all(np.array_equal(x, y) for x, y in zip(a, c))

"""GPU tests of the batched engine and the server (through the C ABI).

Alone vs in the mix: every grid stepped inside a batch (one fused launch per
step for all resident grids, HIP-graph bursts) must end bit for bit where the
same grid ends when stepped by itself with lbt1_step.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import JTOL, TOL, field_errors
from paper_1912_09327_amd import inputs as I

pytestmark = pytest.mark.gpu


def _grid(spec, prec):
    from paper_1912_09327_amd.grid import Grid
    kind, L, param = spec
    if kind == "cavity":
        flags, rho, jx, jy, per = I.cavity(L, param)
        F = (0.0, 0.0)
    else:
        flags, per, _ = I.porous_channel(L, np.random.default_rng(L), porosity=param)
        rho = jx = jy = None
        F = (I.channel_force_for(0.05, L), 0.0)
    g = Grid(L, L, prec=prec, periodic=per, force=F)
    g.set_geometry(flags, rho, jx, jy)
    return g, (flags, rho, jx, jy, per, F)


# odd widths 147 and 261 are not periodic in x: their strips take 2 and 4 columns
# per lane with the last chunk of a row running into the (SOLID) row padding.  In
# the four-column class 256 is one strip wide, 517 three strips (the last of three
# chunks) and 362 two.
SPECS = [("cavity", 37, 0.08), ("cavity", 64, 0.05), ("channel", 96, 0.8), ("cavity", 130, 0.1),
         ("channel", 200, 0.7), ("cavity", 256, 0.03), ("cavity", 147, 0.07), ("cavity", 261, 0.05),
         ("cavity", 362, 0.04), ("cavity", 517, 0.02)]
BUDGETS = [130, 250, 75, 300, 260, 190, 121, 97, 101, 66]


@pytest.mark.parametrize("prec", ["f32", "f16s", "bf16s"])
def test_batch_alone_vs_mix_bitwise(prec):
    from paper_1912_09327_amd.batch import Batch
    b = Batch(1 << 30, 16)
    grids = []
    for spec, budget in zip(SPECS, BUDGETS):
        g, geo = _grid(spec, prec)
        slot = b.admit(g, budget, -1.0)
        assert slot is not None
        grids.append((g, geo, budget, slot))
    for _ in range(10):
        b.run(40)
        if len(b.poll()) == len(grids):
            break
    assert len(b.poll()) == len(grids)
    for g, geo, budget, slot in grids:
        state, steps, _ = b.slot_info(slot)
        assert steps == budget
        b.evict(slot)
        mix = g.read_moments()
        g.close()
        flags, rho, jx, jy, per, F = geo
        from paper_1912_09327_amd.grid import Grid
        h = Grid(flags.shape[1], flags.shape[0], prec=prec, periodic=per, force=F)
        h.set_geometry(flags, rho, jx, jy)
        h.set_kernel("gather")           # one thread per node: no chunks, no padding
        h.step(budget)
        alone = h.read_moments()
        h.close()
        for a, c in zip(mix, alone):
            assert np.array_equal(a, c), (geo[0].shape, budget)
    b.close()


def _run_mix_and_compare(prec, shape=None, burst=40, tune=False):
    """Run SPECS with BUDGETS in one batch (the given tile shape, or the autotuner's
    choice after two bursts) and compare every grid with the gather kernel alone."""
    from paper_1912_09327_amd.batch import Batch
    from paper_1912_09327_amd.grid import Grid
    b = Batch(1 << 30, 16)
    if shape is not None:
        b.set_shape(*shape)
    grids = []
    for spec, budget in zip(SPECS, BUDGETS):
        g, geo = _grid(spec, prec)
        slot = b.admit(g, budget, -1.0)
        assert slot is not None
        grids.append((g, geo, budget, slot))
    got_shape = None
    for k in range(40):
        if tune and k == 2:
            got_shape, ms = b.autotune(burst_steps=20, reps=2)
            assert ms > 0
        b.run(burst)
        if len(b.poll()) == len(grids):
            break
    assert len(b.poll()) == len(grids)
    for g, geo, budget, slot in grids:
        state, steps, _ = b.slot_info(slot)
        assert steps == budget
        b.evict(slot)
        mix = g.read_moments()
        g.close()
        flags, rho, jx, jy, per, F = geo
        h = Grid(flags.shape[1], flags.shape[0], prec=prec, periodic=per, force=F)
        h.set_geometry(flags, rho, jx, jy)
        h.set_kernel("gather")
        h.step(budget)
        alone = h.read_moments()
        h.close()
        for a, c in zip(mix, alone):
            assert np.array_equal(a, c), (shape, got_shape, geo[0].shape, budget)
    b.close()
    return got_shape


# tile shapes: fuse mode, strip heights of the five classes (one step at 1, 2, 4
# columns per lane; two steps at 2; resident in LDS) and LDS residency of small grids
SHAPES = [(1, (6, 6, 6, 2, 0), 0), (1, (14, 14, 14, 6, 0), 0), (2, (6, 14, 6, 14, 0), 0), (1, (0, 0, 0, 30, 0), 0),
          (0, (14, 6, 14, 0, 0), 0), (0, (0, 0, 0, 0, 6), 1), (1, (6, 6, 6, 14, 14), 1), (0, (6, 14, 6, 0, 0), 0),
          (2, (14, 14, 14, 6, 0), 0), (0, (14, 14, 14, 0, 0), 0, 2), (2, (6, 6, 6, 30, 0), 0, 1),
          (0, (30, 30, 30, 0, 0), 0), (2, (0, 0, 30, 14, 0), 0)]


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s", "bf16s"])
@pytest.mark.parametrize("shape", SHAPES)
def test_batch_tile_shapes_alone_vs_mix_bitwise(prec, shape):
    """Every tile shape, odd budgets, bursts of an odd number of steps (the fused class
    then ends a burst with a single step): the bits of each grid alone."""
    if prec == "f64" and 30 in shape[1][:4]:
        pytest.skip("FP64 strips of 30 rows are not built")
    _run_mix_and_compare(prec, shape, burst=33)


@pytest.mark.parametrize("prec", ["f32", "f16s"])
def test_batch_autotune_keeps_state_and_bits(prec):
    """The autotuner times shapes on the resident grids' memory and restores it: after
    it the batch still ends every grid where the grid alone ends."""
    shape = _run_mix_and_compare(prec, None, burst=40, tune=True)
    assert shape["fuse"] in (0, 1, 2) and shape["lds"] in (0, 1) and len(shape["rows"]) == 5
    assert shape["vec_cap"] in (1, 2, 4)


def test_batch_shape_refusals():
    from paper_1912_09327_amd import _capi as C
    from paper_1912_09327_amd.batch import Batch
    b = Batch(1 << 28, 4)
    try:
        for bad in ((3, (0, 0, 0, 0)), (0, (7, 0, 0, 0)), (1, (0, 0, 0, 22)), (0, (0, 0, 0, 0, 22)),
                    (0, (0, 0, 0, 0), 2), (0, (0, 0, 0, 0), 0, 3)):
            with pytest.raises(C.Lbt1Error) as e:
                b.set_shape(*bad)
            assert e.value.status == C.EINVAL
        with pytest.raises(C.Lbt1Error) as e:
            b.autotune()
        assert e.value.status == C.ESTATE          # nothing resident
    finally:
        b.close()


def test_batch_f64_matches_oracle():
    from paper_1912_09327_amd.batch import Batch
    b = Batch(1 << 30, 4)
    items = []
    for spec in (("cavity", 40, 0.1), ("channel", 48, 0.8)):
        g, geo = _grid(spec, "f64")
        items.append((g, geo, b.admit(g, 230, -1.0)))
    while len(b.poll()) < 2:
        b.run(64)
    for g, (flags, rho, jx, jy, per, F), slot in items:
        b.evict(slot)
        got = g.read_moments()
        g.close()
        n = flags.shape[0]
        rho = np.ones((n, n)) if rho is None else rho
        jx = np.zeros((n, n)) if jx is None else jx
        jy = np.zeros((n, n)) if jy is None else jy
        ref = oracle.run(rho, jx, jy, 230, flags, per, F, oracle.WALL_PAPER)
        ex, ej = field_errors(got, ref, flags)
        assert ex <= TOL["f64"] and ej <= JTOL["f64"], (ex, ej)
    b.close()


def test_batch_admission_limits_and_eviction():
    from paper_1912_09327_amd.batch import Batch
    from paper_1912_09327_amd import _capi as C
    g1, _ = _grid(("cavity", 64, 0.05), "f16s")
    g2, _ = _grid(("cavity", 64, 0.05), "f16s")
    g3, _ = _grid(("cavity", 64, 0.05), "f16s")
    need = C.grid_bytes(64, 64, C.F16S)
    b = Batch(2 * need, 8)                          # budget for two
    s1, s2 = b.admit(g1, 10, -1), b.admit(g2, 10, -1)
    assert s1 is not None and s2 is not None
    assert b.admit(g3, 10, -1) is None              # EBUSY: budget
    b.evict(s1)
    s3 = b.admit(g3, 10, -1)
    assert s3 is not None
    b.close()
    b = Batch(1 << 30, 1)                           # one slot
    assert b.admit(g1, 10, -1) is not None
    assert b.admit(g2, 10, -1) is None              # EBUSY: slots
    with pytest.raises(C.Lbt1Error) as e:
        g1.step(1)                                  # resident grids are stepped by the batch only
    assert e.value.status == C.ESTATE
    b.close()
    for g in (g1, g2, g3):
        g.close()


def test_convergence_and_nonfinite_isolation():
    """A grid that blows up is reported non-finite and stops; a grid that reaches its
    residual tolerance stops early; neither disturbs the others."""
    from paper_1912_09327_amd.batch import Batch
    from paper_1912_09327_amd import _capi as C
    from paper_1912_09327_amd.serve import GpuBackend
    b = Batch(1 << 30, 8)
    bad, _ = _grid(("cavity", 24, 2.0), "f32")          # lid far beyond the stable range
    calm, calm_geo = _grid(("cavity", 24, 0.01), "f32")
    other, other_geo = _grid(("cavity", 80, 0.05), "f32")
    sb, sc, so = b.admit(bad, 5000, -1), b.admit(calm, 200000, 1e-7), b.admit(other, 1600, -1)
    for _ in range(2000):
        b.run(100)
        if len(b.poll()) == 3:
            break
    st_b, steps_b, _ = b.slot_info(sb)
    st_c, steps_c, res_c = b.slot_info(sc)
    st_o, steps_o, _ = b.slot_info(so)
    assert st_b == C.SLOT_NONFINITE and steps_b < 5000
    assert st_c == C.SLOT_CONVERGED and res_c <= 1e-7 and steps_c < 200000 and steps_c % 100 == 0
    assert st_o == C.SLOT_BUDGET and steps_o == 1600
    for s in (sb, sc, so):
        b.evict(s)
    # the same grids alone, with the same residual checks every 100 steps
    be = GpuBackend(1 << 30, 1, prec="f32")
    for g, geo, tol, budget, steps in ((calm, calm_geo, 1e-7, 200000, steps_c), (other, other_geo, -1, 1600, 1600)):
        mix = g.read_moments()
        from paper_1912_09327_amd.grid import Grid
        flags, rho, jx, jy, per, F = geo
        h = Grid(flags.shape[1], flags.shape[0], prec="f32", periodic=per, force=F)
        h.set_geometry(flags, rho, jx, jy)
        state, n, _ = be.run_alone(h, budget, tol, 100)
        assert n == steps
        for a, c in zip(mix, h.read_moments()):
            assert np.array_equal(a, c)
        h.close()
    be.close()
    b.close()
    for g in (bad, calm, other):
        g.close()


def test_graph_bursts_replayed_with_host_updates_between():
    """The burst graph is replayed many times with descriptor updates and admissions in
    between; every replay must give what single steps give."""
    from paper_1912_09327_amd.batch import Batch
    from paper_1912_09327_amd.grid import Grid
    b = Batch(1 << 30, 8)
    g1, geo1 = _grid(("cavity", 50, 0.1), "f32")
    s1 = b.admit(g1, 1000, -1)
    b.run(25)
    g2, geo2 = _grid(("channel", 70, 0.8), "f32")      # admitted between replays
    s2 = b.admit(g2, 1000, -1)
    for _ in range(8):
        b.run(25)
    for g, geo, s, n in ((g1, geo1, s1, 225), (g2, geo2, s2, 200)):
        assert b.slot_info(s)[1] == n
        b.evict(s)
        flags, rho, jx, jy, per, F = geo
        h = Grid(flags.shape[1], flags.shape[0], prec="f32", periodic=per, force=F)
        h.set_geometry(flags, rho, jx, jy)
        h.step(n)
        for a, c in zip(g.read_moments(), h.read_moments()):
            assert np.array_equal(a, c)
        h.close()
        g.close()
    b.close()


def test_server_results_equal_alone_results():
    """Continuous-batching server and plain FIFO on the same small request stream: every
    result is bit for bit the same; latencies and throughput are reported."""
    from paper_1912_09327_amd.serve import GpuBackend, PlainFifo, Request, Server, summarize
    rng = np.random.default_rng(11)
    reqs = []
    for i in range(10):
        reqs.append(Request(id=i, arrival=0.002 * i, kind="cavity" if i % 2 else "channel",
                            L=int(rng.integers(32, 100)), steps=int(rng.integers(200, 900)), u=0.05,
                            porosity=0.8, seed=i, tol=-1.0 if i % 3 else 1e-9))
    be = GpuBackend(1 << 30, 4, prec="f16s")
    mix = {r.id: r for r in Server(be, 1 << 30, 4, burst=100, keep_results=True).serve(reqs)}
    be.close()
    be = GpuBackend(1 << 30, 1, prec="f16s")
    alone = {r.id: r for r in PlainFifo(be, burst=100, keep_results=True).serve(reqs)}
    be.close()
    assert set(mix) == set(alone) == set(range(10))
    for i in mix:
        assert mix[i].steps == alone[i].steps and mix[i].state == alone[i].state
        for a, c in zip(mix[i].moments, alone[i].moments):
            assert np.array_equal(a, c)
    s = summarize(list(mix.values()))
    assert s["p99_s"] >= s["p50_s"] > 0 and s["mlups"] > 0

"""lbt1_reduce_noalloc (the allocation-free variant of lbt1_reduce, for callers that
cannot allocate) through the C ABI against lbt1_reduce on twin grids: the same
slots bit for bit, on two calls in a row, the second on a smaller grid, with the
snapshot refresh of the residual and the what-mask behaviour of lbt1_reduce."""
import sys

import numpy as np
import pytest

from paper_1912_09327_amd import _capi as C
from paper_1912_09327_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _twins(nx, ny, prec, seed):
    from paper_1912_09327_amd.grid import Grid
    rng = np.random.default_rng(seed)
    flags, r0, x0, y0, per = I.cavity(nx, 0.08, ny)
    flags[ny // 3, nx // 4] = I.SOLID
    rho, jx, jy = I.random_state(nx, ny, rng)
    lid = flags == I.FIXED
    rho[lid], jx[lid], jy[lid] = r0[lid], x0[lid], y0[lid]
    out = []
    for _ in range(2):
        g = Grid(nx, ny, prec=prec, periodic=per, force=(1e-5, 0.0))
        g.set_geometry(flags, rho, jx, jy)
        out.append(g)
    return out


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
def test_noalloc_reduce_equals_reduce_on_two_calls_second_smaller(prec):
    import torch
    sizes = [(1030, 700), (70, 45)]                  # the second input is smaller
    pairs = [_twins(nx, ny, prec, i) for i, (nx, ny) in enumerate(sizes)]
    try:
        for a, b in pairs:
            a.step(37)
            b.step(37)
        refs = [a.reduce(C.REDUCE_ALL) for a, _ in pairs]
        outs = [torch.full((C.REDUCE_SLOTS,), -7.0, dtype=torch.float64, device="cuda") for _ in pairs]
        _say(f"[no-alloc] {prec}: two calls in a row, grids {sizes}")
        for (_, b), o in zip(pairs, outs):
            b.reduce_noalloc(o.data_ptr(), C.REDUCE_ALL)
        for _, b in pairs:
            b.sync()
        keys = ["mass", "mom_x", "mom_y", "residual", "nonfinite", "fluid"]
        for ref, o, (nx, ny) in zip(refs, outs, sizes):
            got = o.cpu().numpy()
            want = np.array([ref[k] for k in keys], dtype=np.float64)
            assert np.array_equal(got, want), (nx, ny, got, want)
        # the residual refreshed both snapshots alike: step on and compare again
        for a, b in pairs:
            a.step(11)
            b.step(11)
        refs = [a.reduce(C.REDUCE_RESIDUAL | C.REDUCE_MASS) for a, _ in pairs]
        for o in outs:
            o.fill_(-7.0)
        for (_, b), o in zip(pairs, outs):
            b.reduce_noalloc(o.data_ptr(), C.REDUCE_RESIDUAL | C.REDUCE_MASS)
        for _, b in pairs:
            b.sync()
        for ref, o in zip(refs, outs):
            got = o.cpu().numpy()
            assert got[0] == ref["mass"] and got[3] == ref["residual"] and got[5] == ref["fluid"]
            assert (got[[1, 2, 4]] == -7.0).all()          # slots not asked for are untouched
            assert ref["residual"] > 0
    finally:
        for pair in pairs:
            for g in pair:
                g.close()


def test_noalloc_reduce_refusals():
    from paper_1912_09327_amd.grid import Grid
    import torch
    o = torch.zeros(C.REDUCE_SLOTS, dtype=torch.float64, device="cuda")
    g = Grid(64, 32, prec="f32", periodic=3, snapshot=False)
    try:
        with pytest.raises(C.Lbt1Error) as e:
            g.reduce_noalloc(o.data_ptr())
        assert e.value.status == C.ESTATE                 # before set_geometry
        g.set_geometry(None)
        with pytest.raises(C.Lbt1Error) as e:
            g.reduce_noalloc(o.data_ptr(), C.REDUCE_RESIDUAL)
        assert e.value.status == C.EINVAL                 # no snapshot
        with pytest.raises(C.Lbt1Error) as e:
            g.reduce_noalloc(o.data_ptr(), 16)
        assert e.value.status == C.EINVAL
        g.reduce_noalloc(o.data_ptr(), C.REDUCE_MASS)
        g.sync()
        assert o[5].item() == 64 * 32 and o[0].item() == 64 * 32
    finally:
        g.close()

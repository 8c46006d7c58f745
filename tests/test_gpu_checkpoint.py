"""Checkpoint and resume: n steps, save the state, start a new grid from it and take
n more steps -- the result equals 2n steps in one grid, bit for bit, in every
storage format.  Through lbt1_save_state / lbt1_load_state (the stored bits) in all
four formats; through lbt1_read_moments / lbt1_set_geometry in FP32, FP16 and
BF16, whose round trip through rho = 1 + (rho - 1) in FP64 is exact (in FP64 it
rounds, which is why the exact calls exist)."""
import numpy as np
import pytest

from paper_1912_09327_amd import inputs as I

pytestmark = pytest.mark.gpu


def _case(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "periodic":
        rho, jx, jy = I.random_periodic(n, n, seed=seed)
        return None, rho, jx, jy, 3, (0.0, 0.0)
    flags, rho, jx, jy, per = I.cavity(n, 0.08)
    flags[n // 3, n // 2] = I.SOLID
    r, u, v = I.random_state(n, n, rng, 1e-3, 1e-2)
    fl = flags == I.FLUID
    rho[fl], jx[fl], jy[fl] = r[fl], u[fl], v[fl]
    return flags, rho, jx, jy, per, (1e-5, -2e-5)


@pytest.mark.parametrize("prec", ["f32", "f16s", "bf16s"])
@pytest.mark.parametrize("kind", ["periodic", "cavity"])
def test_resume_from_read_back_moments_is_bitwise(prec, kind):
    from paper_1912_09327_amd.grid import Grid
    n, steps = 136, 77                  # an odd count: fused launches end in a remainder
    flags, rho, jx, jy, per, F = _case(kind, n, 9)

    def fresh(state):
        g = Grid(n, n, prec=prec, periodic=per, force=F)
        g.set_geometry(flags, *state)
        return g

    whole = fresh((rho, jx, jy))
    whole.step(2 * steps)
    want = whole.read_moments()
    whole.close()
    first = fresh((rho, jx, jy))
    first.step(steps)
    mid = first.read_moments()
    first.close()
    second = fresh(mid)
    assert all(np.array_equal(a, b) for a, b in zip(second.read_moments(), mid))   # exact round trip
    second.step(steps)
    got = second.read_moments()
    second.close()
    for a, b in zip(got, want):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s", "bf16s"])
@pytest.mark.parametrize("kind", ["periodic", "cavity"])
def test_resume_from_saved_state_is_bitwise(prec, kind):
    from paper_1912_09327_amd import _capi as C
    from paper_1912_09327_amd.grid import Grid
    n, steps = 136, 77
    flags, rho, jx, jy, per, F = _case(kind, n, 9)

    def fresh():
        g = Grid(n, n, prec=prec, periodic=per, force=F)
        g.set_geometry(flags, rho, jx, jy)
        return g

    whole = fresh()
    whole.step(steps)
    r1 = whole.reduce()                   # refreshes the snapshot at step n
    whole.step(steps)
    want = whole.read_moments()
    r2 = whole.reduce()
    whole.close()
    first = fresh()
    first.step(steps)
    first.reduce()
    state = first.save_state()
    first.close()
    second = Grid(n, n, prec=prec, periodic=per, force=F)
    second.set_geometry(flags, rho, jx, jy)   # geometry first, then the saved bits
    second.load_state(state)
    with pytest.raises(C.Lbt1Error):
        second.load_state(state[:-1])
    second.step(steps)
    got = second.read_moments()
    g2 = second.reduce()
    second.close()
    for a, b in zip(got, want):
        assert np.array_equal(a, b)
    assert g2["residual"] == r2["residual"] and g2["mass"] == r2["mass"]   # the snapshot came along
    assert r1["fluid"] == g2["fluid"]

"""CPU oracle for the LBMTau1 D2Q9 step -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's ``cpu_baseline`` leg
may import this package.  The GPU library and its Python binding never do,
and this package never imports them.

Contents
--------
* ``lbt1_oracle.c`` (wrapped here): the moments-only LBMTau1 step in plain
  FP64, following Algorithm 1 of section 2.1 in the paper's direction order,
  and its multiphase form with the Shan-Chen force of Eq. f_sc
  (``run(..., sc=(G, rho0))``, ``sc_force``).
* ``lbt1_oracle3d.c`` (wrapped here): the same step on the 3-D lattices of the
  paper's memory analysis, D3Q19 and D3Q27 (``run3``, ``tables3``).
* ``bgk``: brute-force stored-population BGK (Eq. lbm) with streaming and
  bounce-back, any tau; at tau = 1 it must agree with the moments-only step
  (Eq. LBMTau1).
* ``closed_forms``: Poiseuille profiles, the shear-wave decay factor, the
  exact one-dimensional recurrence, error and memory formulas.

Every function here is pinned by ``tests/test_oracle_pins.py`` against values
fixed by the paper or by mathematics; the pins are listed in the test file.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# A test that plants mistakes in a copy of the oracle points this at its build.
_LIB_PATH = os.environ.get("LBT1_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
_lib = None

FLUID, SOLID, FIXED = 0, 1, 2
WALL_PAPER, WALL_HALFWAY = 0, 1

_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    default = _LIB_PATH == os.path.join(HERE, "liboracle.so")
    if default and (not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < max(
            os.path.getmtime(os.path.join(HERE, f)) for f in ("lbt1_oracle.c", "lbt1_oracle3d.c"))):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_feq.restype = ctypes.c_double
    lib.oracle_feq.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.oracle_tables.argtypes = [ctypes.POINTER(ctypes.c_int)] * 3 + [_dp]
    lib.oracle_step.restype = ctypes.c_int
    lib.oracle_step.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint, _u8p,
                                ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                _dp, _dp, _dp, _dp, _dp, _dp]
    lib.oracle_run.restype = ctypes.c_int
    lib.oracle_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint, _u8p,
                               ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_long,
                               _dp, _dp, _dp]
    lib.oracle_reduce.restype = ctypes.c_int
    lib.oracle_reduce.argtypes = [ctypes.c_int, ctypes.c_int, _u8p, _dp, _dp, _dp,
                                  _dp, _dp, _dp, _dp]
    lib.oracle_run_sc.restype = ctypes.c_int
    lib.oracle_run_sc.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint, _u8p,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_int, ctypes.c_long, _dp, _dp, _dp]
    lib.oracle_sc_force.restype = ctypes.c_int
    lib.oracle_sc_force.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint, _u8p,
                                    ctypes.c_double, ctypes.c_double, _dp, _dp, _dp]
    lib.oracle_sc_psi.restype = ctypes.c_double
    lib.oracle_sc_psi.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.oracle3_tables.restype = ctypes.c_int
    lib.oracle3_tables.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), _dp]
    lib.oracle3_run.restype = ctypes.c_int
    lib.oracle3_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint, _u8p,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_long,
                                _dp, _dp, _dp, _dp]
    lib.oracle3_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_get_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _use_library(path):
    """Load the oracle from another build of the same source (tests that plant
    mistakes in a copy of the oracle use this); ``None`` restores the default."""
    global _lib, _LIB_PATH
    _lib = None
    _LIB_PATH = path or os.path.join(HERE, "liboracle.so")
    return _load()


def _f64(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _flags(flags, shape):
    if flags is None:
        return None
    f = np.ascontiguousarray(flags, dtype=np.uint8)
    if f.shape != shape:
        raise ValueError(f"flags: expected shape {shape}, got {f.shape}")
    return f


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _fptr(f):
    return None if f is None else f.ctypes.data_as(_u8p)


def tables():
    """(ex, ey, inv, w) of the oracle's D2Q9 lattice (section 2)."""
    lib = _load()
    ex = (ctypes.c_int * 9)()
    ey = (ctypes.c_int * 9)()
    inv = (ctypes.c_int * 9)()
    w = (ctypes.c_double * 9)()
    lib.oracle_tables(ex, ey, inv, w)
    return list(ex), list(ey), list(inv), list(w)


def feq(k, r, u, v):
    """Eq. maxwellboltzmann for direction k."""
    return _load().oracle_feq(int(k), float(r), float(u), float(v))


def set_threads(n):
    _load().oracle_set_threads(int(n))
    _load().oracle3_set_threads(int(n))


def get_threads():
    return _load().oracle_get_threads()


def step(rho, jx, jy, flags=None, periodic=0, force=(0.0, 0.0), wall=WALL_PAPER):
    """One LBMTau1 step (Algorithm 1).  Arrays are [ny, nx]; returns new (rho, jx, jy)."""
    rho = np.asarray(rho)
    shape = rho.shape
    ny, nx = shape
    r, u, v = _f64(rho, shape), _f64(jx, shape), _f64(jy, shape)
    f = _flags(flags, shape)
    ro, uo, vo = np.empty(shape), np.empty(shape), np.empty(shape)
    rc = _load().oracle_step(nx, ny, int(periodic), _fptr(f), float(force[0]), float(force[1]),
                             int(wall), _ptr(r), _ptr(u), _ptr(v), _ptr(ro), _ptr(uo), _ptr(vo))
    if rc:
        raise ValueError(f"oracle_step failed ({rc})")
    return ro, uo, vo


def run(rho, jx, jy, nsteps, flags=None, periodic=0, force=(0.0, 0.0), wall=WALL_PAPER, sc=None):
    """``nsteps`` LBMTau1 steps; returns new (rho, jx, jy) (inputs untouched).
    ``sc=(G, rho0)``: multiphase steps with the Shan-Chen force."""
    rho = np.asarray(rho)
    shape = rho.shape
    ny, nx = shape
    r = np.array(_f64(rho, shape), copy=True)
    u = np.array(_f64(jx, shape), copy=True)
    v = np.array(_f64(jy, shape), copy=True)
    f = _flags(flags, shape)
    if sc is None:
        rc = _load().oracle_run(nx, ny, int(periodic), _fptr(f), float(force[0]), float(force[1]),
                                int(wall), int(nsteps), _ptr(r), _ptr(u), _ptr(v))
    else:
        rc = _load().oracle_run_sc(nx, ny, int(periodic), _fptr(f), float(force[0]), float(force[1]),
                                   float(sc[0]), float(sc[1]), int(wall), int(nsteps),
                                   _ptr(r), _ptr(u), _ptr(v))
    if rc:
        raise ValueError(f"oracle_run failed ({rc})")
    return r, u, v


def sc_psi(rho, rho0=1.0):
    return _load().oracle_sc_psi(float(rho), float(rho0))


def sc_force(rho, flags=None, periodic=0, G=-5.0, rho0=1.0):
    """Shan-Chen force (Fx, Fy) of every node for density ``rho``."""
    rho = np.asarray(rho)
    shape = rho.shape
    ny, nx = shape
    r = _f64(rho, shape)
    f = _flags(flags, shape)
    FX, FY = np.empty(shape), np.empty(shape)
    rc = _load().oracle_sc_force(nx, ny, int(periodic), _fptr(f), float(G), float(rho0), _ptr(r), _ptr(FX), _ptr(FY))
    if rc:
        raise ValueError("oracle_sc_force failed")
    return FX, FY


def reduce(rho, jx, jy, flags=None, snapshot=None):
    """FP64 diagnostics over FLUID nodes.

    Returns dict(mass, mom_x, mom_y, residual, nonfinite, fluid); ``residual`` is
    max |u - u_snap| over nodes and components with u = j / rho, 0 without a snapshot.
    """
    rho = np.asarray(rho)
    shape = rho.shape
    ny, nx = shape
    r, u, v = _f64(rho, shape), _f64(jx, shape), _f64(jy, shape)
    f = _flags(flags, shape)
    out = np.zeros(6)
    if snapshot is not None:
        sr, su, sv = (_f64(a, shape) for a in snapshot)
        sp = (_ptr(sr), _ptr(su), _ptr(sv))
    else:
        sp = (None, None, None)
    rc = _load().oracle_reduce(nx, ny, _fptr(f), _ptr(r), _ptr(u), _ptr(v), *sp, _ptr(out))
    if rc:
        raise ValueError("oracle_reduce failed")
    return dict(mass=out[0], mom_x=out[1], mom_y=out[2], residual=out[3],
                nonfinite=int(out[4]), fluid=int(out[5]))


def tables3(q):
    """(e [q, 3], w [q]) of the oracle's D3Q19 or D3Q27 lattice."""
    e = (ctypes.c_int * 81)()
    w = (ctypes.c_double * 27)()
    n = _load().oracle3_tables(int(q), e, w)
    if n < 0:
        raise ValueError(q)
    return np.array(list(e)[:3 * n]).reshape(n, 3), np.array(list(w)[:n])


def run3(rho, jx, jy, jz, nsteps, q=19, flags=None, periodic=0, force=(0.0, 0.0, 0.0), wall=WALL_PAPER):
    """``nsteps`` 3-D LBMTau1 steps on [nz, ny, nx] arrays; returns (rho, jx, jy, jz).
    periodic: bit 0 x, bit 1 y, bit 2 z."""
    rho = np.asarray(rho)
    shape = rho.shape
    nz, ny, nx = shape
    st = [np.array(_f64(a, shape), copy=True) for a in (rho, jx, jy, jz)]
    f = _flags(flags, shape)
    rc = _load().oracle3_run(int(q), nx, ny, nz, int(periodic), _fptr(f), float(force[0]), float(force[1]),
                             float(force[2]), int(wall), int(nsteps), *[_ptr(a) for a in st])
    if rc:
        raise ValueError(f"oracle3_run failed ({rc})")
    return tuple(st)

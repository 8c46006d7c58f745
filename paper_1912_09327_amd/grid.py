"""Python handle for one LBMTau1 grid on the GPU (thin wrapper over the C ABI).

PyTorch provides the device memory (a ``torch.uint8`` tensor of
``lbt1_grid_bytes`` bytes) and the stream; the library does everything else.
"""
import ctypes

import numpy as np

from . import _capi as C

_default_stream = None


def default_stream():
    """A dedicated torch stream (default priority) shared by grids and batches."""
    global _default_stream
    import torch
    if _default_stream is None:
        _default_stream = torch.cuda.Stream()
    return _default_stream


def _prec(p):
    return C.PRECISIONS[p] if isinstance(p, str) else int(p)


def _wall(w):
    return C.WALLS[w] if isinstance(w, str) else int(w)


def _dptr(a):
    return a.ctypes.data_as(C._dp)


class Grid:
    """One ``nx`` x ``ny`` lattice.  Arrays are numpy ``[ny, nx]`` (x fastest).

    ``populations=True`` makes a stored-population BGK grid with relaxation time
    ``tau`` (the standard method, for comparison and tau != 1); by default the
    grid is LBMTau1.  ``multiphase=(G, rho0)`` adds the Shan-Chen force."""

    def __init__(self, nx, ny, prec="f32", wall="paper", periodic=0, force=(0.0, 0.0),
                 scale=(0.0, 0.0), snapshot=True, stream=None, torch_memory=True, planar=False,
                 populations=False, tau=1.0, multiphase=None):
        import torch
        self.nx, self.ny = int(nx), int(ny)
        self.prec = _prec(prec)
        self.wall = _wall(wall)
        self.periodic = int(periodic)
        self.force = (float(force[0]), float(force[1]))
        self.options = ((C.OPT_SNAPSHOT if snapshot else 0) | (C.OPT_PLANAR if planar else 0)
                        | (C.OPT_POPULATIONS if populations else 0)
                        | (C.OPT_MULTIPHASE if multiphase is not None else 0))
        self.tau = float(tau)
        self.stream = stream if stream is not None else default_stream()
        nbytes = C.grid_bytes(self.nx, self.ny, self.prec, self.options)
        if nbytes == 0:
            raise C.Lbt1Error(C.EINVAL, f"bad grid {nx} x {ny} precision {prec}")
        self.nbytes = nbytes
        d = C.GridDesc()
        d.nx, d.ny, d.periodic = self.nx, self.ny, self.periodic
        d.prec, d.wall, d.options = self.prec, self.wall, self.options
        d.force[0], d.force[1] = self.force
        d.scale[0], d.scale[1] = float(scale[0]), float(scale[1])
        d.tau = self.tau
        if multiphase is not None:
            d.sc_G, d.sc_rho0 = float(multiphase[0]), float(multiphase[1])
        self._buf = None
        if torch_memory:
            self._buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            d.device_buffer = self._buf.data_ptr()
            d.device_bytes = nbytes
        d.stream = self.stream.cuda_stream
        h = ctypes.c_void_p()
        C.check(C.lib.lbt1_create_grid(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h

    # -- the paper's problem statement: initialise, step, read back --------------
    def set_geometry(self, flags=None, rho=None, jx=None, jy=None):
        shape = (self.ny, self.nx)
        f = None if flags is None else np.ascontiguousarray(flags, dtype=np.uint8).reshape(shape)
        arrs = []
        for a in (rho, jx, jy):
            arrs.append(None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(shape))
        C.check(C.lib.lbt1_set_geometry(
            self.handle, None if f is None else f.ctypes.data_as(C._u8p),
            *[None if a is None else _dptr(a) for a in arrs]))
        return self

    def step(self, n=1):
        C.check(C.lib.lbt1_step(self.handle, int(n)))
        return self

    def read_moments(self):
        shape = (self.ny, self.nx)
        rho, jx, jy = np.empty(shape), np.empty(shape), np.empty(shape)
        C.check(C.lib.lbt1_read_moments(self.handle, _dptr(rho), _dptr(jx), _dptr(jy)))
        return rho, jx, jy

    def read_populations(self):
        """The nine populations f_q, [9, ny, nx] (population grids only)."""
        f = np.empty((9, self.ny, self.nx))
        C.check(C.lib.lbt1_read_populations(self.handle, _dptr(f)))
        return f

    def read_window(self, x0, y0, w, h):
        """(rho, jx, jy) of the window x0 <= x < x0+w, y0 <= y < y0+h, each [h, w]."""
        shape = (int(h), int(w))
        rho, jx, jy = np.empty(shape), np.empty(shape), np.empty(shape)
        C.check(C.lib.lbt1_read_window(self.handle, int(x0), int(y0), int(w), int(h),
                                       _dptr(rho), _dptr(jx), _dptr(jy)))
        return rho, jx, jy

    def reduce(self, what=C.REDUCE_ALL):
        out = np.full(C.REDUCE_SLOTS, np.nan)
        C.check(C.lib.lbt1_reduce(self.handle, int(what), _dptr(out)))
        return dict(mass=out[0], mom_x=out[1], mom_y=out[2], residual=out[3],
                    nonfinite=out[4], fluid=int(out[5]))

    def save_state(self):
        """The exact state in storage format (bytes): the checkpoint lbt1_load_state takes."""
        n = int(C.lib.lbt1_state_bytes(self.handle))
        buf = ctypes.create_string_buffer(n)
        C.check(C.lib.lbt1_save_state(self.handle, buf, n))
        return buf.raw

    def load_state(self, state):
        """Resume from save_state's bytes (same shape, precision and options; the
        geometry must be set)."""
        buf = ctypes.create_string_buffer(bytes(state), len(state))
        C.check(C.lib.lbt1_load_state(self.handle, buf, len(state)))

    def reduce_noalloc(self, out_ptr, what=C.REDUCE_ALL):
        """lbt1_reduce_noalloc: the diagnostics into caller device memory at ``out_ptr``
        (REDUCE_SLOTS doubles), enqueued on the grid's stream; nothing is allocated
        and nothing synchronises."""
        C.check(C.lib.lbt1_reduce_noalloc(self.handle, int(what), ctypes.c_void_p(int(out_ptr))))

    def sync(self):
        C.check(C.lib.lbt1_sync(self.handle))

    # -- kernel choice --------------------------------------------------------------
    def set_kernel(self, kernel="strip", vec=4, rows=14, waves=0, fuse=1):
        k = {"auto": C.KERNEL_AUTO, "gather": C.KERNEL_GATHER, "strip": C.KERNEL_STRIP}.get(kernel, kernel)
        cfg = C.KernelConfig(int(k), int(vec), int(rows), int(waves), int(fuse))
        C.check(C.lib.lbt1_set_kernel(self.handle, ctypes.byref(cfg)))
        return self

    def kernel(self):
        cfg = C.KernelConfig()
        name = ctypes.create_string_buffer(128)
        C.check(C.lib.lbt1_get_kernel(self.handle, ctypes.byref(cfg), name, 128))
        return cfg.as_dict(), name.value.decode()

    def autotune(self, steps=20, reps=3):
        cfg = C.KernelConfig()
        ms = ctypes.c_double()
        C.check(C.lib.lbt1_autotune(self.handle, int(steps), int(reps), ctypes.byref(cfg), ctypes.byref(ms)))
        return cfg.as_dict(), ms.value

    def close(self):
        if getattr(self, "handle", None):
            C.check(C.lib.lbt1_destroy_grid(self.handle))
            self.handle = None
            self._buf = None

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                C.lib.lbt1_destroy_grid(self.handle)
                self.handle = None
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

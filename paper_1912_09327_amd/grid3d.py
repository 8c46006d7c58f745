"""Python handle for one 3-D LBMTau1 grid (D3Q19 / D3Q27) on the GPU; a thin
wrapper over the lbt1_grid3d_* C ABI.  Arrays are numpy [nz, ny, nx]."""
import ctypes

import numpy as np

from . import _capi as C
from .grid import _dptr, _prec, _wall, default_stream


class Grid3D:
    def __init__(self, nx, ny, nz, q=19, prec="f32", wall="paper", periodic=0, force=(0.0, 0.0, 0.0),
                 scale=(0.0, 0.0), snapshot=True, stream=None):
        import torch
        self.nx, self.ny, self.nz, self.q = int(nx), int(ny), int(nz), int(q)
        self.prec = _prec(prec)
        self.options = C.OPT_SNAPSHOT if snapshot else 0
        self.stream = stream if stream is not None else default_stream()
        nbytes = C.lib.lbt1_grid3d_bytes(self.nx, self.ny, self.nz, self.q, self.prec, self.options)
        if nbytes == 0:
            raise C.Lbt1Error(C.EINVAL, f"bad 3-D grid {nx} x {ny} x {nz} D3Q{q}")
        self.nbytes = nbytes
        d = C.Grid3DDesc()
        d.nx, d.ny, d.nz, d.q = self.nx, self.ny, self.nz, self.q
        d.periodic, d.prec, d.wall, d.options = int(periodic), self.prec, _wall(wall), self.options
        for a in range(3):
            d.force[a] = float(force[a])
        d.scale[0], d.scale[1] = float(scale[0]), float(scale[1])
        self._buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        d.device_buffer, d.device_bytes = self._buf.data_ptr(), nbytes
        d.stream = self.stream.cuda_stream
        h = ctypes.c_void_p()
        C.check(C.lib.lbt1_grid3d_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h

    def set_geometry(self, flags=None, rho=None, jx=None, jy=None, jz=None):
        shape = (self.nz, self.ny, self.nx)
        f = None if flags is None else np.ascontiguousarray(flags, dtype=np.uint8).reshape(shape)
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(shape)
                for a in (rho, jx, jy, jz)]
        C.check(C.lib.lbt1_grid3d_set_geometry(self.handle, None if f is None else f.ctypes.data_as(C._u8p),
                                               *[None if a is None else _dptr(a) for a in arrs]))
        return self

    def set_kernel(self, kernel="auto"):
        k = {"auto": C.KERNEL_AUTO, "gather": C.KERNEL_GATHER, "tile": C.KERNEL_STRIP}[kernel]
        C.check(C.lib.lbt1_grid3d_set_kernel(self.handle, k))
        return self

    def kernel(self):
        k = ctypes.c_int32()
        C.check(C.lib.lbt1_grid3d_get_kernel(self.handle, ctypes.byref(k)))
        return "tile" if k.value == C.KERNEL_STRIP else "gather"

    def step(self, n=1):
        C.check(C.lib.lbt1_grid3d_step(self.handle, int(n)))
        return self

    def read_moments(self):
        shape = (self.nz, self.ny, self.nx)
        out = [np.empty(shape) for _ in range(4)]
        C.check(C.lib.lbt1_grid3d_read_moments(self.handle, *[_dptr(a) for a in out]))
        return tuple(out)

    def reduce(self, what=C.REDUCE_ALL):
        out = np.full(8, np.nan)
        C.check(C.lib.lbt1_grid3d_reduce(self.handle, int(what), _dptr(out)))
        return dict(mass=out[0], mom=(out[1], out[2], out[3]), residual=out[4], nonfinite=out[5],
                    fluid=int(out[6]))

    def sync(self):
        C.check(C.lib.lbt1_grid3d_sync(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            C.check(C.lib.lbt1_grid3d_destroy(self.handle))
            self.handle = None
            self._buf = None

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                C.lib.lbt1_grid3d_destroy(self.handle)
        except Exception:
            pass

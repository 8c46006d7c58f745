"""ctypes binding of ``liblbt1.so`` (the C ABI declared in ``include/lbt1.h``).

Argument marshalling only: every step, reduction and batch burst runs in the
library's HIP kernels.  If the library is not built, importing this module
raises; there is no CPU fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbt1.so")

# status codes
OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EBUSY, ENONFINITE = range(7)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ESTATE", 5: "EBUSY", 6: "ENONFINITE"}
# precisions
F64, F32, F16S, BF16S = 0, 1, 2, 3
PRECISIONS = {"f64": F64, "f32": F32, "f16s": F16S, "bf16s": BF16S}
VALUE_BYTES = {F64: 8, F32: 4, F16S: 2, BF16S: 2}
# wall rules
WALL_PAPER, WALL_HALFWAY = 0, 1
WALLS = {"paper": WALL_PAPER, "halfway": WALL_HALFWAY}
# node flags
FLUID, SOLID, FIXED = 0, 1, 2
PERIODIC_X, PERIODIC_Y = 1, 2
OPT_SNAPSHOT = 1
OPT_PLANAR = 2
OPT_POPULATIONS = 4
OPT_MULTIPHASE = 8
REDUCE_MASS, REDUCE_MOMENTUM, REDUCE_RESIDUAL, REDUCE_NONFINITE = 1, 2, 4, 8
REDUCE_ALL = 15
REDUCE_SLOTS = 6
KERNEL_AUTO, KERNEL_GATHER, KERNEL_STRIP = 0, 1, 2
SLOT_FREE, SLOT_RUNNING, SLOT_BUDGET, SLOT_CONVERGED, SLOT_NONFINITE = range(5)
PROBE_COPY, PROBE_READ, PROBE_WRITE, PROBE_3IN3OUT = range(4)


class Lbt1Error(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{self.name}: {message}")


class GridDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("periodic", ctypes.c_uint32),
        ("prec", ctypes.c_int32), ("wall", ctypes.c_int32), ("options", ctypes.c_uint32),
        ("force", ctypes.c_double * 2), ("scale", ctypes.c_double * 2),
        ("device_buffer", ctypes.c_void_p), ("device_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p), ("tau", ctypes.c_double),
        ("sc_G", ctypes.c_double), ("sc_rho0", ctypes.c_double),
    ]


class KernelConfig(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("vec", ctypes.c_int32), ("rows", ctypes.c_int32),
                ("waves", ctypes.c_int32), ("fuse", ctypes.c_int32)]

    def as_dict(self):
        return dict(kernel=self.kernel, vec=self.vec, rows=self.rows, waves=self.waves, fuse=self.fuse)


class BatchShape(ctypes.Structure):
    _fields_ = [("fuse", ctypes.c_int32), ("lds", ctypes.c_int32), ("rows", ctypes.c_int32 * 5),
                ("vec_cap", ctypes.c_int32)]

    def as_dict(self):
        return dict(fuse=self.fuse, lds=self.lds, rows=list(self.rows), vec_cap=self.vec_cap)


class Grid3DDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("q", ctypes.c_int32),
        ("periodic", ctypes.c_uint32), ("prec", ctypes.c_int32), ("wall", ctypes.c_int32),
        ("options", ctypes.c_uint32), ("force", ctypes.c_double * 3), ("scale", ctypes.c_double * 2),
        ("device_buffer", ctypes.c_void_p), ("device_bytes", ctypes.c_size_t), ("stream", ctypes.c_void_p),
    ]


_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i32 = ctypes.c_int32

# name -> (restype, argtypes); mirrors include/lbt1.h
SIGNATURES = {
    "lbt1_grid_bytes": (ctypes.c_size_t, [_i32, _i32, _i32, ctypes.c_uint32]),
    "lbt1_create_grid": (ctypes.c_int, [ctypes.POINTER(GridDesc), ctypes.POINTER(_vp)]),
    "lbt1_set_geometry": (ctypes.c_int, [_vp, _u8p, _dp, _dp, _dp]),
    "lbt1_step": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "lbt1_read_moments": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
    "lbt1_read_window": (ctypes.c_int, [_vp, _i32, _i32, _i32, _i32, _dp, _dp, _dp]),
    "lbt1_read_populations": (ctypes.c_int, [_vp, _dp]),
    "lbt1_reduce": (ctypes.c_int, [_vp, ctypes.c_uint32, _dp]),
    "lbt1_reduce_noalloc": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp]),
    "lbt1_state_bytes": (ctypes.c_size_t, [_vp]),
    "lbt1_save_state": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "lbt1_load_state": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "lbt1_sync": (ctypes.c_int, [_vp]),
    "lbt1_destroy_grid": (ctypes.c_int, [_vp]),
    "lbt1_last_error": (ctypes.c_char_p, []),
    "lbt1_set_kernel": (ctypes.c_int, [_vp, ctypes.POINTER(KernelConfig)]),
    "lbt1_get_kernel": (ctypes.c_int, [_vp, ctypes.POINTER(KernelConfig), ctypes.c_char_p, ctypes.c_size_t]),
    "lbt1_autotune": (ctypes.c_int, [_vp, _i32, _i32, ctypes.POINTER(KernelConfig), _dp]),
    "lbt1_batch_create": (ctypes.c_int, [ctypes.c_size_t, _i32, _vp, ctypes.POINTER(_vp)]),
    "lbt1_batch_admit": (ctypes.c_int, [_vp, _vp, ctypes.c_int64, ctypes.c_double, ctypes.POINTER(_i32)]),
    "lbt1_batch_run": (ctypes.c_int, [_vp, _i32]),
    "lbt1_batch_poll": (ctypes.c_int, [_vp, ctypes.POINTER(_i32), _i32, ctypes.POINTER(_i32)]),
    "lbt1_batch_slot_info": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_int64), _dp]),
    "lbt1_batch_set_shape": (ctypes.c_int, [_vp, ctypes.POINTER(BatchShape)]),
    "lbt1_batch_get_shape": (ctypes.c_int, [_vp, ctypes.POINTER(BatchShape)]),
    "lbt1_batch_autotune": (ctypes.c_int, [_vp, _i32, _i32, ctypes.POINTER(BatchShape), _dp]),
    "lbt1_batch_evict": (ctypes.c_int, [_vp, _i32]),
    "lbt1_batch_destroy": (ctypes.c_int, [_vp]),
    "lbt1_probe_bandwidth": (ctypes.c_int, [_i32, ctypes.c_size_t, _i32, _i32, _dp]),
    "lbt1_grid3d_bytes": (ctypes.c_size_t, [_i32, _i32, _i32, _i32, _i32, ctypes.c_uint32]),
    "lbt1_grid3d_create": (ctypes.c_int, [ctypes.POINTER(Grid3DDesc), ctypes.POINTER(_vp)]),
    "lbt1_grid3d_set_geometry": (ctypes.c_int, [_vp, _u8p, _dp, _dp, _dp, _dp]),
    "lbt1_grid3d_step": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "lbt1_grid3d_read_moments": (ctypes.c_int, [_vp, _dp, _dp, _dp, _dp]),
    "lbt1_grid3d_reduce": (ctypes.c_int, [_vp, ctypes.c_uint32, _dp]),
    "lbt1_grid3d_set_kernel": (ctypes.c_int, [_vp, _i32]),
    "lbt1_grid3d_get_kernel": (ctypes.c_int, [_vp, ctypes.POINTER(_i32)]),
    "lbt1_grid3d_sync": (ctypes.c_int, [_vp]),
    "lbt1_grid3d_destroy": (ctypes.c_int, [_vp]),
}


def _load():
    # PyTorch provides device memory and streams and brings its own HIP runtime
    # (libamdhip64.so.7).  Loading torch first makes the library bind to that
    # same runtime by soname; loading the library first would start a second
    # HIP runtime in the process, which then sees no device.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1912_09327_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def check(status):
    """Raise Lbt1Error for a non-OK status, with the library's message."""
    if status != OK:
        msg = lib.lbt1_last_error()
        raise Lbt1Error(status, msg.decode() if msg else "")
    return status


def grid_bytes(nx, ny, prec, options=OPT_SNAPSHOT):
    return int(lib.lbt1_grid_bytes(int(nx), int(ny), int(prec), int(options)))


def probe_bandwidth(kind, nbytes=4 << 30, nontemporal=False, reps=5):
    """Achievable GB/s of a plain streaming pattern (PROBE_*) on the current device."""
    out = ctypes.c_double()
    check(lib.lbt1_probe_bandwidth(int(kind), int(nbytes), int(bool(nontemporal)), int(reps), ctypes.byref(out)))
    return out.value

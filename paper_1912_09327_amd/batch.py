"""Python handle for a batch of resident grids (lbt1_batch_* of the C ABI)."""
import ctypes

from . import _capi as C
from .grid import default_stream


class Batch:
    """Resident grids stepped together in HIP-graph bursts.

    ``admit`` returns a slot id, or ``None`` when the HBM budget or the slots
    are exhausted (the library's EBUSY).
    """

    def __init__(self, hbm_budget_bytes, max_slots, stream=None):
        self.stream = stream if stream is not None else default_stream()
        h = ctypes.c_void_p()
        C.check(C.lib.lbt1_batch_create(int(hbm_budget_bytes), int(max_slots), self.stream.cuda_stream,
                                        ctypes.byref(h)))
        self.handle = h
        self.grids = {}

    def admit(self, grid, step_budget, residual_tol=-1.0):
        slot = ctypes.c_int32()
        st = C.lib.lbt1_batch_admit(self.handle, grid.handle, int(step_budget), float(residual_tol),
                                    ctypes.byref(slot))
        if st == C.EBUSY:
            return None
        C.check(st)
        self.grids[slot.value] = grid
        return slot.value

    def run(self, burst_steps):
        C.check(C.lib.lbt1_batch_run(self.handle, int(burst_steps)))

    def set_shape(self, fuse=2, rows=(0, 0, 0, 0, 0), lds=0, vec_cap=0):
        """Tile shape: fuse mode (0 none, 1 all, 2 mixed: the default), LDS residency of
        small grids (0 / 1), the strip height of the five work classes (0 = heuristic)
        and the widest columns per lane of the one-step classes (4, 2, 1; 0 = 4)."""
        rows = list(rows) + [0] * (5 - len(rows))
        sh = C.BatchShape(int(fuse), int(lds), (ctypes.c_int32 * 5)(*[int(r) for r in rows]), int(vec_cap))
        C.check(C.lib.lbt1_batch_set_shape(self.handle, ctypes.byref(sh)))

    def shape(self):
        sh = C.BatchShape()
        C.check(C.lib.lbt1_batch_get_shape(self.handle, ctypes.byref(sh)))
        return sh.as_dict()

    def autotune(self, burst_steps=20, reps=3):
        """Time tile shapes on the running grids (state restored) and keep the fastest;
        returns (shape, ms per burst)."""
        sh = C.BatchShape()
        ms = ctypes.c_double()
        C.check(C.lib.lbt1_batch_autotune(self.handle, int(burst_steps), int(reps), ctypes.byref(sh),
                                          ctypes.byref(ms)))
        return sh.as_dict(), ms.value

    def poll(self):
        cap = max(1, len(self.grids))
        buf = (ctypes.c_int32 * cap)()
        n = ctypes.c_int32()
        C.check(C.lib.lbt1_batch_poll(self.handle, buf, cap, ctypes.byref(n)))
        return [buf[i] for i in range(min(n.value, cap))]

    def slot_info(self, slot):
        st = ctypes.c_int32()
        steps = ctypes.c_int64()
        res = ctypes.c_double()
        C.check(C.lib.lbt1_batch_slot_info(self.handle, int(slot), ctypes.byref(st), ctypes.byref(steps),
                                           ctypes.byref(res)))
        return st.value, steps.value, res.value

    def evict(self, slot):
        C.check(C.lib.lbt1_batch_evict(self.handle, int(slot)))
        return self.grids.pop(slot)

    def close(self):
        if getattr(self, "handle", None):
            C.check(C.lib.lbt1_batch_destroy(self.handle))
            self.handle = None
            self.grids = {}

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                C.lib.lbt1_batch_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

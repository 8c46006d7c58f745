"""MI355X-native LBMTau1 D2Q9 (arXiv:1912.09327): moments-only lattice Boltzmann at tau = 1.

The step runs in hand-written HIP kernels for gfx950 behind the C ABI of
``include/lbt1.h`` (``liblbt1.so``, built by ``paper_1912_09327_amd.build``).
``Grid``, ``Batch`` and ``Server`` load that library on first use and raise if
it is missing; there is no CPU fallback.  ``inputs`` (seeded workloads) does
not need the library.
"""
__all__ = ["Grid", "Batch", "Server", "inputs"]


def __getattr__(name):
    if name == "Grid":
        from .grid import Grid
        return Grid
    if name == "Batch":
        from .batch import Batch
        return Batch
    if name == "Server":
        from .serve import Server
        return Server
    raise AttributeError(name)

"""MI355X-native SFSeg power iteration (Burceanu & Leordeanu, arXiv 1907.02731).

The principal eigenvector of a video's space-time pixel graph, computed by
power iteration with the graph applied as separable 3D Gaussian filtering in
hand-written gfx950 kernels behind the C ABI of ``include/sfseg.h``.
"""
from ._lib import SfsegError, LIB_PATH  # noqa: F401

__all__ = ["Solver", "SfsegError", "LIB_PATH"]


def __getattr__(name):
    if name == "Solver":
        from .solver import Solver
        return Solver
    raise AttributeError(name)

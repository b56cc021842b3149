"""MI355X-native FDLB solver for bounded flows of dense gases (arXiv 2308.15407).

The time step runs in hand-written gfx950 HIP kernels behind the C ABI of
include/fdlb.h (libfdlb.so); ``fdlb`` is the ctypes binding with the same names
and ``Solver`` manages the torch-owned workspace and stream.
"""
from . import fdlb  # noqa: F401


def __getattr__(name):
    if name == "Solver":
        from .solver import Solver
        return Solver
    raise AttributeError(name)

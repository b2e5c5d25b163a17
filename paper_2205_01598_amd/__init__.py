"""Level-blocked sparse matrix power kernel (MPK) for AMD MI355X (gfx950).

Python binding of the C-ABI declared in ``include/mpk.h``.  The library
``libmpk.so`` (host planner in C++, kernels in HIP) must be built in-tree;
there is no fallback path.
"""
from ._lib import MpkError, lib  # noqa: F401
from .mpk import Plan, Recurrence, Spmv, bw_probe  # noqa: F401

__all__ = ["Plan", "Spmv", "Recurrence", "MpkError", "bw_probe", "lib"]

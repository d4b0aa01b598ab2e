"""MI355X-native C-AMS pressure solver (arXiv 1705.05783).

The compute path is libcams.so (hand-written HIP for gfx950, C ABI in
include/cams.h).  `_cams` is the ctypes binding with the ABI's names;
`Solver` wraps one problem.  There is no CPU fallback: using the solver
without the built library raises.
"""

from . import _cams  # noqa: F401


def Solver(*args, **kwargs):  # noqa: N802 - factory keeps torch import lazy
    from .solver import Solver as _S
    return _S(*args, **kwargs)


__all__ = ["Solver", "_cams"]

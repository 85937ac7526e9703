"""MI355X (gfx950) MGRIT for the 2D eddy-current induction-machine problem
of arXiv:1912.03106.

The compute path is libmgrit.so (hand-written HIP kernels behind the C ABI in
include/mgrit.h).  This package only marshals arguments; importing it does not
load the library, creating a `Solver` does (and fails if it is missing).
"""

from ._abi import MgritError, STATUS, lib  # noqa: F401


def Solver(*args, **kwargs):
    from .solver import Solver as _S
    return _S(*args, **kwargs)

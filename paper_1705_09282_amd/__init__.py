"""dfmg: divergence-free geometric multigrid for isogeometric compatible
discretizations of the generalized Stokes and Oseen problems, on MI355X.

The solver lives in the HIP library ``libdfmg.so`` (C-ABI in include/dfmg.h);
``paper_1705_09282_amd.dfmg`` is its Python binding.
"""


def Solver(*args, **kwargs):
    from .dfmg import Solver as _S
    return _S(*args, **kwargs)

"""Hard-coded-gradient GRAPE cost+gradient on AMD MI355X (gfx950).

The product path is libhgrape.so (HIP kernels + C++ host planner) behind the C
ABI declared in include/hgrape.h.  Python provides the ctypes binding
(``_lib``, same names as the C functions), a thin torch wrapper for device
memory and streams (``api``), and the autograd adjoint (``autograd``).
Importing the package fails if the library has not been built.
"""
from . import _lib  # noqa: F401  (raises ImportError when libhgrape.so is missing)
from .api import Context, EvalResult, Problem, evaluate, mem_pool_peak, plan, step_norms  # noqa: F401
from .autograd import HGCost, hg_cost  # noqa: F401
from .serving import Server, percentiles  # noqa: F401

__all__ = ["Context", "Problem", "EvalResult", "evaluate", "mem_pool_peak", "plan", "step_norms", "HGCost",
           "hg_cost", "Server", "percentiles"]

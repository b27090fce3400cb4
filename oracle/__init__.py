"""FP64 CPU oracle for hard-coded-gradient GRAPE.  TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke entry point and the benchmark's CPU-baseline leg
may import this package.  The GPU product path never calls into it, and it
shares no code with the HIP library: no kernels, headers, helpers or constants.

Modules
  grape    exact cost and gradient: dense Pade expm per step, all states
           stored, co-state recursion, Frechet derivative of expm
           (Van Loan block, or Daleckii-Krein in the eigenbasis)
  planner  the paper's error bound E_A(m, s) and its (m, s) selection rule
  taylor   the paper's Taylor scaling-and-squaring action and the auxiliary
           block-matrix derivative action, written plainly in FP64
  chebyshev  the Chebyshev expansion a footnote of Sec. III.B names as the
           faster alternative (planner comparison only)

Every function cites the passage of Lu, Joshi, Dinh, Koch,
"Optimal control of large quantum systems: assessing memory and runtime
performance of GRAPE" (arXiv:2304.06200) that it follows.

Parity status: grape and taylor are pinned by closed forms, invariants, finite
differences and high-precision references (tests/test_oracle_*.py).  The
planner formula is pinned by the special cases App. C writes out (the rounding
part at m = 0 and m = 1, eq. c17, composed over s = 1 and s = 2, eqs. s1 and
C22), by the tight truncation bound of a 1x1 operator, by a 50-digit tail sum
and by the empirical bound property; *which* (m, s) the authors obtained for any
given norm is parity unpinned (the paper prints no such values).  chebyshev's
coefficients are pinned by the Jacobi-Anger identity on the unit circle, its
truncation bound on scalar operators and its action against scipy's expm; its
rounding part, written in the style of App. C.2 for a method the paper only
names, is parity unpinned.
"""
from . import chebyshev, grape, planner, taylor  # noqa: F401

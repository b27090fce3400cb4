"""The paper's error bound E_A(m, s) and (m, s) selection rule (oracle; tests only).

App. C derives, for e^A |Psi> ~ (T_m(B))^s |Psi> with B = A/s and
T_m(B) = sum_{q<=m} B^q/q!  (Sec. III.B, eqs. scaling squaring, eBm):

  R_m(x)  = sum_{q>m} x^q / q!                              (App. C.1)
  trunc   = s R (1 - (s R)^s) / (1 - s R),  R = R_m(||B||_1)  (App. C.1, eq. truncation)
  u'      = 2 sqrt(2) u / (1 - 2u)                           (App. C.2, complex product)
  gamma_n = n u' / (1 - n u')                                (App. C.2)
  beta    = sum_{k=0..m} gamma_{k(sigma'+2)+m+2} ||B||_1^k / k!   (App. C.2, eq. B23)
  alpha   = 1 + R_m(||B||_1)                                 (App. C.3)
  E_A     = trunc + (alpha + beta)^s - alpha^s               (App. C, eq. overallupperbound)

with ||B||_1 = ||A||_1 / s, ||A||_1 the matrix 1-norm (App. C.1, eq. norm
inequality: for anti-Hermitian A the 1-norm bounds the 2-norm), sigma' the
largest number of non-zeros in a row of A (App. C.2, eq. sigmapdef) and u the
unit roundoff of the arithmetic.  The rule (Sec. III.B, around eq. mudefnition):
the smallest s admitting a solution of E_A <= tau, then the smallest m for that s;
the cost is mu = m s matrix-vector products.

Readings where the paper is silent:
  * u is Higham's unit roundoff, 2^-53 for FP64 (and 2^-24 for FP32);
  * gamma_n is infinite (infeasible) once n u' >= 1;
  * the truncation form is valid only for s R < 1; s R >= 1 is infeasible;
  * R_m is summed as its tail directly, stopping once a term falls below
    1e-18 of the running sum (no cancellation from e^x minus a partial sum);
  * (alpha+beta)^s - alpha^s is evaluated as alpha^s expm1(s log1p(beta/alpha)),
    the same number without the cancellation of the literal difference;
  * the search runs s = 1, 2, ... and m = 1..m_max (m_max = 60); the first hit
    wins.  For s with s gamma_3 > tau no larger s can be feasible (the rounding
    part alone exceeds tau), which ends the search as "unreachable".
"""
from __future__ import annotations

import math
from typing import Tuple

U_FP64 = 2.0 ** -53
U_FP32 = 2.0 ** -24
M_MAX = 60


def u_prime(u: float) -> float:
    """Relative error bound of one complex product (App. C.2)."""
    return 2.0 * math.sqrt(2.0) * u / (1.0 - 2.0 * u)


def gamma(n: int, up: float) -> float:
    """gamma_n = n u' / (1 - n u') (App. C.2); infinite once n u' >= 1."""
    nu = n * up
    if nu >= 1.0:
        return math.inf
    return nu / (1.0 - nu)


def taylor_tail(x: float, m: int) -> float:
    """R_m(x) = sum_{q=m+1}^inf x^q / q! for x >= 0 (App. C.1)."""
    if x == 0.0:
        return 0.0
    t = 1.0
    for q in range(1, m + 2):
        t = t * x / q
    total = t
    q = m + 1
    while True:
        q += 1
        t = t * x / q
        total += t
        if not (t >= 1e-18 * total) or math.isinf(total):
            break
    return total


def error_bound(theta: float, m: int, s: int, sigma: int, u: float = U_FP64) -> float:
    """E_A(m, s) for ||A||_1 = theta (App. C, eq. overallupperbound)."""
    x = theta / s
    R = taylor_tail(x, m)
    sR = s * R
    if not (sR < 1.0):
        return math.inf
    trunc = sR * (1.0 - sR ** s) / (1.0 - sR)
    up = u_prime(u)
    alpha = 1.0 + R
    beta = 0.0
    t = 1.0
    for k in range(0, m + 1):
        if k > 0:
            t = t * x / k
        beta += gamma(k * (sigma + 2) + m + 2, up) * t
    if math.isinf(beta):
        return math.inf
    rnd = alpha ** s * math.expm1(s * math.log1p(beta / alpha))
    return trunc + rnd


def s_limit(tau: float, u: float = U_FP64) -> int:
    """Largest s worth trying: for s gamma_3 > tau the rounding part alone
    exceeds tau for every m (it is at least s beta >= s gamma_{m+2} >= s gamma_3)."""
    g3 = gamma(3, u_prime(u))
    return max(1, int(tau / g3))


def select(theta: float, sigma: int, tau: float, u: float = U_FP64,
           m_max: int = M_MAX) -> Tuple[int, int]:
    """(m, s) by the paper's rule: smallest s with a solution of E_A <= tau,
    then the smallest m for that s (Sec. III.B).  Raises ValueError when no
    (m <= m_max, s) satisfies the bound."""
    if not (theta >= 0.0) or math.isinf(theta):
        raise ValueError(f"invalid norm {theta!r}")
    for s in range(1, s_limit(tau, u) + 1):
        for m in range(1, m_max + 1):
            if error_bound(theta, m, s, sigma, u) <= tau:
                return m, s
    raise ValueError(f"tolerance {tau:g} unreachable at norm {theta:g}")


def one_norm(dense_matrix) -> float:
    """||A||_1 = max column sum of |A_ij| (equal to the max row sum for the
    anti-Hermitian A = -i dt H), App. C.1."""
    import numpy as np
    return float(np.max(np.sum(np.abs(np.asarray(dense_matrix)), axis=0)))


def select_min_mu(theta: float, sigma: int, tau: float, u: float = U_FP64,
                  m_max: int = M_MAX) -> Tuple[int, int]:
    """(m, s) with the fewest products mu = m s under the same bound E_A <= tau
    (the alternative Sec. III.B sets aside after eq. accuracy inequality because
    the minimisation costs more than it saves there); ties go to the smaller s.

    For each s the smallest feasible m is the cheapest, so the search takes,
    for s = 1, 2, ..., that m, and stops once s alone exceeds the best mu found
    (every larger s costs at least s products).  Raises ValueError when no
    (m <= m_max, s) satisfies the bound."""
    if not (theta >= 0.0) or math.isinf(theta):
        raise ValueError(f"invalid norm {theta!r}")
    best = None
    for s in range(1, s_limit(tau, u) + 1):
        if best is not None and s > best[0] * best[1]:
            break
        for m in range(1, m_max + 1):
            if error_bound(theta, m, s, sigma, u) <= tau:
                if best is None or m * s < best[0] * best[1]:
                    best = (m, s)
                break
    if best is None:
        raise ValueError(f"tolerance {tau:g} unreachable at norm {theta:g}")
    return best

"""Chebyshev expansion of the propagator-state product (oracle; tests only).

Sec. III.B mentions, in a footnote to the choice of the truncation order,
that a Chebyshev expansion converges faster than the Taylor series with the
same runtime scaling, and keeps Taylor for simplicity.  This module writes the
Chebyshev alternative out plainly so that the number of products it needs can
be compared with the paper's (m, s) rule.

For Hermitian H with spectrum inside [-rho, rho] and theta = dt rho, the
Jacobi-Anger expansion gives

    exp(-i dt H) = J_0(theta) I + 2 sum_{k>=1} (-i)^k J_k(theta) T_k(H / rho),

T_k the Chebyshev polynomials (T_0 = 1, T_1 = x, T_{k+1} = 2 x T_k - T_{k-1}),
J_k the Bessel functions of the first kind.  Truncating after degree m costs m
matrix-vector products (one per recurrence step) and, because |T_k(x)| <= 1 on
[-1, 1], leaves an error of at most 2 sum_{k>m} |J_k(theta)| in the 2-norm.

Readings where the paper says nothing (it only names the method):
  * rho = ||H||_1, the norm App. C uses for the Taylor bound (eq. norm
    inequality: it bounds the spectral radius of Hermitian H), so theta equals
    the Taylor planner's ||A||_1;
  * the step may be split into s equal pieces, each expanded at theta/s, as
    the Taylor rule scales (Sec. III.B): Chebyshev needs about
    theta + O(theta^(1/3)) products for a fixed truncation error, so splitting
    never lowers the truncation cost, but it keeps the rounding part (which
    grows with the square of the degree, below) within tau at large norms;
    the rule is the paper's: the smallest s, then the smallest m;
  * composition over s pieces as App. C.3 composes the Taylor pieces: with
    t the truncation bound of one piece (so ||p|| <= 1 + t next to the unitary
    exact factor) and beta its rounding bound, the error after s pieces is at
    most ((1 + t)^s - 1) + ((alpha + beta)^s - alpha^s), alpha = 1 + t;
  * rounding is bounded in the style of App. C.2: a product with sigma'
    non-zeros per row rounds within gamma_{sigma'+2}, each recurrence step adds
    the product, a scaling by 2 and a subtraction (gamma_{sigma'+4} per step),
    and an error made at step j reaches T_k through the second-kind polynomial
    U_{k-j} (|U_n| <= n + 1 on [-1, 1]), so T_k carries at most
    gamma_{sigma'+4} k (k + 1) / 2 and the weighted sum
    sum_k |c_k| gamma_{sigma'+4} k (k + 1) / 2 + gamma_{m+1} sum_k |c_k|
    (the final accumulation of m + 1 terms);
  * the degree is the smallest m with truncation + rounding <= tau, searched
    up to m_max = 4096.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import jv

from .planner import U_FP64, gamma, u_prime

M_MAX_CHEB = 4096


def coefficients(theta: float, m: int) -> np.ndarray:
    """c_k = (2 - delta_k0) (-i)^k J_k(theta), k = 0..m (Jacobi-Anger)."""
    k = np.arange(m + 1)
    c = 2.0 * (-1j) ** k * jv(k, theta)
    c[0] = jv(0, theta)
    return c.astype(np.complex128)


def truncation_bound(theta: float, m: int) -> float:
    """2 sum_{k>m} |J_k(theta)|, summed until the terms fall below 1e-18 of the sum
    past k = theta (where J_k starts to decay faster than geometrically)."""
    total = 0.0
    k = m + 1
    while True:
        t = abs(float(jv(k, theta)))
        total += t
        if k > theta + 10 and t <= 1e-18 * max(total, 1e-300):
            break
        k += 1
    return 2.0 * total


def rounding_bound(theta: float, m: int, sigma: int, u: float = U_FP64) -> float:
    """Rounding of one piece: sum_k |c_k| gamma_{sigma+4} k (k+1)/2 + gamma_{m+1} sum_k |c_k|."""
    c = np.abs(coefficients(theta, m))
    up = u_prime(u)
    k = np.arange(m + 1, dtype=np.float64)
    return (gamma(sigma + 4, up) * float(np.sum(c * k * (k + 1) / 2.0))
            + gamma(m + 1, up) * float(np.sum(c)))


def error_bound(theta: float, m: int, s: int, sigma: int, u: float = U_FP64) -> float:
    """Error of s pieces of degree m at norm theta (the composition above)."""
    x = theta / s
    t = truncation_bound(x, m)
    beta = rounding_bound(x, m, sigma, u)
    if math.isinf(beta):
        return math.inf
    alpha = 1.0 + t
    trunc = math.expm1(s * math.log1p(t))
    rnd = alpha ** s * math.expm1(s * math.log1p(beta / alpha))
    return trunc + rnd


def select(theta: float, sigma: int, tau: float, u: float = U_FP64, s_max: int = 4096):
    """(m, s): the smallest s admitting a degree m <= M_MAX_CHEB with
    error_bound <= tau, then the smallest such m.  ValueError if none."""
    if not (theta >= 0.0) or math.isinf(theta):
        raise ValueError(f"invalid norm {theta!r}")
    for s in range(1, s_max + 1):
        x = theta / s
        # the degree needed for the truncation part alone is a lower bound
        m = 0
        while truncation_bound(x, m) > tau and m < M_MAX_CHEB:
            m += 1
        while m <= M_MAX_CHEB:
            e = error_bound(theta, m, s, sigma, u)
            if e <= tau:
                return m, s
            # past the truncation floor the rounding part only grows with m
            if truncation_bound(x, m) < 1e-3 * tau:
                break
            m += 1
    raise ValueError(f"tolerance {tau:g} unreachable at norm {theta:g}")


def action(H, psi: np.ndarray, dt: float, m: int, rho: float) -> np.ndarray:
    """sum_{k<=m} c_k T_k(H/rho) psi, the T_k psi by the three-term recurrence
    (m products with H).  rho must bound the spectral radius of H."""
    theta = dt * rho
    c = coefficients(theta, m)
    t_prev = np.array(psi, dtype=np.complex128, copy=True)
    acc = c[0] * t_prev
    if m == 0:
        return acc
    t_cur = (H @ t_prev) / rho
    acc = acc + c[1] * t_cur
    for k in range(2, m + 1):
        t_next = 2.0 * (H @ t_cur) / rho - t_prev
        acc = acc + c[k] * t_next
        t_prev, t_cur = t_cur, t_next
    return acc

"""Pins of the (m, s) planner oracle (App. C error bound, Sec. III.B rule).

The bound is fixed by: its truncation part against a 1x1 anti-Hermitian
matrix, where the triangle-inequality bound is tight to first order (so a
wrong index, a dropped factor s or a wrong scaled norm shows up as a ratio far
from 1); its tail sum against a 50-digit mpmath evaluation of e^x minus the
partial sum; the stable rewrite of (alpha+beta)^s - alpha^s against the literal
difference at 50 digits; the rounding part against the special cases the paper
writes out (m = 0 and m = 1 of App. C.2, s = 1 and s = 2 of App. C.3); and the
selection rule against brute-force minimality.  Which (m, s) the authors obtained for a given norm is parity
unpinned: the paper prints no such values.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import planner

mp.mp.dps = 50


def _tail_mp(x, m):
    x = mp.mpf(x)
    return mp.e ** x - sum(x ** q / mp.factorial(q) for q in range(m + 1))


@pytest.mark.parametrize("x,m", [(0.5, 3), (2.6, 22), (1.0, 10), (7.0, 40), (0.01, 1), (3.4, 27)])
def test_taylor_tail_matches_high_precision(x, m):
    ref = _tail_mp(x, m)
    assert planner.taylor_tail(x, m) == pytest.approx(float(ref), rel=1e-13)


@pytest.mark.parametrize("theta,m,s", [(0.5, 4, 1), (2.0, 8, 1), (3.0, 6, 2), (10.0, 12, 4),
                                       (6.0, 10, 3), (1.5, 5, 2)])
def test_truncation_bound_tight_on_scalar(theta, m, s):
    """A = i theta (1x1, anti-Hermitian): |e^A - T_m(A/s)^s| <= trunc, and the
    bound exceeds the actual error by less than 1.5x when s R << 1."""
    A = mp.mpc(0, theta)
    B = A / s
    Tm = sum(B ** q / mp.factorial(q) for q in range(m + 1))
    actual = abs(mp.e ** A - Tm ** s)
    R = planner.taylor_tail(theta / s, m)
    trunc = s * R * (1 - (s * R) ** s) / (1 - s * R)
    # the full bound with zero roundoff is the truncation part alone
    assert planner.error_bound(theta, m, s, sigma=1, u=0.0) == pytest.approx(trunc, rel=1e-15)
    assert float(actual) <= trunc * (1 + 1e-12)
    assert trunc / float(actual) < 1.5


def test_rounding_part_stable_form_vs_literal():
    """(alpha+beta)^s - alpha^s at 50 digits equals the bound minus its truncation part."""
    for theta, m, s, sigma in [(10.3, 22, 4, 9), (4.2, 18, 2, 5), (0.47, 11, 1, 3), (26.6, 30, 9, 5)]:
        x = theta / s
        R = planner.taylor_tail(x, m)
        sR = s * R
        trunc = sR * (1 - sR ** s) / (1 - sR)
        up = mp.mpf(2) * mp.sqrt(2) * mp.mpf(2) ** -53 / (1 - 2 * mp.mpf(2) ** -53)
        beta = mp.mpf(0)
        for k in range(m + 1):
            n = k * (sigma + 2) + m + 2
            beta += (n * up / (1 - n * up)) * mp.mpf(x) ** k / mp.factorial(k)
        alpha = 1 + mp.mpf(R)
        literal = (alpha + beta) ** s - alpha ** s
        got = planner.error_bound(theta, m, s, sigma) - trunc
        assert got == pytest.approx(float(literal), rel=1e-12)


def test_gamma_bounds_products_of_roundings():
    """|prod_{i<=n}(1+d_i) - 1| <= gamma_n for |d_i| <= u' (App. C.2), worst case d_i = u'."""
    up = planner.u_prime(planner.U_FP64)
    for n in (1, 3, 11, 100, 10_000):
        worst = (1 + mp.mpf(up)) ** n - 1
        assert float(worst) <= planner.gamma(n, up)
        assert planner.gamma(n, up) / float(worst) < 1.01


@pytest.mark.parametrize("theta", [0.01, 0.47, 2.3, 4.29, 8.46, 10.05, 11.66, 26.6, 41.0])
@pytest.mark.parametrize("sigma", [3, 5, 9])
def test_selection_is_minimal(theta, sigma):
    tau = 1e-12
    m, s = planner.select(theta, sigma, tau)
    assert planner.error_bound(theta, m, s, sigma) <= tau
    # no smaller s admits any m, and no smaller m works for this s
    for s2 in range(1, s):
        assert all(planner.error_bound(theta, mm, s2, sigma) > tau
                   for mm in range(1, planner.M_MAX + 1))
    for m2 in range(1, m):
        assert planner.error_bound(theta, m2, s, sigma) > tau


def test_selection_monotone_in_norm():
    thetas = np.linspace(0.05, 30, 60)
    sel = [planner.select(t, 9, 1e-12) for t in thetas]
    s_vals = [s for _, s in sel]
    assert all(b >= a for a, b in zip(s_vals, s_vals[1:]))
    # within one s the degree never decreases with the norm
    for (m1, s1), (m2, s2) in zip(sel, sel[1:]):
        if s1 == s2:
            assert m2 >= m1


def test_mu_grows_linearly_with_norm():
    """mu = m s grows roughly linearly with ||A||_1 at tau = 1e-8 (App. E
    observation, made there at the same tolerance)."""
    thetas = np.array([10.0, 20.0, 40.0, 80.0])
    mu = np.array([np.prod(planner.select(t, 5, 1e-8)) for t in thetas])
    ratios = mu[1:] / mu[:-1]
    assert np.all(ratios > 1.4) and np.all(ratios < 2.6)


def test_unreachable_tolerance():
    # the FP64 rounding floor makes 1e-15 unreachable already at a moderate norm
    with pytest.raises(ValueError):
        planner.select(5.0, 9, 1e-15)
    # and an FP32 roundoff cannot reach 1e-8 at a cfg3-sized norm
    with pytest.raises(ValueError):
        planner.select(10.0, 9, 1e-8, u=planner.U_FP32)
    with pytest.raises(ValueError):
        planner.select(float("nan"), 9, 1e-12)


# ---- the rounding part against the special cases the paper writes out ------
# App. C.2 spells out the per-component rounding bound for m = 0 (gamma_2) and
# for m = 1 (gamma_3 + gamma_{sigma+5} ||B||_1 after summing over the row, eq.
# c17); App. C.3 spells out the bound after s = 1 (beta, eq. s1) and s = 2
# (beta (beta + alpha) + beta alpha, eq. C22).  These are typed here from those
# printed forms, not from the general index k(sigma'+2)+m+2 of eq. B23, so a
# wrong index or a wrong composition over s in the oracle (or in the C++
# planner, checked the same way) fails.  A large unit roundoff keeps the
# rounding part well above the FP64 noise of the truncation part.
_U_BIG = mp.mpf(2) ** -20


def _gamma_printed(n):
    up = 2 * mp.sqrt(2) * _U_BIG / (1 - 2 * _U_BIG)
    return n * up / (1 - n * up)


def _printed_case(m, s, theta, sigma):
    x = mp.mpf(theta) / s
    if m == 0:
        beta = _gamma_printed(2)
    else:
        beta = _gamma_printed(3) + _gamma_printed(sigma + 5) * x
    R = _tail_mp(x, m)
    alpha = 1 + R
    rnd = beta if s == 1 else beta * (beta + alpha) + beta * alpha
    sR = s * R
    trunc = sR * (1 - sR ** s) / (1 - sR)
    return trunc, rnd


PRINTED_CASES = [(0, 1, 0.02, 3), (0, 2, 0.02, 5), (0, 1, 0.3, 9),
                 (1, 1, 0.05, 3), (1, 2, 0.05, 3), (1, 1, 0.2, 9), (1, 2, 0.4, 5), (1, 2, 0.1, 13)]


@pytest.mark.parametrize("m,s,theta,sigma", PRINTED_CASES)
def test_rounding_part_printed_special_cases(m, s, theta, sigma):
    trunc, rnd = _printed_case(m, s, theta, sigma)
    got = planner.error_bound(theta, m, s, sigma, u=float(_U_BIG))
    # the rounding part is ~1e-3..1e-2 of the total here, so comparing it alone
    # keeps FP64 noise of the total far below the tolerance
    assert got - float(trunc) == pytest.approx(float(rnd), rel=1e-9)
    assert got == pytest.approx(float(trunc + rnd), rel=1e-13)


@pytest.mark.parametrize("m,s,theta,sigma", [c for c in PRINTED_CASES if c[0] >= 1])
def test_library_rounding_part_printed_special_cases(m, s, theta, sigma):
    """The C++ planner's bound (hg_error_bound, m >= 1) against the same printed cases."""
    from paper_2304_06200_amd import _lib
    trunc, rnd = _printed_case(m, s, theta, sigma)
    got = _lib.hg_error_bound(theta, m, s, sigma, float(_U_BIG))
    assert got - float(trunc) == pytest.approx(float(rnd), rel=1e-9)

"""Planner variants (host and oracle): the fewest-products (m, s) choice, the
Chebyshev expansion the paper's Sec. III.B footnote names, and the scaling of
mu with the dimension that App. E reports for H_1, H_2 and H_3 at tau = 1e-8.

Pins: brute-force minimality of the min-mu rule; the C++ planner's min-mu
decisions bitwise equal to the oracle's; the Chebyshev coefficients against
the Jacobi-Anger identity on the unit circle (T_k(cos phi) = cos k phi) and the
Chebyshev action against scipy's expm within its truncation bound.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import chebyshev, planner

TAU = 1e-12


# ------------------------------------------------------------------- min-mu --
@pytest.mark.parametrize("theta", [0.3, 2.3, 8.5, 10.3, 11.7, 26.0, 28.4, 33.0, 41.0])
@pytest.mark.parametrize("sigma", [5, 9])
def test_min_mu_is_minimal(theta, sigma):
    m, s = planner.select_min_mu(theta, sigma, TAU)
    assert planner.error_bound(theta, m, s, sigma) <= TAU
    mu = m * s
    for s2 in range(1, mu + 1):
        for m2 in range(1, planner.M_MAX + 1):
            if m2 * s2 > mu or (m2 * s2 == mu and s2 >= s):
                break
            assert planner.error_bound(theta, m2, s2, sigma) > TAU, (m2, s2)


def test_min_mu_against_the_papers_rule():
    """min-mu never costs more than the paper's rule.  At tau = 1e-8 the two
    coincide on theta in [0.05, 45]; at tau = 1e-12 they coincide up to
    theta ~ 21.5 and min-mu saves at most ~5% of the products beyond (sigma' = 9)."""
    saved = []
    for tau in (1e-8, 1e-12):
        for th in np.linspace(0.05, 45.0, 120):
            a = planner.select(th, 9, tau)
            b = planner.select_min_mu(th, 9, tau)
            assert b[0] * b[1] <= a[0] * a[1]
            if tau == 1e-8 or th < 21.5:
                assert a == b, (tau, th, a, b)
            elif b != a:
                saved.append((a[0] * a[1] - b[0] * b[1]) / (a[0] * a[1]))
    assert saved and max(saved) < 0.05


def test_library_min_mu_matches_oracle_bitwise():
    from paper_2304_06200_amd import _lib
    rng = np.random.default_rng(17)
    thetas = np.concatenate([rng.uniform(0.0, 44.0, 60), [0.0, 1e-9, 10.3, 27.4, 28.2, 41.0]])
    for sigma in (5, 9):
        m, s = _lib.hg_plan_rule(thetas, sigma, TAU, 2.0 ** -53, _lib.HG_PLAN_MIN_MU)
        for t, mm, ss in zip(thetas, m, s):
            assert (int(mm), int(ss)) == planner.select_min_mu(float(t), sigma, TAU), (t, sigma)
    # the paper's rule through the same entry point is hg_plan
    m0, s0 = _lib.hg_plan_rule(thetas, 9, TAU, 2.0 ** -53, _lib.HG_PLAN_SMALLEST_S)
    m1, s1 = _lib.hg_plan(thetas, 9, TAU, 2.0 ** -53)
    assert np.array_equal(m0, m1) and np.array_equal(s0, s1)


# ---------------------------------------------------------------- Chebyshev --
@pytest.mark.parametrize("theta", [0.7, 4.0, 10.3, 23.0])
def test_chebyshev_coefficients_jacobi_anger(theta):
    """sum_k c_k cos(k phi) = exp(-i theta cos phi) once the tail is below 1e-15."""
    m = int(theta + 40)
    c = chebyshev.coefficients(theta, m)
    for phi in np.linspace(0.0, np.pi, 7):
        val = np.sum(c * np.cos(np.arange(m + 1) * phi))
        assert abs(val - np.exp(-1j * theta * np.cos(phi))) < 1e-13


@pytest.mark.parametrize("m", [5, 12, 25])
def test_chebyshev_truncation_bound_holds_on_scalars(m):
    theta = 10.0
    c = chebyshev.coefficients(theta, m)
    bound = chebyshev.truncation_bound(theta, m)
    worst = 0.0
    for x in np.linspace(-1.0, 1.0, 41):
        val = np.sum(c * np.cos(np.arange(m + 1) * np.arccos(x)))
        worst = max(worst, abs(val - np.exp(-1j * theta * x)))
    assert worst <= bound * (1 + 1e-9)
    assert worst > 0.1 * bound  # attained near x = +-1 to within an order of magnitude


def test_chebyshev_action_matches_expm():
    rng = np.random.default_rng(5)
    d = 40
    X = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    H = (X + X.conj().T) / 2
    dt = 0.7
    rho = float(np.max(np.sum(np.abs(H), axis=0)))
    psi = rng.normal(size=(d, 3)) + 1j * rng.normal(size=(d, 3))
    psi /= np.linalg.norm(psi, axis=0)
    exact = sla.expm(-1j * dt * H) @ psi
    for tau in (1e-6, 1e-10):
        m, s = chebyshev.select(dt * rho, int(d), tau)
        out = psi
        for _ in range(s):
            out = chebyshev.action(H, out, dt / s, m, rho)
        err = np.max(np.linalg.norm(out - exact, axis=0))
        assert err <= tau, (tau, m, s, err)


def test_chebyshev_needs_fewer_products_than_taylor():
    """The footnote's faster convergence: at the cfg3 norms (theta ~ 8-12,
    sigma' = 9, tau = 1e-12) a third or fewer of the Taylor products."""
    for th in (8.5, 10.3, 11.7):
        mt, st = planner.select(th, 9, TAU)
        mc, sc = chebyshev.select(th, 9, TAU)
        assert mc * sc * 2.5 < mt * st, (th, mc, sc, mt, st)


# ------------------------------------------------------- mu scaling (App. E) --
def _theta(H0, Hk, amps, dt):
    H = H0.copy()
    for a, h in zip(amps, Hk):
        H = H + a * h
    return dt * float(np.max(np.asarray(abs(H).sum(axis=0)))), H


def _sigma(H):
    return int(np.max(np.diff(sp.csr_matrix(H).indptr)))


def _fit_exponent(d, mu):
    return float(np.polyfit(np.log(d), np.log(mu), 1)[0])


def test_mu_scaling_transmon_cavity():
    """H_1 (eq. fockH; Delta/2pi = 3, g/2pi = 0.1, alpha/2pi = -0.225, a_z/2pi =
    a_x/2pi = 0.1 GHz, 6 transmon levels), d grown through the cavity:
    mu grows as d^(1/2) (App. E; the local exponent approaches 1/2 from below
    because the transmon terms add a constant to ||A||_1)."""
    from workloads.circuits import fock_transmon_cavity
    tp = 2 * np.pi
    ds, mus = [], []
    for dc in (2 ** 14, 2 ** 15, 2 ** 16, 2 ** 17):
        H0, Hk, _ = fock_transmon_cavity(6, dc, tp * 3.0, -tp * 0.225, tp * 0.1)
        th, H = _theta(H0, Hk, [tp * 0.1, tp * 0.1], 1.0)
        m, s = planner.select(th, _sigma(H), 1e-8)
        ds.append(6 * dc)
        mus.append(m * s)
    p = _fit_exponent(ds, mus)
    assert 0.38 <= p <= 0.55, p
    assert all(b > a for a, b in zip(mus, mus[1:]))


def test_mu_scaling_three_transmons():
    """H_2 (eq. gateH; alpha/2pi = -0.225, g/2pi = 0.1, a/2pi = 0.1 GHz), every
    transmon enlarged together: mu grows as d^(2/3) (App. E).  mu / ||A||_1
    itself creeps up slowly with the norm at this tolerance (about 4.1 to 4.5
    over the range), so the fitted exponent sits a little above 2/3."""
    from workloads.circuits import three_transmon_chain
    tp = 2 * np.pi
    ds, mus = [], []
    for dt_ in (16, 24, 32, 48, 64):
        H0, Hk, _ = three_transmon_chain(dt_, -tp * 0.225, tp * 0.1)
        th, H = _theta(H0, Hk, [tp * 0.1] * 3, 0.02)
        m, s = planner.select(th, _sigma(H), 1e-8)
        ds.append(dt_ ** 3)
        mus.append(m * s)
    p = _fit_exponent(ds, mus)
    assert 0.6 <= p <= 0.76, p


def test_mu_scaling_qubit_chain():
    """H_3 (driven qubit chain, a_x/2pi = a_y/2pi = 0.5 GHz, g/2pi = 0.1 GHz):
    mu grows linearly in the number of qubits, i.e. as log2 d (App. E)."""
    from workloads.circuits import qubit_chain
    tp = 2 * np.pi
    nq, mus = [], []
    for n in range(4, 15, 2):
        H0, Hk, _ = qubit_chain(n, tp * 0.1)
        th, H = _theta(H0, Hk, [tp * 0.5] * (2 * n), 1.0)
        m, s = planner.select(th, _sigma(H), 1e-8)
        nq.append(n)
        mus.append(m * s)
    coef = np.polyfit(nq, mus, 1)
    resid = np.array(mus) - np.polyval(coef, nq)
    assert coef[0] > 0 and np.max(np.abs(resid)) < 0.06 * max(mus), (mus, coef)

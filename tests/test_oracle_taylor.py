"""Pins of the Taylor-action and auxiliary-matrix oracle (Sec. III.B, App. C/D).

T8: the FP64 Taylor action at the planner's (m, s) stays within tau of a
50-digit mpmath reference (the paper's own check against a high-precision
Taylor reference, App. D).  T16: the bottom block of the auxiliary action is
the propagated state, and its top block matches the exact Frechet derivative
to within the bound.  The discrete-method gradient equals central finite
differences of the discrete cost with the schedule frozen.
"""
import mpmath as mp
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import grape, planner, taylor
from workloads import make_config

mp.mp.dps = 40


def _exact_action_mp(A: np.ndarray, psi: np.ndarray) -> np.ndarray:
    d = A.shape[0]
    Am = mp.matrix(d, d)
    for i in range(d):
        for j in range(d):
            Am[i, j] = mp.mpc(A[i, j].real, A[i, j].imag)
    v = mp.matrix(d, 1)
    for i in range(d):
        v[i] = mp.mpc(psi[i].real, psi[i].imag)
    out = mp.expm(Am) * v
    return np.array([complex(out[i]) for i in range(d)])


def _one_norm(A):
    return float(np.max(np.sum(np.abs(A), axis=0)))


@pytest.mark.parametrize("tau", [1e-8, 1e-10, 1e-12])
def test_action_error_below_tau_high_precision(tau):
    p = make_config("cfg2", d_c=6)  # transmon(3) x cavity(6), d = 18
    d = p.dim
    rng = np.random.default_rng(21)
    for n in (0, 17):
        H = (p.H0 + sum(p.u[k, n] * p.Hk[k] for k in range(p.n_ctrl))).toarray()
        A = -1j * 2.5 * H          # a larger step to exercise s > 1
        sigma = int(np.max(np.count_nonzero(A, axis=1)))
        m, s = planner.select(_one_norm(A), sigma, tau)
        psi = rng.standard_normal(d) + 1j * rng.standard_normal(d)
        psi /= np.linalg.norm(psi)
        ref = _exact_action_mp(A, psi)
        got = taylor.taylor_action(A, psi, m, s)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err <= tau
        assert err <= planner.error_bound(_one_norm(A), m, s, sigma)


def test_aux_bottom_is_propagated_state_and_top_is_frechet():
    p = make_config("cfg2", d_c=5)
    rng = np.random.default_rng(22)
    H = p.H0 + sum(p.u[k, 3] * p.Hk[k] for k in range(p.n_ctrl))
    A = (-1j * p.dt * H).tocsr()
    sigma = int(np.max(np.diff(A.indptr)))
    m, s = planner.select(_one_norm(A.toarray()), sigma, 1e-12)
    psi = rng.standard_normal(p.dim) + 1j * rng.standard_normal(p.dim)
    psi /= np.linalg.norm(psi)
    for k in range(p.n_ctrl):
        E = (-1j * p.dt * p.Hk[k]).tocsr()
        X, Y = taylor.aux_action(A, E, psi, m, s)
        np.testing.assert_allclose(Y, taylor.taylor_action(A, psi, m, s), rtol=0, atol=1e-15)
        L = grape.frechet_block(A.toarray(), E.toarray())
        np.testing.assert_allclose(X, L @ psi, rtol=0, atol=1e-11)


def _schedule(p, tau=1e-12):
    ms, ss = [], []
    for n in range(p.n_steps):
        H = (p.H0 + sum(p.u[k, n] * p.Hk[k] for k in range(p.n_ctrl))).toarray()
        A = -1j * p.dt * H
        sig = int(np.max(np.count_nonzero(A, axis=1)))
        m, s = planner.select(_one_norm(A), sig, tau)
        ms.append(m)
        ss.append(s)
    return np.array([ms, ss])


def test_discrete_gradient_equals_fd_of_discrete_cost():
    p = make_config("cfg2", d_c=4, N=6)
    sched = _schedule(p)
    kw = dict(omega=p.omega, w_fid=p.w_fid, w_pen=p.w_pen, w_int=0.7)
    r = taylor.hg_discrete(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets, sched, **kw)
    h = 1e-5
    for (k, n) in [(0, 0), (1, 3), (3, 5), (2, 2)]:
        up = p.u.copy(); up[k, n] += h
        um = p.u.copy(); um[k, n] -= h
        cp = taylor.hg_discrete(p.H0, p.Hk, up, p.dt, p.psi0, p.targets, sched, **kw)["cost"]
        cm = taylor.hg_discrete(p.H0, p.Hk, um, p.dt, p.psi0, p.targets, sched, **kw)["cost"]
        assert (cp - cm) / (2 * h) == pytest.approx(r["grad"][k, n], abs=1e-9)


def test_discrete_matches_exact_within_tau():
    p = make_config("cfg2", d_c=8, N=40)
    sched = _schedule(p)
    kw = dict(omega=p.omega, w_fid=p.w_fid, w_pen=p.w_pen, w_int=0.5)
    a = taylor.hg_discrete(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets, sched, **kw)
    b = grape.cost_and_grad(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets, **kw)
    assert a["cost"] == pytest.approx(b["cost"], rel=1e-11)
    assert a["integrated_infidelity"] == pytest.approx(b["integrated_infidelity"], rel=1e-11)
    assert np.linalg.norm(a["grad"] - b["grad"]) <= 1e-10 * np.linalg.norm(b["grad"])

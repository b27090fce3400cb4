"""Pins of the FP64 oracle against closed forms, invariants and brute force.

Each test fixes one part of oracle/grape.py against something other than the
oracle itself: textbook Rabi solutions, unitarity, central finite differences,
scipy's independent Frechet derivative, special cases of the cost, and the
explicit chain-rule sums (no co-state recursion).
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import grape

SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def _rand_herm(rng, d, scale=1.0):
    a = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    return scale * (a + a.conj().T) / 2


def _rand_states(rng, S, d):
    v = rng.standard_normal((S, d)) + 1j * rng.standard_normal((S, d))
    q, _ = np.linalg.qr(v.T)
    return q.T[:S]


def _small_problem(rng, d=5, K=2, N=6, S=2, penalty=True):
    H0 = _rand_herm(rng, d, 0.7)
    Hk = [_rand_herm(rng, d, 0.5) for _ in range(K)]
    u = rng.uniform(-1, 1, size=(K, N))
    psi0 = _rand_states(rng, S, d)
    tg = _rand_states(rng, S, d)
    om = (rng.uniform(size=d) < 0.4).astype(float) if penalty else None
    return H0, Hk, u, 0.3, psi0, tg, om


# ---- T1: resonant Rabi rotation, closed-form cost and gradient -------------
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rabi_closed_form(seed):
    rng = np.random.default_rng(seed)
    N, dt = 25, 0.1
    u = rng.uniform(-2, 2, size=(1, N))
    psi0 = np.array([[1, 0]], dtype=np.complex128)
    tg = np.array([[0, 1]], dtype=np.complex128)
    r = grape.cost_and_grad(np.zeros((2, 2)), [SX], u, dt, psi0, tg)
    th = dt * u.sum()
    assert r["cost"] == pytest.approx(np.cos(th) ** 2, abs=1e-13)
    np.testing.assert_allclose(r["grad"][0], -dt * np.sin(2 * th), atol=1e-12)


# ---- T1c: resonant Rabi, time-integrated infidelity C3 (App. A) -----------
# psi_n = cos(th_n)|0> - i sin(th_n)|1>, th_n = dt sum_{j<=n} u_j, so
# C3 = 1 - (1/N) sum_n sin^2(th_n) and dC3/du_k = -(dt/N) sum_{n>=k} sin(2 th_n)
@pytest.mark.parametrize("seed", [0, 1])
def test_rabi_time_integrated_closed_form(seed):
    rng = np.random.default_rng(seed)
    N, dt = 25, 0.1
    u = rng.uniform(-2, 2, size=(1, N))
    psi0 = np.array([[1, 0]], dtype=np.complex128)
    tg = np.array([[0, 1]], dtype=np.complex128)
    r = grape.cost_and_grad(np.zeros((2, 2)), [SX], u, dt, psi0, tg, w_fid=0.0, w_int=1.0)
    th = dt * np.cumsum(u[0])
    assert r["integrated_infidelity"] == pytest.approx(1 - np.mean(np.sin(th) ** 2), abs=1e-13)
    assert r["cost"] == pytest.approx(r["integrated_infidelity"], abs=1e-15)
    expect = -(dt / N) * np.cumsum(np.sin(2 * th)[::-1])[::-1]
    np.testing.assert_allclose(r["grad"][0], expect, atol=1e-12)


# ---- T1b: detuned Rabi, P1 = (a/Omega)^2 sin^2(Omega T), Omega^2 = a^2 + delta^2/4
@pytest.mark.parametrize("a,delta", [(0.7, 0.4), (1.3, -2.0), (0.2, 3.0)])
def test_detuned_rabi(a, delta):
    N, dt = 40, 0.05
    T = N * dt
    u = np.full((1, N), a)
    H0 = 0.5 * delta * SZ
    psi0 = np.array([[1, 0]], dtype=np.complex128)
    tg = np.array([[0, 1]], dtype=np.complex128)
    r = grape.cost_and_grad(H0, [SX], u, dt, psi0, tg)
    W = np.sqrt(a * a + delta * delta / 4)
    P1 = (a / W) ** 2 * np.sin(W * T) ** 2
    assert r["cost"] == pytest.approx(1 - P1, abs=1e-13)
    # for a constant drive, the sum over steps of dC/du_n is -dP1/da
    dW = a / W
    dP1 = (2 * a / W ** 2 - 2 * a ** 3 / W ** 4) * np.sin(W * T) ** 2 \
        + (a / W) ** 2 * 2 * np.sin(W * T) * np.cos(W * T) * T * dW
    assert r["grad"].sum() == pytest.approx(-dP1, abs=1e-11)


# ---- T2: unitarity and norm conservation ------------------------------------
def test_unitarity_and_norm():
    rng = np.random.default_rng(3)
    H0, Hk, u, dt, psi0, tg, om = _small_problem(rng, d=7, N=10, S=3)
    for n in range(u.shape[1]):
        U = grape.propagator(grape.hamiltonian(H0, Hk, u[:, n]), dt)
        np.testing.assert_allclose(U.conj().T @ U, np.eye(7), atol=1e-14)
    psi = grape.forward_states(H0, Hk, u, dt, psi0)
    np.testing.assert_allclose(np.linalg.norm(psi, axis=1), 1.0, atol=1e-14)
    # Pade forward agrees with the eigendecomposition form used backwards
    H = grape.hamiltonian(H0, Hk, u[:, 0])
    w, V = np.linalg.eigh(H)
    np.testing.assert_allclose(grape.propagator(H, dt),
                               V @ np.diag(np.exp(-1j * dt * w)) @ V.conj().T, atol=1e-13)


# ---- T3: central finite differences of the composite cost -------------------
@pytest.mark.parametrize("frechet", ["eig", "block"])
def test_finite_differences(frechet):
    rng = np.random.default_rng(4)
    H0, Hk, u, dt, psi0, tg, om = _small_problem(rng, d=6, K=2, N=5, S=2)
    kw = dict(omega=om, w_fid=1.0, w_pen=0.7, w_int=0.6)
    r = grape.cost_and_grad(H0, Hk, u, dt, psi0, tg, frechet=frechet, **kw)
    errs = {}
    for h in (1e-3, 1e-4):
        fd = np.zeros_like(u)
        for k in range(u.shape[0]):
            for n in range(u.shape[1]):
                up = u.copy(); up[k, n] += h
                um = u.copy(); um[k, n] -= h
                fd[k, n] = (grape.cost_only(H0, Hk, up, dt, psi0, tg, **kw)
                            - grape.cost_only(H0, Hk, um, dt, psi0, tg, **kw)) / (2 * h)
        errs[h] = np.max(np.abs(fd - r["grad"]))
    assert errs[1e-4] < 1e-8
    # second-order convergence: error drops by ~100 for a 10x smaller step
    assert errs[1e-3] / errs[1e-4] > 30


# ---- T4: three Frechet derivatives agree, also on a degenerate spectrum -----
@pytest.mark.parametrize("degenerate", [False, True])
def test_frechet_three_ways(degenerate):
    rng = np.random.default_rng(5)
    d, dt = 6, 0.8
    if degenerate:
        # transmon-like drift: levels 0 and 1 share energy 0 (n(n-1) = 0)
        H = np.diag(np.array([0.0, 0.0, -1.2, -3.6, 0.0, 2.5]))
    else:
        H = _rand_herm(rng, d)
    Eh = _rand_herm(rng, d)
    A = -1j * dt * H
    E = -1j * dt * Eh
    w, V = np.linalg.eigh(H)
    L_eig = grape.frechet_eig(w, V, dt, E)
    L_blk = grape.frechet_block(A, E)
    _, L_sp = sla.expm_frechet(A, E)
    np.testing.assert_allclose(L_eig, L_sp, atol=1e-12)
    np.testing.assert_allclose(L_blk, L_sp, atol=1e-12)


# ---- T5: Omega = identity => C2 = 1 and grad C2 = 0; Omega = 0 => C2 = 0 ----
def test_penalty_identity_and_zero():
    rng = np.random.default_rng(6)
    H0, Hk, u, dt, psi0, tg, _ = _small_problem(rng, d=5, N=7, S=2)
    r = grape.cost_and_grad(H0, Hk, u, dt, psi0, tg, omega=np.ones(5), w_fid=0.0, w_pen=1.0)
    assert r["penalty"] == pytest.approx(1.0, abs=1e-14)
    assert np.max(np.abs(r["grad"])) < 1e-13
    r0 = grape.cost_and_grad(H0, Hk, u, dt, psi0, tg, omega=np.zeros(5), w_fid=0.0, w_pen=1.0)
    assert r0["penalty"] == 0.0 and np.max(np.abs(r0["grad"])) == 0.0


# ---- T6: target = realised state => C1 = 0 and grad C1 = 0; phase invariance
def test_stationary_target_and_global_phase():
    rng = np.random.default_rng(7)
    H0, Hk, u, dt, psi0, _, om = _small_problem(rng, d=5, N=6, S=3)
    psiN = grape.forward_states(H0, Hk, u, dt, psi0)[-1].T
    r = grape.cost_and_grad(H0, Hk, u, dt, psi0, psiN)
    assert r["infidelity"] == pytest.approx(0.0, abs=1e-14)
    assert np.max(np.abs(r["grad"])) < 1e-13
    tg = _rand_states(rng, 3, 5)
    a = grape.cost_and_grad(H0, Hk, u, dt, psi0, tg, omega=om, w_pen=0.3)
    b = grape.cost_and_grad(H0, Hk, u, dt, psi0, np.exp(0.77j) * tg, omega=om, w_pen=0.3)
    assert a["cost"] == pytest.approx(b["cost"], abs=1e-14)
    np.testing.assert_allclose(a["grad"], b["grad"], atol=1e-13)


# ---- T7: commuting (diagonal) operators, closed-form gradient --------------
def test_commuting_closed_form():
    rng = np.random.default_rng(8)
    d, N, S, dt = 6, 9, 2, 0.4
    e = rng.uniform(-2, 2, d)
    f = rng.uniform(-1, 1, d)
    u = rng.uniform(-1, 1, (1, N))
    psi0 = _rand_states(rng, S, d)
    tg = _rand_states(rng, S, d)
    r = grape.cost_and_grad(np.diag(e), [np.diag(f)], u, dt, psi0, tg)
    phase = np.exp(-1j * dt * (N * e + u.sum() * f))
    psiN = phase[None, :] * psi0
    g = np.sum(np.conj(tg) * psiN) / S
    dg = np.sum(np.conj(tg) * (-1j * dt * f[None, :] * psiN)) / S   # same for every step
    assert r["cost"] == pytest.approx(1 - abs(g) ** 2, abs=1e-13)
    np.testing.assert_allclose(r["grad"][0], -2 * np.real(np.conj(g) * dg), atol=1e-13)


# ---- T11: co-state recursion equals the explicit chain-rule sums -----------
@pytest.mark.parametrize("seed", [9, 10])
def test_costate_vs_brute_force(seed):
    rng = np.random.default_rng(seed)
    H0, Hk, u, dt, psi0, tg, om = _small_problem(rng, d=4, K=2, N=5, S=2)
    kw = dict(omega=om, w_fid=0.8, w_pen=1.3, w_int=0.9)
    r = grape.cost_and_grad(H0, Hk, u, dt, psi0, tg, **kw)
    bf = grape.gradient_brute_force(H0, Hk, u, dt, psi0, tg, **kw)
    np.testing.assert_allclose(r["grad"], bf, atol=1e-13)


# ---- gate infidelity: S = d full basis reduces to 1 - |tr(U_T^dag U_R)/d|^2 --
def test_full_basis_is_gate_infidelity():
    rng = np.random.default_rng(11)
    d, K, N, dt = 4, 2, 5, 0.5
    H0, Hk, u, _, _, _, _ = _small_problem(rng, d=d, K=K, N=N, S=1)
    UT = np.linalg.qr(rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d)))[0]
    psi0 = np.eye(d, dtype=np.complex128)
    tg = (UT @ psi0.T).T
    r = grape.cost_and_grad(H0, Hk, u, dt, psi0, tg)
    UR = np.eye(d, dtype=np.complex128)
    for n in range(N):
        UR = grape.propagator(grape.hamiltonian(H0, Hk, u[:, n]), dt) @ UR
    assert r["infidelity"] == pytest.approx(1 - abs(np.trace(UT.conj().T @ UR) / d) ** 2, abs=1e-13)


def test_sparse_and_dense_inputs_agree():
    rng = np.random.default_rng(12)
    H0, Hk, u, dt, psi0, tg, om = _small_problem(rng, d=5, N=4, S=2)
    a = grape.cost_and_grad(H0, Hk, u, dt, psi0, tg, omega=om, w_pen=0.5)
    b = grape.cost_and_grad(sp.csr_matrix(H0), [sp.csr_matrix(h) for h in Hk], u, dt, psi0, tg,
                            omega=om, w_pen=0.5)
    assert a["cost"] == b["cost"]
    np.testing.assert_array_equal(a["grad"], b["grad"])


# ---- C3^g: with a full basis the time-integrated cost is App. A's gate form --
def test_full_basis_time_integrated_gate_infidelity():
    rng = np.random.default_rng(12)
    d, K, N, dt = 4, 2, 6, 0.5
    H0, Hk, u, _, _, _, _ = _small_problem(rng, d=d, K=K, N=N, S=1)
    UT = np.linalg.qr(rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d)))[0]
    psi0 = np.eye(d, dtype=np.complex128)
    tg = (UT @ psi0.T).T
    r = grape.cost_and_grad(H0, Hk, u, dt, psi0, tg, w_fid=0.0, w_int=1.0)
    UR = np.eye(d, dtype=np.complex128)
    acc = 0.0
    for n in range(N):
        UR = grape.propagator(grape.hamiltonian(H0, Hk, u[:, n]), dt) @ UR
        acc += abs(np.trace(UT.conj().T @ UR)) ** 2
    assert r["integrated_infidelity"] == pytest.approx(1 - acc / (N * d * d), abs=1e-13)


# ---- C3 with one step is C1 -----------------------------------------------
def test_time_integrated_single_step_is_final_infidelity():
    rng = np.random.default_rng(13)
    H0, Hk, u, dt, psi0, tg, _ = _small_problem(rng, d=5, N=1, S=2)
    a = grape.cost_and_grad(H0, Hk, u, dt, psi0, tg, w_fid=0.0, w_int=1.0)
    b = grape.cost_and_grad(H0, Hk, u, dt, psi0, tg, w_fid=1.0)
    assert a["cost"] == pytest.approx(b["cost"], abs=1e-14)
    np.testing.assert_allclose(a["grad"], b["grad"], atol=1e-14)

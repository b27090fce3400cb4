"""Exact FP64 cost and gradient of piecewise-constant GRAPE (oracle; tests only).

Notation follows the paper (arXiv:2304.06200):
  H_n   = H_s + sum_k u[k, n] h_k                  Sec. II (reading: H_n is the
          Hamiltonian itself, A_n = -i dt H_n the exponent, as in eq. propagator
          and Sec. III.B; the printed "H_n = -i(...)dt" is taken as a typo)
  U_n   = exp(-i H_n dt)                            Sec. II, eq. propagator
  psi_n = U_n psi_{n-1}                             Sec. II, eq. statepropagation
  g     = (1/S) sum_h <phi_T^h | psi_N^h>           Sec. III.A (C1^st for S=1,
          tr(U_T^dag U_R)/d when the S states are a full basis, eq. gategradient)
  C1    = 1 - |g|^2                                 Sec. III.A, eq. C1st
  C2    = 1/(N S) sum_h sum_{n'=1..N} <psi_n'|Omega|psi_n'>   App. A, eq. c2st
  g_n   = (1/S) sum_h <phi_T^h | psi_n^h>           (overlap after step n)
  C3    = 1 - (1/N) sum_{n'=1..N} |g_n'|^2          App. A (time-integrated
          infidelity: C3^st for S=1, C3^g when the S states are a full basis)
  C     = w_fid C1 + w_pen C2 + w_int C3            Sec. II (composite cost)

Gradient (Sec. III.A eqs. stgradient / gategradient, App. A eqs. C2stgrad and
state time gradient):
  dC/du[k,n] = 2 Re sum_h <Lambda_n^h | dU_n/du_k | psi_{n-1}^h>
  Lambda_N   = -(w_fid g / S) phi_T + src_N
  Lambda_n-1 = U_n^dag Lambda_n + src_{n-1}                         (n-1 >= 1)
  src_n      = (w_pen/(N S)) Omega psi_n - (w_int/(N S)) g_n phi_T
The fidelity part is eq. stgradient with the factor conj(g) folded into the
co-state (linearity); the penalty part is the Phi_n recursion of App. A, the
time-integrated part its Phi_{T,n} recursion (one source per step).
dU_n/du_k is the Frechet derivative L(A_n, E_k) of expm at A_n = -i dt H_n in
direction E_k = -i dt h_k.

The forward pass uses scipy's Pade scaling-and-squaring expm and stores every
state, so no inverse reconstruction is involved.  The backward pass uses the
eigendecomposition of H_n (App. F) for U_n^dag and, by default, for the
Frechet derivative.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def _dense(m) -> np.ndarray:
    if sp.issparse(m):
        return np.asarray(m.toarray(), dtype=np.complex128)
    return np.asarray(m, dtype=np.complex128)


def hamiltonian(H0: np.ndarray, Hk: Sequence[np.ndarray], u_n: np.ndarray) -> np.ndarray:
    """H_n = H_s + sum_k u_kn h_k (Sec. II, multiple control channels as in its
    footnote on the generalisation to several channels)."""
    H = H0.copy()
    for k, h in enumerate(Hk):
        H = H + u_n[k] * h
    return H


def propagator(H: np.ndarray, dt: float) -> np.ndarray:
    """U = exp(-i H dt) by dense Pade scaling and squaring (Sec. II, eq. propagator)."""
    return sla.expm(-1j * dt * H)


def frechet_block(A: np.ndarray, E: np.ndarray) -> np.ndarray:
    """L(A, E): upper-right block of expm([[A, E], [0, A]]) -- the auxiliary
    block-matrix identity of Sec. III.B (eq. auxiliary equation) with the
    exact exponential in place of the truncated series."""
    d = A.shape[0]
    big = np.zeros((2 * d, 2 * d), dtype=np.complex128)
    big[:d, :d] = A
    big[:d, d:] = E
    big[d:, d:] = A
    return sla.expm(big)[:d, d:]


def divided_difference_exp(a: np.ndarray) -> np.ndarray:
    """Gamma_ij = (e^{a_i} - e^{a_j}) / (a_i - a_j), with e^{a_i} on coinciding
    eigenvalues, for purely imaginary a (eigenvalues of -i dt H).

    This is App. F's factor (e^D + E o F) with the degenerate entries kept:
    with delta = a_i - a_j = 2 i y it equals exp((a_i + a_j)/2) * sin(y)/y,
    which is finite and exact at y = 0 (reading of the degenerate case)."""
    y = (a[:, None] - a[None, :]).imag / 2.0
    mid = np.exp((a[:, None] + a[None, :]) / 2.0)
    return mid * np.sinc(y / np.pi)


def frechet_eig(w: np.ndarray, V: np.ndarray, dt: float, E: np.ndarray) -> np.ndarray:
    """L(A, E) for A = -i dt H with H = V diag(w) V^dag (App. F, eq. propagator der):
    dU = V [Gamma o (V^dag E V)] V^dag."""
    a = -1j * dt * w
    G = divided_difference_exp(a)
    return V @ (G * (V.conj().T @ E @ V)) @ V.conj().T


def forward_states(H0, Hk, u, dt, psi0) -> np.ndarray:
    """All states psi_0..psi_N as an array (N+1, d, S) (Sec. II, eq. statepropagation)."""
    H0d = _dense(H0)
    Hkd = [_dense(h) for h in Hk]
    K, N = u.shape
    d = H0d.shape[0]
    S = psi0.shape[0]
    psi = np.empty((N + 1, d, S), dtype=np.complex128)
    psi[0] = np.asarray(psi0, dtype=np.complex128).T
    for n in range(1, N + 1):
        U = propagator(hamiltonian(H0d, Hkd, u[:, n - 1]), dt)
        psi[n] = U @ psi[n - 1]
    return psi


def step_overlaps(psi: np.ndarray, targets: np.ndarray) -> np.ndarray:
    """g_n = (1/S) sum_h <phi_T^h | psi_n^h> for n = 0..N (complex, (N+1,))."""
    S = psi.shape[2]
    return np.einsum("hd,ndh->n", np.conj(targets), psi) / S


def cost_terms(psi: np.ndarray, targets: np.ndarray, omega: Optional[np.ndarray],
               w_fid: float, w_pen: float, w_int: float = 0.0):
    """Cost parts from stored states (Sec. III.A eq. C1st; App. A eq. c2st and
    the time-integrated infidelity).  Returns g, C1, C2, C3, C."""
    N = psi.shape[0] - 1
    S = psi.shape[2]
    g = np.sum(np.conj(targets.T) * psi[N]) / S
    C1 = 1.0 - abs(g) ** 2
    if omega is not None:
        occ = np.sum(omega[None, :, None] * np.abs(psi[1:]) ** 2)
        C2 = float(occ) / (N * S)
    else:
        C2 = 0.0
    gn = step_overlaps(psi, targets)
    C3 = 1.0 - float(np.sum(np.abs(gn[1:]) ** 2)) / N
    return g, C1, C2, C3, w_fid * C1 + w_pen * C2 + w_int * C3


def cost_and_grad(H0, Hk, u, dt, psi0, targets, omega=None, w_fid=1.0, w_pen=0.0,
                  frechet: str = "eig", want_states: bool = False, w_int: float = 0.0) -> dict:
    """Exact cost and gradient of the composite cost (oracle).

    H0, Hk   drift and control operators (dense or scipy.sparse), (d, d)
    u        (K, N) control amplitudes
    psi0     (S, d) initial states, targets (S, d) target states phi_T^h
    omega    (d,) diagonal of the Hermitian penalty operator Omega, or None
    frechet  "eig" (Daleckii-Krein in the eigenbasis of H_n, App. F) or
             "block" (Van Loan block exponential, Sec. III.B identity)
    w_int    weight of the time-integrated infidelity C3 (App. A)
    Returns a dict with cost, infidelity (C1), penalty (C2), integrated
    infidelity (C3), overlap g, grad (K, N) and, on request, the stored states.
    """
    u = np.asarray(u, dtype=np.float64)
    K, N = u.shape
    H0d = _dense(H0)
    Hkd = [_dense(h) for h in Hk]
    d = H0d.shape[0]
    psi0 = np.asarray(psi0, dtype=np.complex128)
    targets = np.asarray(targets, dtype=np.complex128)
    S = psi0.shape[0]
    om = None if omega is None else np.asarray(omega, dtype=np.float64)

    psi = forward_states(H0d, Hkd, u, dt, psi0)
    g, C1, C2, C3, C = cost_terms(psi, targets, om, w_fid, w_pen, w_int)
    gn = step_overlaps(psi, targets)

    cpen = (w_pen / (N * S)) if om is not None else 0.0
    cint = w_int / (N * S)

    def source(n):
        # co-state source of step n: penalty (Phi_n) and time-integrated (Phi_T,n)
        src = -cint * gn[n] * targets.T
        if om is not None:
            src = src + cpen * om[:, None] * psi[n]
        return src

    lam = -(w_fid * g / S) * targets.T.copy() + source(N)

    E = [-1j * dt * h for h in Hkd]
    grad = np.zeros((K, N), dtype=np.float64)
    for n in range(N, 0, -1):
        H = hamiltonian(H0d, Hkd, u[:, n - 1])
        w, V = np.linalg.eigh(H)
        prev = psi[n - 1]
        if frechet == "block":
            A = -1j * dt * H
            for k in range(K):
                L = frechet_block(A, E[k])
                grad[k, n - 1] = 2.0 * np.real(np.sum(np.conj(lam) * (L @ prev)))
        else:
            a = -1j * dt * w
            G = divided_difference_exp(a)
            pt = V.conj().T @ prev          # (d, S) in the eigenbasis
            lt = V.conj().T @ lam
            M = pt @ lt.conj().T            # sum_h psi~^h lam~^h^dag
            Q = V @ (G.T * M) @ V.conj().T  # sum_h <lam|L(A,E)|psi> = tr(E Q)
            for k in range(K):
                grad[k, n - 1] = 2.0 * np.real(np.sum(E[k] * Q.T))
        if n - 1 >= 1:
            # Lambda_{n-1} = U_n^dag Lambda_n + src_{n-1}, U_n^dag = V e^{+i dt w} V^dag
            lam = V @ (np.exp(1j * dt * w)[:, None] * (V.conj().T @ lam)) + source(n - 1)
    out = {"cost": float(C), "infidelity": float(C1), "penalty": float(C2),
           "integrated_infidelity": float(C3), "overlap": complex(g), "grad": grad}
    if want_states:
        out["states"] = psi
    return out


def cost_only(H0, Hk, u, dt, psi0, targets, omega=None, w_fid=1.0, w_pen=0.0,
              w_int=0.0) -> float:
    """The composite cost alone (used by finite-difference pins)."""
    psi = forward_states(H0, Hk, np.asarray(u, dtype=np.float64), dt,
                         np.asarray(psi0, dtype=np.complex128))
    om = None if omega is None else np.asarray(omega, dtype=np.float64)
    return float(cost_terms(psi, np.asarray(targets, dtype=np.complex128), om,
                            w_fid, w_pen, w_int)[4])


def gradient_brute_force(H0, Hk, u, dt, psi0, targets, omega=None, w_fid=1.0, w_pen=0.0,
                         w_int=0.0):
    """Gradient by the explicit chain-rule sums, without any co-state recursion:
    d psi_n'/du[k,n] = U_n' ... U_{n+1} L(A_n, E_k) psi_{n-1} for n' >= n (the
    first lines of eqs. stgradient and C2stgrad).  O(N^2) products: tiny cases only."""
    u = np.asarray(u, dtype=np.float64)
    K, N = u.shape
    H0d = _dense(H0)
    Hkd = [_dense(h) for h in Hk]
    psi0 = np.asarray(psi0, dtype=np.complex128)
    targets = np.asarray(targets, dtype=np.complex128)
    S = psi0.shape[0]
    om = None if omega is None else np.asarray(omega, dtype=np.float64)
    psi = forward_states(H0d, Hkd, u, dt, psi0)
    g = cost_terms(psi, targets, om, w_fid, w_pen, w_int)[0]
    gn = step_overlaps(psi, targets)
    Hs = [hamiltonian(H0d, Hkd, u[:, n]) for n in range(N)]
    Us = [propagator(H, dt) for H in Hs]
    grad = np.zeros((K, N))
    for n in range(1, N + 1):
        A = -1j * dt * Hs[n - 1]
        for k in range(K):
            dpsi = frechet_block(A, -1j * dt * Hkd[k]) @ psi[n - 1]   # d psi_n
            total = 0.0
            for npr in range(n, N + 1):
                if npr > n:
                    dpsi = Us[npr - 1] @ dpsi
                if om is not None and w_pen != 0.0:
                    total += w_pen / (N * S) * 2.0 * np.real(
                        np.sum(np.conj(psi[npr]) * (om[:, None] * dpsi)))
                if w_int != 0.0:
                    # d|g_n'|^2 = 2 Re conj(g_n') dg_n'
                    dgn = np.sum(np.conj(targets.T) * dpsi) / S
                    total -= w_int / N * 2.0 * np.real(np.conj(gn[npr]) * dgn)
            dg = np.sum(np.conj(targets.T) * dpsi) / S
            total += w_fid * (-2.0 * np.real(np.conj(g) * dg))
            grad[k, n - 1] = total
    return grad

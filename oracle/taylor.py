"""The paper's Taylor scaling-and-squaring action and auxiliary-matrix
derivative, written plainly in FP64 (oracle; tests only).

  e^A |Psi> ~ (T_m(A/s))^s |Psi>,  T_m(B) = sum_{q<=m} B^q / q!
      Sec. III.B, eqs. scaling squaring, eBm, eBmpsi; evaluated by repeated
      matrix-vector products: b_j = (B/j) b_{j-1}, partial sums S_j = S_{j-1} + b_j
      (App. C.2, recursion relation 1; the printed "e^B_j b_0 = b_{j-1} + b_j"
      is read as this partial-sum update), and c_l = T_m(B) c_{l-1}
      (App. C.3, recursion relation 2).

  (T_m(Aux/s))^s (0; Psi) = (d/du (T_m(B))^s Psi ; (T_m(B))^s Psi),
      Aux = [[A, E], [0, A]],  E = dA/du = -i dt h     Sec. III.B, eq. auxiliary equation.
      Here the 2d x 2d block matrix is built explicitly and pushed through the
      same Taylor routine as any other matrix.

  hg_discrete: cost and gradient of the *discretised* method (every U_n replaced
      by (T_{m_n}(A_n/s_n))^{s_n}), with all forward states stored.  It is the
      exact gradient of that discrete cost, the quantity the GPU path computes
      before rounding, so the two agree to rounding error rather than to tau.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np
import scipy.sparse as sp


def taylor_action(A, psi: np.ndarray, m: int, s: int) -> np.ndarray:
    """(T_m(A/s))^s psi by 1 + m s matrix-vector products (Sec. III.B)."""
    c = np.array(psi, dtype=np.complex128, copy=True)
    for _ in range(s):
        b = c
        acc = c.copy()
        for j in range(1, m + 1):
            b = (A @ b) / (s * j)
            acc = acc + b
        c = acc
    return c


def aux_action(A, E, psi: np.ndarray, m: int, s: int):
    """(X, Y) with (X; Y) = (T_m(Aux/s))^s (0; psi), Aux = [[A, E], [0, A]]
    (Sec. III.B, eq. auxiliary equation).  Returns (derivative action, propagated psi)."""
    d = A.shape[0]
    if sp.issparse(A) or sp.issparse(E):
        big = sp.bmat([[sp.csr_matrix(A), sp.csr_matrix(E)], [None, sp.csr_matrix(A)]],
                      format="csr")
    else:
        big = np.zeros((2 * d, 2 * d), dtype=np.complex128)
        big[:d, :d] = A
        big[:d, d:] = E
        big[d:, d:] = A
    v = np.concatenate([np.zeros_like(psi, dtype=np.complex128),
                        np.asarray(psi, dtype=np.complex128)], axis=0)
    out = taylor_action(big, v, m, s)
    return out[:d], out[d:]


def hg_discrete(H0, Hk: Sequence, u, dt, psi0, targets, schedule, omega=None,
                w_fid=1.0, w_pen=0.0, w_int=0.0) -> dict:
    """Cost and gradient of the Taylor-discretised problem (oracle).

    schedule: (2, N) int array, rows m_n and s_n.  The cost is the composite
    cost of Sec. II with psi_n = (T_{m_n}(A_n/s_n))^{s_n} psi_{n-1}; the
    gradient uses the same co-state recursion as the exact oracle with U_n^dag
    replaced by the adjoint of the Taylor map (T_m(B))^dag = T_m(B^dag) = T_m(-B)
    for anti-Hermitian B, and dU_n/du_k psi replaced by the auxiliary action.
    """
    u = np.asarray(u, dtype=np.float64)
    K, N = u.shape
    H0 = sp.csr_matrix(H0, dtype=np.complex128)
    Hk = [sp.csr_matrix(h, dtype=np.complex128) for h in Hk]
    psi0 = np.asarray(psi0, dtype=np.complex128)
    targets = np.asarray(targets, dtype=np.complex128)
    S = psi0.shape[0]
    ms = np.asarray(schedule[0], dtype=np.int64)
    ss = np.asarray(schedule[1], dtype=np.int64)

    def A_of(n):
        H = H0.copy()
        for k in range(K):
            H = H + u[k, n - 1] * Hk[k]
        return -1j * dt * H

    psi = [psi0.T.copy()]
    for n in range(1, N + 1):
        psi.append(taylor_action(A_of(n), psi[-1], int(ms[n - 1]), int(ss[n - 1])))
    g = np.sum(np.conj(targets.T) * psi[N]) / S
    C1 = 1.0 - abs(g) ** 2
    if omega is not None:
        om = np.asarray(omega, dtype=np.float64)
        C2 = sum(float(np.sum(om[:, None] * np.abs(psi[n]) ** 2)) for n in range(1, N + 1)) / (N * S)
    else:
        om = None
        C2 = 0.0
    # time-integrated infidelity C3 = 1 - (1/N) sum_n |g_n|^2 (App. A)
    gn = [np.sum(np.conj(targets.T) * psi[n]) / S for n in range(N + 1)]
    C3 = 1.0 - sum(abs(gn[n]) ** 2 for n in range(1, N + 1)) / N
    cpen = (w_pen / (N * S)) if om is not None else 0.0
    cint = w_int / (N * S)

    def source(n):
        src = -cint * gn[n] * targets.T
        if om is not None:
            src = src + cpen * om[:, None] * psi[n]
        return src

    lam = -(w_fid * g / S) * targets.T + source(N)
    grad = np.zeros((K, N))
    for n in range(N, 0, -1):
        A = A_of(n)
        m, s = int(ms[n - 1]), int(ss[n - 1])
        for k in range(K):
            X, _ = aux_action(A, -1j * dt * Hk[k], psi[n - 1], m, s)
            grad[k, n - 1] = 2.0 * np.real(np.sum(np.conj(lam) * X))
        if n - 1 >= 1:
            lam = taylor_action(-A, lam, m, s) + source(n - 1)
    return {"cost": float(w_fid * C1 + w_pen * C2 + w_int * C3), "infidelity": float(C1),
            "penalty": float(C2), "integrated_infidelity": float(C3), "overlap": complex(g),
            "grad": grad, "final_states": psi[N].T.copy()}

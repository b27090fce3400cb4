"""Operator builders for the synthetic circuit-QED workloads (inputs only).

Every operator is returned as a ``scipy.sparse.csr_matrix`` of complex128 with
sorted indices and no explicit zeros.  The product basis is ordered with the
last factor running fastest (``kron(A, B)`` convention), so for a transmon
(levels t) times a cavity (levels c) the basis index is ``t * d_c + c``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import scipy.sparse as sp


def destroy(n: int) -> sp.csr_matrix:
    """Annihilation operator truncated to ``n`` levels: <k-1|a|k> = sqrt(k)."""
    data = np.sqrt(np.arange(1, n, dtype=np.float64)).astype(np.complex128)
    return sp.diags(data, offsets=1, shape=(n, n), format="csr", dtype=np.complex128)


def number(n: int) -> sp.csr_matrix:
    """Number operator b^dagger b truncated to ``n`` levels."""
    return sp.diags(np.arange(n, dtype=np.float64).astype(np.complex128), 0,
                    shape=(n, n), format="csr", dtype=np.complex128)


def embed(op: sp.spmatrix, which: int, dims: Sequence[int]) -> sp.csr_matrix:
    """Place ``op`` on tensor factor ``which`` of a product space with ``dims``."""
    out = None
    for i, d in enumerate(dims):
        f = op if i == which else sp.identity(d, dtype=np.complex128, format="csr")
        out = f if out is None else sp.kron(out, f, format="csr")
    return _clean(out)


def _clean(m: sp.spmatrix) -> sp.csr_matrix:
    m = sp.csr_matrix(m, dtype=np.complex128)
    m.eliminate_zeros()
    m.sort_indices()
    return m


def _drives(a: sp.spmatrix):
    """x and y quadrature drive operators of one mode: a + a^dag, i(a^dag - a)."""
    ad = a.conj().T
    return _clean(a + ad), _clean(1j * (ad - a))


def transmon_cavity_system(d_t: int, d_c: int, alpha: float, chi: float):
    """Transmon (d_t levels) dispersively coupled to a cavity (d_c levels).

    Drift   H0 = (alpha/2) n_t (n_t - 1) + chi n_t n_c   (rotating frame)
    Drives  x, y on the transmon, then x, y on the cavity.
    This is the structure of the paper's transmon-cavity benchmark system
    (Sec. IV.B, H_1) in the dispersive limit with the drive in the frame.
    """
    dims = (d_t, d_c)
    b = embed(destroy(d_t), 0, dims)
    c = embed(destroy(d_c), 1, dims)
    nt = embed(number(d_t), 0, dims)
    nc = embed(number(d_c), 1, dims)
    ident = sp.identity(d_t * d_c, dtype=np.complex128, format="csr")
    H0 = _clean(0.5 * alpha * (nt @ (nt - ident)) + chi * (nt @ nc))
    bx, by = _drives(b)
    cx, cy = _drives(c)
    return H0, [bx, by, cx, cy], dims


def three_transmon_chain(d_t: int, alpha: float, g: float):
    """Three resonantly driven transmons (d_t levels each) with nearest-neighbour
    exchange, in the rotating frame (Sec. IV.B, eq. gateH):

    H0 = sum_nu (alpha/2) n_nu (n_nu - 1) + g (b1 b2^dag + b2 b3^dag + h.c.)
    Drives: b_nu + b_nu^dag for nu = 1, 2, 3 (three controls).
    """
    dims = (d_t, d_t, d_t)
    b = [embed(destroy(d_t), i, dims) for i in range(3)]
    n = [embed(number(d_t), i, dims) for i in range(3)]
    ident = sp.identity(d_t ** 3, dtype=np.complex128, format="csr")
    H0 = sum(0.5 * alpha * (n[i] @ (n[i] - ident)) for i in range(3))
    hop = b[0] @ b[1].conj().T + b[1] @ b[2].conj().T
    H0 = _clean(H0 + g * (hop + hop.conj().T))
    return H0, [_clean(bi + bi.conj().T) for bi in b], dims


def two_transmon_cavity_system(d_t: int, d_c: int, alpha: float, chi: float, g: float):
    """Two transmons (d_t levels each) sharing a cavity (d_c levels).

    H0 = sum_j [(alpha/2) n_j (n_j - 1) + chi n_j n_c] + g (b1 b2^dag + b2 b1^dag)
    Drives: x, y on b1, on b2, then on the cavity (six controls).
    """
    dims = (d_t, d_t, d_c)
    b1 = embed(destroy(d_t), 0, dims)
    b2 = embed(destroy(d_t), 1, dims)
    c = embed(destroy(d_c), 2, dims)
    n1 = embed(number(d_t), 0, dims)
    n2 = embed(number(d_t), 1, dims)
    nc = embed(number(d_c), 2, dims)
    ident = sp.identity(d_t * d_t * d_c, dtype=np.complex128, format="csr")
    H0 = (0.5 * alpha * (n1 @ (n1 - ident)) + 0.5 * alpha * (n2 @ (n2 - ident))
          + chi * (n1 @ nc) + chi * (n2 @ nc)
          + g * (b1 @ b2.conj().T + b2 @ b1.conj().T))
    ctrls = []
    for a in (b1, b2, c):
        ctrls.extend(_drives(a))
    return _clean(H0), ctrls, dims


def haar_unitary(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random n x n unitary: QR of a complex Ginibre matrix with the
    phases of R's diagonal moved into Q (Mezzadri 2007)."""
    z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diagonal(r) / np.abs(np.diagonal(r))
    return q * ph[None, :]


def basis_state(d: int, index: int) -> np.ndarray:
    v = np.zeros(d, dtype=np.complex128)
    v[index] = 1.0
    return v


@dataclass
class Problem:
    """One cost+gradient evaluation request (host arrays, FP64)."""
    name: str
    H0: sp.csr_matrix
    Hk: List[sp.csr_matrix]
    dt: float
    u: np.ndarray                 # (K, N) float64 control amplitudes, rad/ns
    psi0: np.ndarray              # (S, d) complex128 initial states (rows)
    targets: np.ndarray           # (S, d) complex128 target states (rows)
    omega: Optional[np.ndarray]   # (d,) float64 diagonal of the penalty operator, or None
    w_fid: float = 1.0
    w_pen: float = 0.0
    tau: float = 1e-12
    dims: tuple = ()
    meta: dict = field(default_factory=dict)

    @property
    def dim(self) -> int:
        return self.H0.shape[0]

    @property
    def n_ctrl(self) -> int:
        return len(self.Hk)

    @property
    def n_steps(self) -> int:
        return self.u.shape[1]

    @property
    def n_states(self) -> int:
        return self.psi0.shape[0]


def fock_transmon_cavity(d_t: int, d_c: int, delta: float, alpha: float, g: float):
    """The paper's Fock-state benchmark system (Sec. IV.B, eq. fockH), in the
    frame co-rotating with the transmon drive:

    H0 = Delta b^dag b + (alpha/2) b^dag b (b^dag b - 1) + g (c b^dag + c^dag b)
    Controls: b^dag b (longitudinal a_z) and b + b^dag (transverse a_x).
    Product basis transmon x cavity (cavity index fastest).
    """
    dims = (d_t, d_c)
    b = embed(destroy(d_t), 0, dims)
    c = embed(destroy(d_c), 1, dims)
    nt = embed(number(d_t), 0, dims)
    ident = sp.identity(d_t * d_c, dtype=np.complex128, format="csr")
    H0 = delta * nt + 0.5 * alpha * (nt @ (nt - ident)) + g * (c @ b.conj().T + c.conj().T @ b)
    return _clean(H0), [_clean(nt), _clean(b + b.conj().T)], dims


def qubit_chain(n_q: int, g: float):
    """Driven qubit chain with nearest-neighbour sigma_z coupling (App. E, H_3):

    H0 = g sum_{nu < n_q} sigma_z^(nu) sigma_z^(nu+1)
    Controls: sigma_x^(nu), sigma_y^(nu) for every qubit (x then y, qubit by qubit).
    """
    sx = sp.csr_matrix(np.array([[0, 1], [1, 0]], dtype=np.complex128))
    sy = sp.csr_matrix(np.array([[0, -1j], [1j, 0]], dtype=np.complex128))
    sz = sp.csr_matrix(np.array([[1, 0], [0, -1]], dtype=np.complex128))
    dims = (2,) * n_q
    z = [embed(sz, i, dims) for i in range(n_q)]
    H0 = sp.csr_matrix((2 ** n_q, 2 ** n_q), dtype=np.complex128)
    for i in range(n_q - 1):
        H0 = H0 + g * (z[i] @ z[i + 1])
    ctrls = []
    for i in range(n_q):
        ctrls.extend([embed(sx, i, dims), embed(sy, i, dims)])
    return _clean(H0), ctrls, dims

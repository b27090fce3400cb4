"""Matrix-diagonalisation HG (App. F) on the GPU: per step a Jacobi
eigendecomposition of H_n, U_n = V e^{-i dt D} V^H, and the derivative from
the divided differences of exp in the eigenbasis.  Parity is checked against
the oracle's Pade forward pass with the Van Loan block Frechet derivative
(frechet="block"), which shares nothing with the eigenbasis formula.

Cases: dense random Hermitian operators (penalty, time-integrated infidelity,
one state and several), the full-basis three-transmon gate with odd and even
dimensions, a degenerate spectrum (no drive, transmon anharmonicity only on two
levels), a batch, agreement with the Taylor method on the same problem, and the
automatic choice of Sec. V."""
import numpy as np
import pytest
import scipy.sparse as sp

from gpu_common import TOL, assert_parity, context, device_inputs, log
from workloads import make_config
from workloads.circuits import Problem

pytestmark = pytest.mark.gpu


def _prob(p):
    import paper_2304_06200_amd as hg
    return hg.Problem(context(), p.H0, p.Hk, p.omega, dense=True)


def _run(p, dtype, prob=None, batch_u=None, w_int=0.0, method="diag"):
    import paper_2304_06200_amd as hg
    prob = prob or _prob(p)
    u, psi0, tg = device_inputs(p, batch_u)
    return hg.evaluate(prob, u, psi0, tg, p.dt, w_fid=p.w_fid, w_pen=p.w_pen, w_int=w_int,
                       tau=p.tau, dtype=dtype, method=method)


def _block_oracle(p, w_int=0.0, u=None):
    from oracle import grape
    return grape.cost_and_grad(p.H0, p.Hk, p.u if u is None else u, p.dt, p.psi0, p.targets,
                               omega=p.omega, w_fid=p.w_fid, w_pen=p.w_pen, w_int=w_int,
                               frechet="block")


def _herm(rng, d, scale):
    a = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) * scale / np.sqrt(2 * d)
    return sp.csr_matrix(a + a.conj().T)


def _random(seed, d, S, K, N, penalty=True):
    rng = np.random.default_rng(7000 + seed)
    H0 = _herm(rng, d, 1.0)
    Hk = [_herm(rng, d, 0.5) for _ in range(K)]
    u = rng.uniform(-1, 1, (K, N))
    q, _ = np.linalg.qr(rng.standard_normal((d, S)) + 1j * rng.standard_normal((d, S)))
    q2, _ = np.linalg.qr(rng.standard_normal((d, S)) + 1j * rng.standard_normal((d, S)))
    om = (rng.uniform(size=d) < 0.3).astype(float) if penalty else None
    return Problem(f"diag{seed}", H0, Hk, 0.3, u, q.T.copy(), q2.T.copy(), om, w_fid=1.0,
                   w_pen=0.7 if penalty else 0.0)


@pytest.mark.parametrize("seed,d,S,K,N,w_int", [(0, 40, 3, 2, 4, 0.0), (1, 65, 1, 3, 3, 0.4),
                                                 (2, 96, 96, 2, 2, 0.0)])
def test_diag_random_dense(seed, d, S, K, N, w_int):
    p = _random(seed, d, S, K, N)
    ref = _block_oracle(p, w_int=w_int)
    prob = _prob(p)
    for dtype in ("c128", "c64"):
        log(f"[case] diag random d={d} S={S} K={K} N={N} w_int={w_int} {dtype}")
        r = _run(p, dtype, prob=prob, w_int=w_int)
        assert int(r.sum_mu[0]) == 0
        assert_parity(r, ref, dtype, label=f"diag-rand{seed}")


@pytest.mark.parametrize("d_t", [3, 4])
def test_diag_gate3(d_t):
    """Three coupled transmons, full basis S = d (27: odd, padded round-robin; 64)."""
    p = make_config("gate3", d_t=d_t, N=3, random_amps=True)
    ref = _block_oracle(p)
    prob = _prob(p)
    for dtype in ("c128", "c64"):
        log(f"[case] diag gate3 d={p.dim} S={p.n_states} N=3 {dtype}")
        assert_parity(_run(p, dtype, prob=prob), ref, dtype, label=f"diag-gate3-{d_t}")


def test_diag_degenerate_spectrum():
    """No drive on the first steps (u = 0): H_0 of two uncoupled transmons has
    exactly degenerate levels, where the divided differences take their limit."""
    from workloads.circuits import destroy, embed, number
    d_t = 4
    dims = (d_t, d_t)
    n1, n2 = embed(number(d_t), 0, dims), embed(number(d_t), 1, dims)
    I = sp.identity(d_t * d_t, format="csr", dtype=complex)
    H0 = sp.csr_matrix(-0.7 * (n1 @ (n1 - I)) - 0.7 * (n2 @ (n2 - I)))
    b1 = embed(destroy(d_t), 0, dims)
    Hk = [sp.csr_matrix(b1 + b1.conj().T), sp.csr_matrix(n2)]
    rng = np.random.default_rng(3)
    u = rng.uniform(-0.5, 0.5, (2, 4))
    u[:, :2] = 0.0
    d = d_t * d_t
    psi0 = np.eye(d, dtype=complex)[[0, 1, 4, 5]]
    q, _ = np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))
    p = Problem("degenerate", H0, Hk, 0.4, u, psi0, q.T @ psi0, None, w_fid=1.0, w_pen=0.0)
    ref = _block_oracle(p)
    for dtype in ("c128", "c64"):
        log(f"[case] diag degenerate spectrum d={d} {dtype}")
        assert_parity(_run(p, dtype), ref, dtype, label="diag-degenerate")


def test_diag_batch_and_taylor_agree():
    """A batch of 3 amplitude sets: each equals its single evaluation, and the
    diagonalisation and Taylor methods agree within the Taylor tolerance."""
    p = _random(5, 48, 4, 2, 3)
    prob = _prob(p)
    rng = np.random.default_rng(9)
    ub = np.stack([p.u] + [rng.uniform(-1, 1, p.u.shape) for _ in range(2)])
    log("[case] diag batch of 3 vs single, vs Taylor, c128")
    rb = _run(p, "c128", prob=prob, batch_u=ub)
    rt = _run(p, "c128", prob=prob, batch_u=ub, method="taylor")
    for b in range(3):
        r1 = _run(p, "c128", prob=prob, batch_u=ub[b:b + 1])
        assert abs(rb.cost[b] - r1.cost[0]) <= 1e-13 * abs(r1.cost[0])
        g = rb.grad[b].cpu().numpy()
        gt = rt.grad[b].cpu().numpy()
        assert np.linalg.norm(g - r1.grad[0].cpu().numpy()) <= 1e-12 * np.linalg.norm(g)
        assert np.linalg.norm(g - gt) <= 1e-10 * np.linalg.norm(gt)


def test_auto_method_choice():
    """Sec. V: for a full-basis gate (S = d) with long steps (many Taylor
    products per step) the diagonalisation is chosen, for a single state of a
    dense problem the Taylor action (sum_mu > 0)."""
    g = make_config("gate3", d_t=4, N=2, dt=1.0, random_amps=True)
    r = _run(g, "c128", method="auto")
    assert int(r.sum_mu[0]) == 0
    assert_parity(r, _block_oracle(g), "c128", label="auto-gate")
    p = _random(6, 60, 1, 2, 3)
    r = _run(p, "c128", method="auto")
    assert int(r.sum_mu[0]) > 0

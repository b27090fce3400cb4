"""Dense operator storage (the paper's benchmark setting, Sec. IV.B): the MFMA
path against the exact oracle.

Cases: genuinely dense random Hermitian operators (more diagonals than the DIA
kernels take, so only this path runs them), ragged sizes that span several
128-row tiles and pad the state block, the full-basis three-transmon gate
(S = d) up to its benchmark size d = 512, the penalty and the time-integrated
infidelity, batches whose evaluations choose different (m, s), and agreement
with the DIA path where both run."""
import numpy as np
import pytest
import scipy.sparse as sp

from gpu_common import TOL, assert_parity, context, device_inputs, log, rel
from workloads import make_config
from workloads.circuits import Problem

pytestmark = pytest.mark.gpu


def _dense_problem(p):
    import paper_2304_06200_amd as hg
    return hg.Problem(context(), p.H0, p.Hk, p.omega, dense=True)


def _run(p, dtype, prob=None, batch_u=None, w_int=0.0, **kw):
    import paper_2304_06200_amd as hg
    prob = prob or _dense_problem(p)
    u, psi0, tg = device_inputs(p, batch_u)
    return hg.evaluate(prob, u, psi0, tg, p.dt, w_fid=p.w_fid, w_pen=p.w_pen, w_int=w_int,
                       tau=p.tau, dtype=dtype, **kw)


def _oracle(p, w_int=0.0, u=None):
    from oracle import grape
    return grape.cost_and_grad(p.H0, p.Hk, p.u if u is None else u, p.dt, p.psi0, p.targets,
                               omega=p.omega, w_fid=p.w_fid, w_pen=p.w_pen, w_int=w_int)


def _herm_dense(rng, d, scale):
    a = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) * scale / np.sqrt(2 * d)
    return sp.csr_matrix(a + a.conj().T)


def _random_dense(seed, d, S, K, N, penalty=True):
    rng = np.random.default_rng(5000 + seed)
    H0 = _herm_dense(rng, d, 1.0)
    Hk = [_herm_dense(rng, d, 0.5) for _ in range(K)]
    u = rng.uniform(-1, 1, (K, N))
    q, _ = np.linalg.qr(rng.standard_normal((d, S)) + 1j * rng.standard_normal((d, S)))
    q2, _ = np.linalg.qr(rng.standard_normal((d, S)) + 1j * rng.standard_normal((d, S)))
    om = (rng.uniform(size=d) < 0.3).astype(float) if penalty else None
    return Problem(f"dense{seed}", H0, Hk, 0.3, u, q.T.copy(), q2.T.copy(), om, w_fid=1.0,
                   w_pen=0.7 if penalty else 0.0)


@pytest.mark.parametrize("seed,d,S,K,N,w_int", [(0, 70, 5, 2, 3, 0.0), (1, 130, 9, 3, 2, 0.5),
                                                 (2, 200, 64, 1, 2, 0.0), (3, 37, 1, 4, 5, 0.3)])
def test_dense_random_operators(seed, d, S, K, N, w_int):
    from paper_2304_06200_amd import _lib as L
    import paper_2304_06200_amd as hg
    p = _random_dense(seed, d, S, K, N, penalty=seed % 2 == 0)
    log(f"[case] dense random seed={seed} d={d} S={S} K={K} N={N} w_int={w_int}")
    # more diagonals than the DIA kernels hold: only the dense path takes it
    with pytest.raises(hg._lib.HGError) as e:
        hg.Problem(context(), p.H0, p.Hk, p.omega)
    assert e.value.status == L.HG_ERR_UNSUPPORTED
    ref = _oracle(p, w_int)
    prob = _dense_problem(p)
    for dtype in ("c128", "c64"):
        r = _run(p, dtype, prob=prob, w_int=w_int)
        assert_parity(r, ref, dtype, label=f"dense-rand{seed}")
        if w_int:
            assert rel(r.integrated_infidelity[0], float(ref["integrated_infidelity"])) <= TOL[dtype]


@pytest.mark.parametrize("d_t,N,random_amps", [(3, 2, True), (4, 4, True), (8, 1, False),
                                                 (10, 1, False)])
def test_dense_gate_full_basis(d_t, N, random_amps):
    """Three-transmon Hadamard gate with S = d states; d_t = 8 is d = S = 512 (the
    bench size), d_t = 10 is d = S = 1000 (padded to 1024: 16 row tiles with a
    ragged edge, 50 scaling steps of degree 16)."""
    p = make_config("gate3", d_t=d_t, N=N, random_amps=random_amps)
    log(f"[case] dense gate3 d_t={d_t} d={p.dim} S={p.n_states} N={N}")
    ref = _oracle(p)
    prob = _dense_problem(p)
    for dtype in ("c128", "c64"):
        r = _run(p, dtype, prob=prob)
        assert_parity(r, ref, dtype, label=f"dense-gate3-t{d_t}")


def test_dense_matches_dia_path():
    """cfg2 (transmon x cavity, penalty, d = 60): dense and DIA storage agree with
    each other and with the oracle, with C3 on."""
    import paper_2304_06200_amd as hg
    p = make_config("cfg2", N=12)
    ref = _oracle(p, w_int=0.4)
    u, psi0, tg = device_inputs(p)
    dia = hg.Problem(context(), p.H0, p.Hk, p.omega)
    den = _dense_problem(p)
    for dtype in ("c128", "c64"):
        a = hg.evaluate(dia, u, psi0, tg, p.dt, w_fid=p.w_fid, w_pen=p.w_pen, w_int=0.4,
                        tau=p.tau, dtype=dtype)
        b = _run(p, dtype, prob=den, w_int=0.4)
        assert_parity(b, ref, dtype, label="dense-cfg2")
        ga, gb = a.grad[0].cpu().numpy(), b.grad[0].cpu().numpy()
        e = np.linalg.norm(ga - gb) / np.linalg.norm(ga)
        log(f"  dense vs DIA {dtype}: cost rel {rel(b.cost[0], a.cost[0]):.2e} grad rel {e:.2e}")
        assert rel(b.cost[0], a.cost[0]) <= TOL[dtype] and e <= TOL[dtype]
        assert a.sum_mu[0] == b.sum_mu[0]


def test_dense_batch_is_bitwise_per_evaluation():
    """Evaluations with different amplitudes (so different (m, s) per step) in one
    batch give exactly the numbers of the same evaluations run alone."""
    p = _random_dense(7, 90, 6, 2, 3)
    rng = np.random.default_rng(77)
    U = np.stack([p.u, 2.5 * rng.uniform(-1, 1, p.u.shape), 0.2 * rng.uniform(-1, 1, p.u.shape)])
    prob = _dense_problem(p)
    for dtype in ("c128", "c64"):
        rb = _run(p, dtype, prob=prob, batch_u=U)
        assert len(set(rb.sum_mu.tolist())) > 1, "batch should mix schedules"
        for b in range(U.shape[0]):
            r1 = _run(p, dtype, prob=prob, batch_u=U[b:b + 1])
            assert rb.cost[b] == r1.cost[0]
            assert np.array_equal(rb.grad[b].cpu().numpy(), r1.grad[0].cpu().numpy())
        ref = _oracle(p, u=U[1])
        assert_parity(rb, ref, dtype, b=1, label="dense-batch")


@pytest.mark.parametrize("C", [1, 3, 7, 50])
def test_dense_checkpoint_mode(C):
    """Checkpointed-state variant on dense storage: psi stored every C steps,
    each segment re-propagated forward from its checkpoint, only Lambda
    propagated backwards.  Against the exact oracle (penalty and C3 on,
    segments that do not divide N), and against the reconstruction mode of the
    same library; the drift of a never-rebuilt psi_0 is its rounding only.  A
    batch whose evaluations take different (m, s) checks the per-evaluation
    schedule in the re-propagation."""
    p = _random_dense(9, 70, 3, 2, 11)
    U = np.stack([p.u, 1.7 * p.u])
    ref = _oracle(p, w_int=0.4)
    for dtype in ("c128", "c64"):
        log(f"[case] dense checkpoint C={C} {dtype}")
        a = _run(p, dtype, batch_u=U, w_int=0.4, mode="checkpoint", ckpt_every=C)
        assert_parity(a, ref, dtype, label=f"dense-ckpt{C}")
        assert_parity(a, _oracle(p, w_int=0.4, u=U[1]), dtype, b=1, label=f"dense-ckpt{C}-b1")
        r = _run(p, dtype, batch_u=U, w_int=0.4)
        assert int(a.sum_mu[0]) == int(r.sum_mu[0]) and int(a.sum_mu[1]) == int(r.sum_mu[1])
        assert a.drift[0] <= (1e-15 if dtype == "c128" else 1e-6)


def test_dense_checkpoint_rejected_with_diagonalisation():
    import paper_2304_06200_amd as hg
    from paper_2304_06200_amd import _lib as L
    p = _random_dense(9, 20, 2, 1, 4)
    with pytest.raises(hg._lib.HGError) as e:
        _run(p, "c128", mode="checkpoint", ckpt_every=2, method="diag")
    assert e.value.status == L.HG_ERR_UNSUPPORTED


def test_dense_no_controls():
    """K = 0 (drift only): cost, overlap and penalty against the oracle; no gradient."""
    from oracle import grape
    p = _random_dense(11, 45, 3, 0, 4)
    ref = grape.cost_and_grad(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets, omega=p.omega,
                              w_fid=p.w_fid, w_pen=p.w_pen)
    for dtype in ("c128", "c64"):
        r = _run(p, dtype)
        log(f"[case] dense K=0 {dtype}: cost {r.cost[0]:.15g} ref {float(ref['cost']):.15g}")
        assert r.grad is None
        assert rel(r.cost[0], float(ref["cost"])) <= TOL[dtype]
        assert abs(r.overlap[0] - ref["overlap"]) <= TOL[dtype]

"""Row-indexed (ELL) storage: operator patterns that are not a few diagonals
run the same sweep kernels with per-row gather columns.  The driven qubit
chain of App. E (H_3: sigma_z sigma_z couplings, sigma_x and sigma_y drives
on every qubit; sigma_x alone at 10 qubits, the library taking 16 controls) flips one bit per control, i.e. offsets +-2^j: 2 n_q + 1
diagonals but only n_q + 1 entries per row.  Cases: qubit chains of 7, 8
and 10 qubits (15, 17 and 21 diagonals), both precisions and both backward
variants, against the exact oracle; a random sparse Hermitian pattern with
complex controls; a batch and spread backward sweeps; the width limit."""
import numpy as np
import pytest
import scipy.sparse as sp

from gpu_common import assert_parity, context, log, make_problem, run
from workloads.circuits import Problem, haar_unitary, qubit_chain

pytestmark = pytest.mark.gpu

TP = 2 * np.pi


def _oracle(p, u=None):
    from oracle import grape
    return grape.cost_and_grad(p.H0, p.Hk, p.u if u is None else u, p.dt, p.psi0, p.targets,
                               omega=p.omega, w_fid=p.w_fid, w_pen=p.w_pen)


def _qubits(n_q, N, S=4, seed=0, drives="xy"):
    rng = np.random.default_rng(700 + n_q + seed)
    H0, Hk, _ = qubit_chain(n_q, TP * 0.1)
    if drives == "x":  # sigma_x drives only (at most 16 controls)
        Hk = Hk[0::2]
    d = 2 ** n_q
    u = TP * rng.uniform(-0.5, 0.5, (len(Hk), N))
    idx = rng.choice(d, size=S, replace=False)
    psi0 = np.zeros((S, d), complex)
    psi0[np.arange(S), idx] = 1.0
    om = (rng.uniform(size=d) < 0.2).astype(float)
    return Problem(f"qubits{n_q}", H0, Hk, 0.1, u, psi0, haar_unitary(S, rng).T @ psi0, om,
                   w_fid=1.0, w_pen=0.3)


@pytest.mark.parametrize("n_q,N,drives", [(7, 8, "xy"), (8, 8, "xy"), (10, 3, "x")])
def test_qubit_chain(n_q, N, drives):
    p = _qubits(n_q, N, drives=drives)
    prob = make_problem(p)
    assert prob.info["ell_width"] == n_q + 1
    ref = _oracle(p)
    for dtype in ("c128", "c64"):
        log(f"[case] qubit chain n_q={n_q} d={p.dim} N={N} {dtype}")
        assert_parity(run(p, dtype, prob=prob), ref, dtype, label=f"q{n_q}")
        assert_parity(run(p, dtype, prob=prob, mode="checkpoint", ckpt_every=3), ref, dtype,
                      label=f"q{n_q}-ckpt")


def _matching(rng, d, scale):
    """Hermitian coupling along a random perfect matching of the rows (one
    entry per row, at a random column), complex random phases."""
    perm = rng.permutation(d)
    c = sp.lil_matrix((d, d), dtype=complex)
    for a, b in zip(perm[0::2], perm[1::2]):
        v = np.exp(1j * rng.uniform(0, TP)) * scale * rng.uniform(0.5, 1.5)
        c[a, b] = v
        c[b, a] = np.conj(v)
    return sp.csr_matrix(c)


def _random_sparse(d=300, N=6, S=3, seed=4):
    """Random Hermitian pattern: a real diagonal plus three random matchings
    (three couplings per row at random columns, hundreds of distinct
    diagonals), and two complex controls, each one more random matching."""
    rng = np.random.default_rng(seed)
    H0 = sp.csr_matrix(sp.diags(rng.uniform(-1, 1, d)).astype(complex))
    for _ in range(3):
        H0 = H0 + _matching(rng, d, 0.3)
    Hk = [_matching(rng, d, 0.4) for _ in range(2)]
    u = rng.uniform(-1, 1, (2, N))
    q, _ = np.linalg.qr(rng.standard_normal((d, S)) + 1j * rng.standard_normal((d, S)))
    q2, _ = np.linalg.qr(rng.standard_normal((d, S)) + 1j * rng.standard_normal((d, S)))
    om = (rng.uniform(size=d) < 0.3).astype(float)
    return Problem("sparse", sp.csr_matrix(H0), Hk, 0.2, u, q.T.copy(), q2.T.copy(), om,
                   w_fid=1.0, w_pen=0.5)


def test_random_sparse_pattern():
    p = _random_sparse()
    prob = make_problem(p)
    assert prob.info["ell_width"] <= 6
    ref = _oracle(p)
    for dtype in ("c128", "c64"):
        log(f"[case] random sparse pattern d={p.dim} width {prob.info['ell_width']} {dtype}")
        assert_parity(run(p, dtype, prob=prob), ref, dtype, label="sparse")
        assert_parity(run(p, dtype, prob=prob, mode="checkpoint", ckpt_every=4), ref, dtype,
                      label="sparse-ckpt")


def test_complex_main_diagonal_and_integrated_cost():
    """Row-indexed storage with a main diagonal that is complex somewhere (an
    imaginary part inside the Hermiticity tolerance: slot 0 stays an all-zero
    stand-in, the diagonal takes a slot of its own) and the time-integrated
    infidelity on, against the Taylor-discretised oracle."""
    from gpu_common import oracle_schedule
    from oracle import taylor
    p = _random_sparse(d=200, N=5, S=2, seed=8)
    H0 = p.H0.tolil()
    for i in range(0, p.dim, 7):
        H0[i, i] = H0[i, i] + 1e-14j
    p = Problem("sparse-cdiag", sp.csr_matrix(H0), p.Hk, p.dt, p.u, p.psi0, p.targets, p.omega,
                w_fid=p.w_fid, w_pen=p.w_pen)
    prob = make_problem(p)
    sched = oracle_schedule(p)
    ref = taylor.hg_discrete(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets, sched, omega=p.omega,
                             w_fid=p.w_fid, w_pen=p.w_pen, w_int=0.7)
    for dtype in ("c128", "c64"):
        log(f"[case] row-indexed, complex main diagonal, C3 on, {dtype}")
        assert_parity(run(p, dtype, prob=prob, w_int=0.7), ref, dtype, label="sparse-cdiag")


def test_batch_and_spread():
    import paper_2304_06200_amd as hg
    p = _qubits(8, 6, S=2)
    prob = make_problem(p)
    U = np.stack([p.u, 0.6 * p.u, -p.u])
    for dtype in ("c128", "c64"):
        rb = run(p, dtype, prob=prob, batch_u=U)
        r1 = run(p, dtype, prob=prob)
        assert rb.cost[0] == r1.cost[0]
        assert np.array_equal(rb.grad[0].cpu().numpy(), r1.grad[0].cpu().numpy())
        assert_parity(rb, _oracle(p, u=U[2]), dtype, b=2, label="q8-batch")
        rs = run(p, dtype, prob=prob, spread=True)
        assert_parity(rs, _oracle(p), dtype, label="q8-spread")


def test_row_width_limit():
    import paper_2304_06200_amd as hg
    d = 64
    rng = np.random.default_rng(1)
    a = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    H0 = sp.csr_matrix(a + a.conj().T)
    with pytest.raises(hg._lib.HGError) as e:
        hg.Problem(context(), H0, [], None)
    assert e.value.status == hg._lib.HG_ERR_UNSUPPORTED

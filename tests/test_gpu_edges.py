"""GPU edge cases: degenerate sizes, batching, determinism and error paths."""
import numpy as np
import pytest
import scipy.sparse as sp

from gpu_common import TOL, assert_parity, context, log, make_problem, run
from workloads import make_config
from workloads.circuits import Problem, destroy, haar_unitary

pytestmark = pytest.mark.gpu


def _oracle(p):
    from oracle import grape
    return grape.cost_and_grad(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets, omega=p.omega,
                               w_fid=p.w_fid, w_pen=p.w_pen)


def _cavity_problem(d, K=2, N=20, S=2, seed=0, penalty=True, dt=0.3):
    """Driven anharmonic oscillator with d levels (tridiagonal union pattern)."""
    rng = np.random.default_rng(seed)
    a = destroy(d) / np.sqrt(max(d, 1))       # bounded drive norm at any d
    n = sp.diags(np.arange(d, dtype=float) / max(d, 1)).astype(complex)
    H0 = sp.csr_matrix(sp.diags(rng.uniform(-2.0, 2.0, d)).astype(complex))
    Hk = [sp.csr_matrix(a + a.conj().T), sp.csr_matrix(1j * (a.conj().T - a)),
          sp.csr_matrix(n)][:K]
    for h in Hk:
        h.eliminate_zeros()
    u = rng.uniform(-0.5, 0.5, (K, N))
    psi0 = np.zeros((S, d), complex)
    for h in range(S):
        psi0[h, h % d] = 1.0
    UT = haar_unitary(S, rng)
    om = (np.arange(d) == d - 1).astype(float) if penalty else None
    return Problem(f"osc{d}", sp.csr_matrix(H0), Hk, dt, u, psi0, UT.T @ psi0, om,
                   w_fid=1.0, w_pen=0.5 if penalty else 0.0)


@pytest.mark.parametrize("d", [1, 2, 63, 65, 513, 1031])
def test_ragged_dimensions(d):
    p = _cavity_problem(d, S=1 if d == 1 else 2, N=12)
    log(f"[case] ragged d={d}")
    for dt in ("c128", "c64"):
        assert_parity(run(p, dt), _oracle(p), dt, label=f"osc{d}")


@pytest.mark.parametrize("d", [1600, 2600, 2850, 4000])
def test_large_ragged_dimensions(d):
    """Launch shapes above 512 rows: 1024-thread complex64 kernels (1600, with a
    last plane of 9 row slabs), 512 threads with 6 or 8 rows per thread (2600:
    a single slab in the last plane, 2850: five, 4000: seven).  Compared with
    the Taylor-discretised oracle on the oracle planner's schedule.  complex128
    holds its (psi, Lambda) block in one workgroup's LDS only up to 2048 rows;
    above, its columns run split over several workgroups (contiguous row ranges
    here, the oscillator having a single band)."""
    import paper_2304_06200_amd as hg
    from gpu_common import oracle_schedule
    from oracle import taylor
    p = _cavity_problem(d, S=2, N=12)
    sched = oracle_schedule(p)
    ref = taylor.hg_discrete(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets, sched, omega=p.omega,
                             w_fid=p.w_fid, w_pen=p.w_pen)
    log(f"[case] large ragged d={d}, sum_mu {int(np.sum(sched[0] * sched[1]))}")
    for dt in ("c128", "c64"):
        assert_parity(run(p, dt), ref, dt, label=f"osc{d}")


def test_wide_pattern_above_2048_rows():
    """Nine-diagonal cfg3 structure with a 177-level cavity (d = 2832): 512
    threads with 6 rows each and a last plane of 5 row slabs (the fifth shared
    by vector); three steps against the discretised oracle, complex64."""
    from gpu_common import oracle_schedule
    from oracle import taylor
    p = make_config("cfg3", N=3, d_c=177)
    sched = oracle_schedule(p)
    ref = taylor.hg_discrete(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets, sched, omega=p.omega,
                             w_fid=p.w_fid, w_pen=p.w_pen)
    log(f"[case] cfg3 structure d={p.dim}, sum_mu {int(np.sum(sched[0] * sched[1]))}")
    assert_parity(run(p, "c64"), ref, "c64", label=f"cfg3c177")


def _banded(d, diag, off_re, off_im, ctrl_imag, N=10, S=2, seed=3):
    """A band of offsets 0 and +-1: main diagonal `diag`, off-diagonal with
    real part off_re and imaginary part off_im; controls a + a^dag and, with
    ctrl_imag, i(a^dag - a)."""
    rng = np.random.default_rng(seed)
    a = destroy(d) / np.sqrt(d)
    sup = sp.diags((off_re + 1j * off_im) * rng.uniform(0.5, 1.5, d - 1), 1)
    H0 = sp.csr_matrix(sp.diags(diag) + sup + sup.conj().T)
    H0.eliminate_zeros()
    Hk = [sp.csr_matrix(a + a.conj().T)]
    if ctrl_imag:
        Hk.append(sp.csr_matrix(1j * (a.conj().T - a)))
    u = rng.uniform(-0.5, 0.5, (len(Hk), N))
    psi0 = np.zeros((S, d), complex)
    for h in range(S):
        psi0[h, h] = 1.0
    return Problem(f"band{d}", H0, Hk, 0.4, u, psi0, haar_unitary(S, rng).T @ psi0, None,
                   w_fid=1.0, w_pen=0.0)


@pytest.mark.parametrize("case", ["real", "no_main_diagonal", "complex_main_diagonal"])
def test_union_order_and_imaginary_diagonals(case):
    """The union puts the main diagonal first and the other diagonals on which
    every operator is real next; their entries of B are purely imaginary and
    take half the multiply-adds.  Cases: everything real (all three leading
    diagonals purely imaginary in B), no main diagonal at all (an all-zero
    slot stands in for it), and a main diagonal with an imaginary part inside
    the Hermiticity tolerance (a slot of its own, after the others).  Against
    the discretised oracle, both precisions."""
    from gpu_common import oracle_schedule
    from oracle import taylor
    d = 70
    rng = np.random.default_rng(11)
    diag = rng.uniform(-2.0, 2.0, d)
    if case == "real":
        p = _banded(d, diag, 1.0, 0.0, ctrl_imag=False)
        width = 3
    elif case == "no_main_diagonal":
        p = _banded(d, np.zeros(d), 0.6, 0.8, ctrl_imag=True)
        width = 3
    else:
        p = _banded(d, diag + 1e-14j * np.max(np.abs(diag)), 0.6, 0.8, ctrl_imag=True)
        width = 4
    prob = make_problem(p)
    assert prob.info["ell_width"] == width
    sched = oracle_schedule(p)
    ref = taylor.hg_discrete(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets, sched, omega=p.omega,
                             w_fid=p.w_fid, w_pen=p.w_pen)
    log(f"[case] union order {case}")
    for dt in ("c128", "c64"):
        assert_parity(run(p, dt, prob=prob), ref, dt, label=case)


@pytest.mark.parametrize("mode,w_int", [("reconstruct", 0.0), ("checkpoint", 0.6)])
def test_two_columns_per_forward_workgroup(mode, w_int):
    """A batch large enough that the complex64 forward runs two state columns
    per workgroup (32 evaluations x 16 states at d = 640): every evaluation
    bitwise equal to the same evaluation alone (one column per workgroup),
    and one against the oracle."""
    from workloads.configs import _amps
    p = make_config("cfg3", N=4, d_c=40)
    prob = make_problem(p)
    U = np.stack([p.u] + [_amps(np.random.default_rng(300 + i), p.n_ctrl, p.n_steps)
                          for i in range(31)])
    kw = dict(mode=mode, ckpt_every=2 if mode == "checkpoint" else 0, w_int=w_int)
    log(f"[case] two columns per forward workgroup, {mode}, w_int={w_int}")
    rb = run(p, "c64", prob=prob, batch_u=U, **kw)
    for i in (0, 17, 31):
        r1 = run(p, "c64", prob=prob, batch_u=U[i:i + 1], **kw)
        assert rb.cost[i] == r1.cost[0], i
        assert np.array_equal(rb.grad[i].cpu().numpy(), r1.grad[0].cpu().numpy()), i
    from oracle import grape
    ref = grape.cost_and_grad(p.H0, p.Hk, U[17], p.dt, p.psi0, p.targets, omega=p.omega,
                              w_fid=p.w_fid, w_pen=p.w_pen, w_int=w_int)
    assert_parity(rb, ref, "c64", b=17, label="cpw2")


def test_single_step_single_state_no_penalty():
    p = _cavity_problem(10, K=1, N=1, S=1, penalty=False)
    log("[case] N=1 S=1 K=1 no penalty")
    assert_parity(run(p, "c128"), _oracle(p), "c128", label="N1")


def test_no_controls():
    """K = 0: cost only (the drift alone); the library returns no gradient."""
    p = _cavity_problem(12, K=1, N=5, S=2)
    p0 = Problem("drift-only", p.H0, [], p.dt, np.zeros((0, 5)), p.psi0, p.targets, p.omega,
                 w_fid=1.0, w_pen=0.5)
    log("[case] K=0")
    r = run(p0, "c128")
    from oracle import grape
    ref = grape.cost_and_grad(p0.H0, [], np.zeros((0, 5)), p0.dt, p0.psi0, p0.targets,
                              omega=p0.omega, w_fid=1.0, w_pen=0.5)
    assert abs(r.cost[0] - ref["cost"]) <= 1e-10 * abs(ref["cost"])
    assert r.grad is None


def test_number_operator_control_one_diagonal():
    p = _cavity_problem(30, K=3, N=15, S=3)
    log("[case] K=3 with a diagonal control")
    for dt in ("c128", "c64"):
        assert_parity(run(p, dt), _oracle(p), dt, label="ndiag")


def test_batch_equals_single_bitwise():
    p = make_config("cfg2", N=50, d_c=12)
    prob = make_problem(p)
    rng = np.random.default_rng(5)
    us = np.stack([p.u, p.u + 0.01 * rng.standard_normal(p.u.shape), -p.u])
    log("[case] batch of 3 vs singles")
    for dt in ("c128", "c64"):
        rb = run(p, dt, prob=prob, batch_u=us)
        for b in range(3):
            r1 = run(p, dt, prob=prob, batch_u=us[b])
            assert r1.cost[0] == rb.cost[b]
            assert np.array_equal(r1.grad[0].cpu().numpy(), rb.grad[b].cpu().numpy())


def test_repeatable_bitwise():
    p = make_config("cfg3", N=4, d_c=30)
    prob = make_problem(p)
    log("[case] repeatability")
    a = run(p, "c64", prob=prob)
    b = run(p, "c64", prob=prob)
    assert a.cost[0] == b.cost[0]
    assert np.array_equal(a.grad.cpu().numpy(), b.grad.cpu().numpy())


def test_drift_reported_and_small():
    p = make_config("cfg2", N=200)
    r128 = run(p, "c128")
    r64 = run(p, "c64")
    log(f"[case] drift c128 {r128.drift[0]:.2e} c64 {r64.drift[0]:.2e}")
    assert r128.drift[0] < 1e-11
    assert r64.drift[0] < 1e-3


def test_error_paths():
    import torch
    import paper_2304_06200_amd as hg
    from paper_2304_06200_amd import _lib as L
    p = make_config("cfg2", N=10, d_c=6)
    prob = make_problem(p)
    u, psi0, tg = (torch.tensor(p.u, device="cuda"),
                   torch.tensor(p.psi0, dtype=torch.complex128, device="cuda"),
                   torch.tensor(p.targets, dtype=torch.complex128, device="cuda"))
    log("[case] error paths")
    with pytest.raises(L.HGError) as e:
        hg.evaluate(prob, u, 2 * psi0, tg, p.dt)
    assert e.value.status == L.HG_ERR_INVALID_ARG
    bad = u.clone()
    bad[1, 3] = float("nan")
    with pytest.raises(L.HGError) as e:
        hg.evaluate(prob, bad, psi0, tg, p.dt)
    assert e.value.status == L.HG_ERR_NONFINITE
    with pytest.raises(L.HGError) as e:
        hg.evaluate(prob, u, psi0, tg, p.dt, tau=1e-16)
    assert e.value.status == L.HG_ERR_TOLERANCE_UNREACHABLE
    with pytest.raises(L.HGError) as e:
        hg.evaluate(prob, u, psi0, tg, -1.0)
    assert e.value.status == L.HG_ERR_INVALID_ARG
    nh = sp.csr_matrix(np.triu(np.ones((6, 6))) * (1 + 1j))
    with pytest.raises(L.HGError) as e:
        hg.Problem(context(), nh, [], None)
    assert e.value.status == L.HG_ERR_NOT_HERMITIAN
    # a union pattern with too many diagonals is rejected cleanly
    dense = sp.csr_matrix(np.ones((40, 40), complex))
    with pytest.raises(L.HGError) as e:
        hg.Problem(context(), dense, [], None)
    assert e.value.status == L.HG_ERR_UNSUPPORTED
    # 15 diagonals: within the DIA storage but wider than the kernels, rejected at creation
    band = sp.diags([np.ones(40 - abs(o)) for o in range(-7, 8)], list(range(-7, 8)),
                    dtype=complex).tocsr()
    with pytest.raises(L.HGError) as e:
        hg.Problem(context(), band, [], None)
    assert e.value.status == L.HG_ERR_UNSUPPORTED and "13" in str(e.value)
    # the evaluation still works after the errors
    r = hg.evaluate(prob, u, psi0, tg, p.dt)
    assert np.isfinite(r.cost[0])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_spread_backward(dtype):
    """HG_FLAG_SPREAD (several workgroups per column in the backward sweep,
    each repeating phase 1 and taking a share of the controls): parity with
    the oracle, agreement with the plain launch to rounding, and bitwise
    repeatability; cfg3 structure (6 controls) with a 20-level cavity, one
    evaluation, and a batch of 3."""
    import paper_2304_06200_amd as hg
    p = make_config("cfg3", N=30, d_c=20)
    prob = make_problem(p)
    ref = _oracle(p)
    log(f"[case] spread backward cfg3c20 {dtype}")
    a = run(p, dtype, prob=prob, spread=True)
    b = run(p, dtype, prob=prob)
    c = run(p, dtype, prob=prob, spread=True)
    assert_parity(a, ref, dtype, label="spread")
    ga, gb = a.grad[0].cpu().numpy(), b.grad[0].cpu().numpy()
    assert np.linalg.norm(ga - gb) <= (1e-13 if dtype == "c128" else 1e-6) * np.linalg.norm(gb)
    assert a.cost[0] == c.cost[0] and np.array_equal(ga, c.grad[0].cpu().numpy())
    from workloads.configs import _amps
    u3 = np.stack([p.u] + [_amps(np.random.default_rng(300 + i), p.n_ctrl, p.n_steps)
                           for i in range(2)])
    r3 = run(p, dtype, prob=prob, batch_u=u3, spread=True)
    assert r3.cost[0] == a.cost[0] or abs(r3.cost[0] - a.cost[0]) <= 1e-12 * abs(a.cost[0])

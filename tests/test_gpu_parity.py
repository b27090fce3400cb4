"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Expected values come only from oracle/ (live, or from tests/golden files
written by tests/golden/make_golden.py).  Bars: relative error <= 1e-10 on
cost and gradient in complex128, <= 1e-4 in complex64 (element-wise on the
gradient relative to its largest entry as well).
"""
import numpy as np
import pytest

from gpu_common import (assert_parity, golden, log, make_problem, oracle_schedule, rel, run,
                        TOL)
from workloads import make_config

pytestmark = pytest.mark.gpu


def _oracle(p):
    from oracle import grape
    return grape.cost_and_grad(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets, omega=p.omega,
                               w_fid=p.w_fid, w_pen=p.w_pen)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_cfg1_full(dtype):
    p = make_config("cfg1")
    log(f"[case] cfg1 d=4 N=200 S=1 {dtype}")
    assert_parity(run(p, dtype), golden("cfg1"), dtype, label="cfg1")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_cfg2_full(dtype):
    p = make_config("cfg2")
    log(f"[case] cfg2 d=60 N=1000 S=4 {dtype}")
    assert_parity(run(p, dtype), golden("cfg2"), dtype, label="cfg2")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_cfg3_prefix_full_dimension(dtype):
    """d = 1600, all 16 states, first 3 steps (oracle at full dimension)."""
    p = make_config("cfg3", N=3)
    log(f"[case] cfg3 prefix d=1600 N=3 S=16 {dtype}")
    assert_parity(run(p, dtype), _oracle(p), dtype, label="cfg3[:3]")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_cfg3_reduced_cavity(dtype):
    """cfg3 structure with a 20-level cavity (d = 320), N = 60: several tiles
    of rows per thread and a ragged last wavefront."""
    p = make_config("cfg3", N=60, d_c=20)
    log(f"[case] cfg3 d_c=20 d=320 N=60 S=16 {dtype}")
    assert_parity(run(p, dtype), _oracle(p), dtype, label="cfg3c20")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_cfg3_full_size(dtype):
    ref = golden("cfg3")
    if ref is None:
        pytest.skip("tests/golden/cfg3_oracle.npz not generated")
    p = make_config("cfg3")
    log(f"[case] cfg3 full d=1600 N=2000 S=16 {dtype}")
    assert_parity(run(p, dtype), ref, dtype, label="cfg3")


def test_discrete_oracle_tight():
    """With the oracle's own schedule frozen on both sides, the c128 GPU path
    and the discretised-method oracle agree to rounding (much tighter than tau)."""
    from oracle import taylor
    p = make_config("cfg2", N=40, d_c=10)
    sched = oracle_schedule(p)
    ref = taylor.hg_discrete(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets, sched, omega=p.omega,
                             w_fid=p.w_fid, w_pen=p.w_pen)
    log("[case] discrete oracle cfg2 d_c=10 N=40 frozen schedule")
    r = run(p, "c128", schedule=sched)
    g = r.grad[0].cpu().numpy()
    assert rel(r.cost[0], ref["cost"]) < 1e-13
    assert np.linalg.norm(g - ref["grad"]) / np.linalg.norm(ref["grad"]) < 1e-12
    assert int(r.sum_mu[0]) == int(np.sum(sched[0] * sched[1]))


def test_schedule_matches_oracle_planner():
    """The library's norms + planner choose the oracle's (m, s) on every step
    (compare sum of mu and the per-step norms)."""
    import torch
    import paper_2304_06200_amd as hg
    p = make_config("cfg2", N=200)
    prob = make_problem(p)
    th = hg.step_norms(prob, torch.tensor(p.u, device="cuda"), p.dt)[0].cpu().numpy()
    sched = oracle_schedule(p)
    from oracle import planner
    th_ref = np.array([float(np.max(np.asarray(abs(-1j * p.dt * (p.H0 + sum(
        p.u[k, n] * p.Hk[k] for k in range(p.n_ctrl)))).sum(axis=0)))) for n in range(p.n_steps)])
    np.testing.assert_allclose(th, th_ref, rtol=1e-14)
    m, s = hg.plan(th, prob.info["sigma"], p.tau)
    assert np.array_equal(m, sched[0]) and np.array_equal(s, sched[1])


def test_finite_differences_of_gpu_cost():
    """Central differences of the GPU c128 cost (schedule frozen) match its gradient."""
    p = make_config("cfg2", N=30, d_c=8)
    sched = oracle_schedule(p)
    prob = make_problem(p)
    r = run(p, "c128", prob=prob, schedule=sched)
    g = r.grad[0].cpu().numpy()
    rng = np.random.default_rng(33)
    h = 1e-6
    for _ in range(8):
        k, n = int(rng.integers(p.n_ctrl)), int(rng.integers(p.n_steps))
        up = p.u.copy(); up[k, n] += h
        um = p.u.copy(); um[k, n] -= h
        cp = run(p, "c128", prob=prob, schedule=sched, batch_u=up).cost[0]
        cm = run(p, "c128", prob=prob, schedule=sched, batch_u=um).cost[0]
        fd = (cp - cm) / (2 * h)
        assert abs(fd - g[k, n]) <= 1e-7 * max(1.0, np.max(np.abs(g))), (k, n, fd, g[k, n])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_cfg3_fidelity_dominated_full_dimension(dtype):
    """d = 1600, 16 states, N = 24, no penalty, and targets that the amplitudes
    nearly reach (|g| ~ 0.97): the gradient is then carried by the fidelity
    co-state at full strength, unlike the Haar-target run where |g| ~ 0.01.
    The targets are the oracle's Taylor-discretised evolution under a second
    seeded amplitude set within 2 pi * 0.01 GHz of u; the reference is the
    discretised oracle on the oracle planner's schedule, frozen on both sides."""
    import dataclasses
    from oracle import taylor
    p = make_config("cfg3", N=24)
    sched = oracle_schedule(p)
    u2 = p.u + 2 * np.pi * 0.01 * np.random.default_rng(303).uniform(-1, 1, p.u.shape)
    psi = p.psi0.T.copy()
    for n in range(p.n_steps):
        H = p.H0 + sum(u2[k, n] * p.Hk[k] for k in range(p.n_ctrl))
        psi = taylor.taylor_action(-1j * p.dt * H, psi, int(sched[0, n]), int(sched[1, n]))
    q = dataclasses.replace(p, targets=psi.T.copy(), omega=None, w_pen=0.0)
    ref = taylor.hg_discrete(q.H0, q.Hk, q.u, q.dt, q.psi0, q.targets, sched, omega=None,
                             w_fid=1.0, w_pen=0.0)
    log(f"[case] cfg3 fidelity-dominated d=1600 N=24 S=16 {dtype} |g|={abs(ref['overlap']):.4f}")
    assert abs(ref["overlap"]) > 0.9
    assert_parity(run(q, dtype, schedule=sched), ref, dtype, label="cfg3-fid")

"""Time-integrated infidelity C3 = 1 - (1/N) sum_n |g_n|^2 (App. A) on the GPU:
cost parts and gradient against the oracle, alone and combined with C1 and C2,
in both backward variants and batched."""
import numpy as np
import pytest

from gpu_common import TOL, assert_parity, log, make_problem, oracle_schedule, run
from workloads import make_config

pytestmark = pytest.mark.gpu


def _oracle(p, w_fid, w_int):
    from oracle import grape
    return grape.cost_and_grad(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets, omega=p.omega,
                               w_fid=w_fid, w_pen=p.w_pen, w_int=w_int)


def _check_c3(res, ref, dtype, b=0):
    e = abs(res.integrated_infidelity[b] - ref["integrated_infidelity"])
    log(f"  C3 {res.integrated_infidelity[b]:.15g} ref {ref['integrated_infidelity']:.15g} abs {e:.2e}")
    assert e <= TOL[dtype] * max(1.0, abs(ref["integrated_infidelity"]))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("w_fid,w_int", [(0.0, 1.0), (1.0, 0.5)])
def test_integrated_cfg1(dtype, w_fid, w_int):
    p = make_config("cfg1")
    log(f"[case] C3 cfg1 {dtype} w_fid={w_fid} w_int={w_int}")
    ref = _oracle(p, w_fid, w_int)
    r = run(p, dtype, w_fid=w_fid, w_int=w_int)
    assert_parity(r, ref, dtype, label="cfg1-C3")
    _check_c3(r, ref, dtype)


@pytest.mark.parametrize("mode", ["reconstruct", "checkpoint"])
def test_integrated_cfg2_reduced(mode):
    """Transmon x cavity(8), 40 steps, 4 states, penalty on: C1 + C2 + C3."""
    p = make_config("cfg2", d_c=8, N=40)
    ref = _oracle(p, 1.0, 0.8)
    kw = dict(mode=mode, ckpt_every=7) if mode == "checkpoint" else {}
    log(f"[case] C3 cfg2 d_c=8 N=40 {mode}")
    for dtype in ("c128", "c64"):
        r = run(p, dtype, w_fid=1.0, w_int=0.8, **kw)
        assert_parity(r, ref, dtype, label=f"cfg2r-C3-{mode}")
        _check_c3(r, ref, dtype)


def test_integrated_cfg3_structure_discrete():
    """The benchmark's structure (d = 1600 rows, 16 states, wide launch) for a few
    steps, against the discretised oracle on the oracle planner's schedule."""
    from oracle import taylor
    p = make_config("cfg3", N=4)
    sched = oracle_schedule(p)
    ref = taylor.hg_discrete(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets, sched, omega=p.omega,
                             w_fid=p.w_fid, w_pen=p.w_pen, w_int=0.7)
    log("[case] C3 cfg3 N=4 vs discretised oracle")
    for dtype in ("c128", "c64"):
        r = run(p, dtype, w_int=0.7)
        assert_parity(r, ref, dtype, label="cfg3-C3")
        _check_c3(r, ref, dtype)


def test_integrated_off_is_unchanged_and_batch_bitwise():
    """w_int = 0 reproduces the plain cost bitwise; with w_int a batch entry equals
    the same amplitudes evaluated alone."""
    p = make_config("cfg2", d_c=6, N=30)
    prob = make_problem(p)
    a = run(p, "c64", prob=prob)
    b = run(p, "c64", prob=prob, w_int=0.0)
    assert a.cost[0] == b.cost[0] and b.integrated_infidelity[0] == 0.0
    rng = np.random.default_rng(3)
    us = np.stack([p.u, p.u + 0.01 * rng.standard_normal(p.u.shape)])
    batch = run(p, "c64", prob=prob, batch_u=us, w_int=0.6)
    alone = run(p, "c64", prob=prob, w_int=0.6)
    log(f"[case] C3 batch: {batch.cost} alone {alone.cost}")
    assert batch.cost[0] == alone.cost[0]
    assert batch.integrated_infidelity[0] == alone.integrated_infidelity[0]
    assert np.array_equal(batch.grad[0].cpu().numpy(), alone.grad[0].cpu().numpy())

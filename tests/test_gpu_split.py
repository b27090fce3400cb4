"""Columns too long for one workgroup: split over several co-resident
workgroups by row blocks (cavity-index ranges for a transmon x cavity basis),
halo rows exchanged after every Taylor term.  Parity with the
Taylor-discretised oracle on the oracle planner's schedule, both precisions
and both backward variants; batching; and the timeout path of the bounded
neighbour wait, forced from the host."""
import os

import numpy as np
import pytest

from gpu_common import assert_parity, context, log, make_problem, oracle_schedule, run
from workloads import make_config

pytestmark = pytest.mark.gpu


def _discrete(p, sched):
    from oracle import taylor
    return taylor.hg_discrete(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets, sched, omega=p.omega,
                              w_fid=p.w_fid, w_pen=p.w_pen)


@pytest.mark.parametrize("mode,C", [("reconstruct", 0), ("checkpoint", 3)])
def test_split_transmon_cavity(mode, C):
    """transmon(8) x cavity(520), d = 4160 (beyond one workgroup in either
    precision), N = 8, S = 4, penalty on."""
    p = make_config("cfg5", N=8, d_c=520)
    prob = make_problem(p)
    sched = oracle_schedule(p)
    ref = _discrete(p, sched)
    for dt in ("c128", "c64"):
        log(f"[case] split d={p.dim} N=8 S=4 {dt} {mode}")
        r = run(p, dt, prob=prob, mode=mode, ckpt_every=C)
        assert_parity(r, ref, dt, label=f"split{p.dim}-{mode}")


def test_split_complex128_cfg3_structure():
    """Nine-diagonal cfg3 structure with a 160-level cavity (d = 2560):
    complex128 runs split (two parts of the cavity range), complex64 in one
    workgroup; both against the same oracle."""
    p = make_config("cfg3", N=4, d_c=160)
    sched = oracle_schedule(p)
    ref = _discrete(p, sched)
    prob = make_problem(p)
    for dt in ("c128", "c64"):
        log(f"[case] cfg3 structure d={p.dim} N=4 S=16 {dt}")
        assert_parity(run(p, dt, prob=prob), ref, dt, label="cfg3c160")


def test_split_batch_equals_alone():
    """Two amplitude sets in one call equal each evaluated alone (bitwise)."""
    from workloads.configs import _amps
    p = make_config("cfg5", N=6, d_c=520)
    prob = make_problem(p)
    u2 = np.stack([p.u, _amps(np.random.default_rng(77), p.n_ctrl, p.n_steps)])
    log("[case] split batch of 2 vs alone, c64")
    both = run(p, "c64", prob=prob, batch_u=u2)
    for b in range(2):
        alone = run(p, "c64", prob=prob, batch_u=u2[b:b + 1])
        assert both.cost[b] == alone.cost[0]
        assert np.array_equal(both.grad[b].cpu().numpy(), alone.grad[0].cpu().numpy())


def test_split_wait_timeout_is_reported(monkeypatch):
    """With the longest neighbour wait set to zero ticks, waits that are not
    satisfied at once give up: the kernels still finish and the call returns
    HG_ERR_DEVICE; with the default limit the same call succeeds afterwards."""
    import paper_2304_06200_amd as hg
    p = make_config("cfg5", N=4, d_c=520)
    prob = make_problem(p)
    monkeypatch.setenv("HG_SPLIT_WAIT_TICKS", "0")
    log("[case] split wait limit 0 ticks: expect DEVICE")
    with pytest.raises(hg._lib.HGError) as e:
        run(p, "c64", prob=prob)
    assert e.value.status == hg._lib.HG_ERR_DEVICE, str(e.value)
    monkeypatch.delenv("HG_SPLIT_WAIT_TICKS")
    ref = _discrete(p, oracle_schedule(p))
    assert_parity(run(p, "c64", prob=prob), ref, "c64", label="after-timeout")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_cfg5_full_dimension_prefix(dtype):
    """transmon(8) x cavity(1024), d = 8192, S = 4: the first 12 steps, both
    backward variants, against the discretised oracle."""
    p = make_config("cfg5", N=12)
    prob = make_problem(p)
    sched = oracle_schedule(p)
    ref = _discrete(p, sched)
    for mode, C in (("reconstruct", 0), ("checkpoint", 5)):
        log(f"[case] cfg5 d=8192 N=12 {dtype} {mode}")
        assert_parity(run(p, dtype, prob=prob, mode=mode, ckpt_every=C), ref, dtype,
                      label=f"cfg5[:12]-{mode}")

"""Checkpointed-state variant of the backward sweep, and the memory footprint
of both variants (Table I: HG state memory does not grow with N)."""
import numpy as np
import pytest

from gpu_common import assert_parity, golden, log, make_problem, run
from workloads import make_config

pytestmark = pytest.mark.gpu


def _oracle(p):
    from oracle import grape
    return grape.cost_and_grad(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets, omega=p.omega,
                               w_fid=p.w_fid, w_pen=p.w_pen)


@pytest.mark.parametrize("C", [1, 7, 30, 200, 1000])
def test_checkpoint_parity(C):
    p = make_config("cfg2", N=200, d_c=12)
    ref = _oracle(p)
    log(f"[case] checkpoint C={C} cfg2 d_c=12 N=200")
    for dt in ("c128", "c64"):
        r = run(p, dt, mode="checkpoint", ckpt_every=C)
        assert_parity(r, ref, dt, label=f"ckpt{C}")
        assert r.drift[0] == 0.0


def test_checkpoint_matches_reconstruction_c128():
    p = make_config("cfg3", N=40, d_c=20)
    prob = make_problem(p)
    a = run(p, "c128", prob=prob)
    b = run(p, "c128", prob=prob, mode="checkpoint", ckpt_every=9)
    log(f"[case] ckpt vs reconstruct cfg3c20: drift(reconstruct) {a.drift[0]:.2e}")
    assert abs(a.cost[0] - b.cost[0]) <= 1e-13
    ga, gb = a.grad.cpu().numpy(), b.grad.cpu().numpy()
    assert np.linalg.norm(ga - gb) <= 1e-12 * np.linalg.norm(gb)


def test_cfg2_full_checkpoint_vs_golden():
    p = make_config("cfg2")
    log("[case] cfg2 full, checkpoint every 100")
    for dt in ("c128", "c64"):
        assert_parity(run(p, dt, mode="checkpoint", ckpt_every=100), golden("cfg2"), dt,
                      label="cfg2-ckpt")


def test_footprint_state_memory():
    """Reconstruction: the state part of the workspace does not grow with N
    (only O(N) scalars per step: norms, schedule, gradient partials).
    Checkpoint: (ceil(N/C) + C) d S extra states."""
    import torch
    from paper_2304_06200_amd import _lib as L
    from paper_2304_06200_amd.api import make_desc
    p = make_config("cfg3", N=10)
    prob = make_problem(p)
    d, S, K = p.dim, p.n_states, p.n_ctrl

    def fp(N, mode=L.HG_MODE_RECONSTRUCT, C=0, dtype=L.HG_C64):
        desc = make_desc(N, 1, p.dt, 1, S, 1, 1, 1.0, 1.0, 1e-12, dtype, 1, None, mode=mode,
                         ckpt_every=C)
        return L.hg_eval_footprint(prob.handle, desc)
    per_step = 8 + 8 + 8 * S * K          # theta, (m,s), FP64 gradient partials
    a, b = fp(1000), fp(5000)
    log(f"[case] footprint reconstruct N=1000 {a} B, N=5000 {b} B")
    assert abs((b - a) - 4000 * per_step) <= 4 * 256 * 8
    c = fp(5000, L.HG_MODE_CHECKPOINT, 100)
    extra = (50 + 100) * d * S * 8
    assert abs((c - b) - extra) <= 2 * 256


def test_checkpoint_drift_is_rounding_of_psi0():
    """In the checkpoint variant the states are never rebuilt, so the reported
    drift is only the rounding of psi_0 to the working precision when it is
    stored as checkpoint 0: exactly 0 in complex128 and ||fl32(psi_0) - psi_0||
    in complex64 (a random normalised psi_0 is not representable in FP32)."""
    import dataclasses
    p = make_config("cfg2", N=60, d_c=10)
    rng = np.random.default_rng(61)
    psi0 = rng.normal(size=p.psi0.shape) + 1j * rng.normal(size=p.psi0.shape)
    psi0 /= np.linalg.norm(psi0, axis=1, keepdims=True)
    q = dataclasses.replace(p, psi0=psi0)
    ref = _oracle(q)
    log("[case] checkpoint drift, random psi0, cfg2 d_c=10 N=60")
    r128 = run(q, "c128", mode="checkpoint", ckpt_every=7)
    assert_parity(r128, ref, "c128", label="ckpt-rand-psi0")
    assert r128.drift[0] == 0.0
    r64 = run(q, "c64", mode="checkpoint", ckpt_every=7)
    assert_parity(r64, ref, "c64", label="ckpt-rand-psi0")
    expect = max(np.linalg.norm(psi0[h].astype(np.complex64).astype(np.complex128) - psi0[h])
                 for h in range(psi0.shape[0]))
    log(f"[case] c64 checkpoint drift {r64.drift[0]:.3e}, FP32 rounding of psi0 {expect:.3e}")
    assert 0.0 < r64.drift[0] <= 1e-7
    assert r64.drift[0] == pytest.approx(expect, rel=1e-6)

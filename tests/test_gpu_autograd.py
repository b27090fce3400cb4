"""The HG gradient as a torch.autograd.Function, checked against finite differences."""
import numpy as np
import pytest

from gpu_common import log, make_problem, oracle_schedule
from workloads import make_config

pytestmark = pytest.mark.gpu


def _dev(p):
    import torch
    return (torch.tensor(p.psi0, dtype=torch.complex128, device="cuda"),
            torch.tensor(p.targets, dtype=torch.complex128, device="cuda"))


def test_autograd_vs_finite_differences_cfg3_full():
    """d=1600, N=2000, S=16: the autograd gradient on 32 random (k, n) entries
    against central differences of the same (schedule-frozen) cost; all 64
    perturbed evaluations run as one batch."""
    import torch
    import paper_2304_06200_amd as hg
    p = make_config("cfg3")
    sched = oracle_schedule(p)
    prob = make_problem(p)
    psi0, tg = _dev(p)
    opts = dict(w_fid=p.w_fid, w_pen=p.w_pen, tau=p.tau, dtype="c128", schedule=sched)
    u = torch.tensor(p.u, dtype=torch.float64, device="cuda", requires_grad=True)
    log("[case] autograd cfg3 full size, 32 FD pairs")
    cost = hg.hg_cost(prob, u, psi0, tg, p.dt, **opts)
    cost.backward()
    g = u.grad.cpu().numpy()
    rng = np.random.default_rng(33)
    pairs = [(int(rng.integers(p.n_ctrl)), int(rng.integers(p.n_steps))) for _ in range(32)]
    h = 1e-6
    batch = []
    for k, n in pairs:
        for sgn in (1.0, -1.0):
            v = p.u.copy()
            v[k, n] += sgn * h
            batch.append(v)
    ub = torch.tensor(np.stack(batch), dtype=torch.float64, device="cuda")
    r = hg.evaluate(prob, ub, psi0, tg, p.dt, want_grad=False, **opts)
    fd = (r.cost[0::2] - r.cost[1::2]) / (2 * h)
    ref = np.array([g[k, n] for k, n in pairs])
    err = np.max(np.abs(fd - ref)) / np.max(np.abs(g))
    log(f"[autograd] max |fd - grad| / max|grad| = {err:.2e}")
    assert err < 1e-6


def test_autograd_batched_and_descent_step():
    """Batched costs: d(sum of costs)/du gives each entry's gradient; one GRAPE
    steepest-descent step (Sec. II) with a small rate lowers the cost."""
    import torch
    import paper_2304_06200_amd as hg
    p = make_config("cfg2", N=100, d_c=10)
    prob = make_problem(p)
    psi0, tg = _dev(p)
    us = np.stack([p.u, 0.5 * p.u])
    u = torch.tensor(us, dtype=torch.float64, device="cuda", requires_grad=True)
    c = hg.hg_cost(prob, u, psi0, tg, p.dt, w_fid=p.w_fid, w_pen=p.w_pen, tau=p.tau)
    assert c.shape == (2,)
    (3.0 * c[0] + 0.5 * c[1]).backward()
    single = hg.evaluate(prob, torch.tensor(us, device="cuda"), psi0, tg, p.dt, w_fid=p.w_fid,
                         w_pen=p.w_pen, tau=p.tau)
    np.testing.assert_allclose(u.grad[0].cpu().numpy(), 3.0 * single.grad[0].cpu().numpy(), rtol=1e-15)
    np.testing.assert_allclose(u.grad[1].cpu().numpy(), 0.5 * single.grad[1].cpu().numpy(), rtol=1e-15)
    # one steepest-descent step
    v = torch.tensor(p.u, dtype=torch.float64, device="cuda", requires_grad=True)
    c0 = hg.hg_cost(prob, v, psi0, tg, p.dt, w_fid=p.w_fid, w_pen=p.w_pen, tau=p.tau)
    c0.backward()
    with torch.no_grad():
        v2 = v - 1e-3 * v.grad / v.grad.norm()
    c1 = hg.hg_cost(prob, v2, psi0, tg, p.dt, w_fid=p.w_fid, w_pen=p.w_pen, tau=p.tau)
    log(f"[autograd] descent step: {float(c0):.9f} -> {float(c1):.9f}")
    assert float(c1) < float(c0)

"""hg_eval_noalloc (the entry point that allocates nothing) against hg_eval:
the same results on two calls in a row, the second with a smaller input, with
every buffer preallocated by the caller and the library's workspace pool left
untouched."""
import numpy as np
import pytest

from gpu_common import context, log, make_problem
from workloads import make_config

pytestmark = pytest.mark.gpu


def _inputs(p, B):
    import torch
    from workloads.configs import _amps
    us = np.stack([p.u] + [_amps(np.random.default_rng(900 + b), p.n_ctrl, p.n_steps)
                           for b in range(1, B)])
    return (torch.tensor(us, dtype=torch.float64, device="cuda"),
            torch.tensor(p.psi0, dtype=torch.complex128, device="cuda"),
            torch.tensor(p.targets, dtype=torch.complex128, device="cuda"))


def _compare(a, b):
    for f in ("cost", "infidelity", "penalty", "sum_mu", "drift"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    assert np.array_equal(a.overlap, b.overlap)
    assert np.array_equal(a.grad.cpu().numpy(), b.grad.cpu().numpy())


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_noalloc_equals_eval_twice_second_smaller(dtype):
    import torch
    import paper_2304_06200_amd as hg
    from paper_2304_06200_amd import _lib as L
    scratch, stage = L.hg_eval_noalloc_limits()
    assert scratch == 64 << 20 and stage == 2 << 20
    cases = [(make_config("cfg3", N=40, d_c=40), 3, "reconstruct", 0),
             (make_config("cfg2", N=25, d_c=10), 1, "checkpoint", 7)]
    for p, B, mode, C in cases:
        prob = make_problem(p)
        u, psi0, tg = _inputs(p, B)
        kw = dict(w_fid=p.w_fid, w_pen=p.w_pen, tau=p.tau, dtype=dtype, mode=mode, ckpt_every=C)
        ref = hg.evaluate(prob, u, psi0, tg, p.dt, **kw)
        g = torch.empty((B, p.n_ctrl, p.n_steps), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        hg.api.mem_pool_peak(context(), reset=True)
        log(f"[case] noalloc {dtype} d={p.dim} N={p.n_steps} B={B} {mode}")
        got = hg.evaluate(prob, u, psi0, tg, p.dt, noalloc=True, grad_out=g, **kw)
        assert hg.api.mem_pool_peak(context()) == 0  # nothing taken from the pool
        _compare(got, ref)


def test_noalloc_rejects_oversized_and_timing():
    import paper_2304_06200_amd as hg
    from paper_2304_06200_amd import _lib as L
    p = make_config("cfg3", N=2000)
    prob = make_problem(p)
    u, psi0, tg = _inputs(p, 16)
    log("[case] noalloc oversized workspace (cfg3 batch 16 with checkpoints every step)")
    with pytest.raises(L.HGError) as e:
        hg.evaluate(prob, u, psi0, tg, p.dt, dtype="c64", mode="checkpoint", ckpt_every=1,
                    noalloc=True)
    assert e.value.status == L.HG_ERR_OUT_OF_MEMORY
    q = make_config("cfg2", N=10, d_c=8)
    pq = make_problem(q)
    uq, p0, t0 = _inputs(q, 1)
    with pytest.raises(L.HGError) as e:
        hg.evaluate(pq, uq, p0, t0, q.dt, dtype="c64", timing=True, noalloc=True)
    assert e.value.status == L.HG_ERR_INVALID_ARG

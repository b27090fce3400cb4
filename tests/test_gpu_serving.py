"""Serving: continuous admission of heterogeneous requests (transmon x cavity
with different cavity sizes, step counts and state counts) onto one GPU."""
import numpy as np
import pytest

from gpu_common import TOL, assert_parity, context, log
from workloads.configs import serving_request, serving_stream

pytestmark = pytest.mark.gpu


def _dev(p):
    import torch
    return (torch.tensor(p.u, dtype=torch.float64, device="cuda"),
            torch.tensor(p.psi0, dtype=torch.complex128, device="cuda"),
            torch.tensor(p.targets, dtype=torch.complex128, device="cuda"))


_probs = {}


def _problem(p):
    import paper_2304_06200_amd as hg
    key = p.dims
    if key not in _probs:
        _probs[key] = hg.Problem(context(), p.H0, p.Hk, p.omega)
    return _probs[key]


def _stream(n, seed=4):
    shapes = serving_stream(n_req=n, seed=seed, d_c_max=120, n_max=300)
    return [serving_request(s["index"], s["d_c"], s["N"], s["S"]) for s in shapes]


def _kw(p, dtype):
    return dict(w_fid=p.w_fid, w_pen=p.w_pen, tau=p.tau, dtype=dtype)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_mixed_stream_equals_alone(dtype):
    import paper_2304_06200_amd as hg
    reqs = _stream(20)
    sv = hg.Server(context(), hbm_budget_bytes=4 << 30, max_inflight=6)
    log(f"[case] serving 20 mixed requests {dtype}")
    handles = [sv.submit(_problem(p), *_dev(p), p.dt, **_kw(p, dtype)) for p in reqs]
    out = [sv.wait(h) for h in handles]
    sv.close()
    for p, (r, lat, q) in zip(reqs, out):
        alone = hg.evaluate(_problem(p), *_dev(p), p.dt, **_kw(p, dtype))
        assert r.cost[0] == alone.cost[0], p.name
        assert np.array_equal(r.grad.cpu().numpy(), alone.grad.cpu().numpy()), p.name
        assert lat >= q >= 0.0
    # the smallest requests against the oracle
    from oracle import grape
    small = sorted(range(len(reqs)), key=lambda i: reqs[i].dim * reqs[i].n_steps)[:3]
    for i in small:
        p = reqs[i]
        ref = grape.cost_and_grad(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets, omega=p.omega,
                                  w_fid=p.w_fid, w_pen=p.w_pen)
        assert_parity(out[i][0], ref, dtype, label=p.name)
    lats = [o[1] for o in out]
    log(f"[serving] {dtype}: p50 {np.percentile(lats, 50):.1f} ms p99 {np.percentile(lats, 99):.1f} ms")


def test_admission_respects_budget_and_rejects_oversize():
    import paper_2304_06200_amd as hg
    from paper_2304_06200_amd import _lib as L
    reqs = _stream(8, seed=5)
    big = max(reqs, key=lambda p: p.dim * p.n_states * p.n_steps)
    # budget that holds the largest request but not two of them
    sv0 = hg.Server(context(), hbm_budget_bytes=1 << 40, max_inflight=1)
    h = sv0.submit(_problem(big), *_dev(big), big.dt, **_kw(big, "c64"))
    sv0.wait(h)
    sv0.close()
    from paper_2304_06200_amd.api import make_desc
    d = make_desc(big.n_steps, 1, big.dt, 1, big.n_states, 1, 1, 1.0, 1.0, big.tau, L.HG_C64, 1)
    need = L.hg_eval_footprint(_problem(big).handle, d)
    budget = int(1.5 * (need + 64 * big.dim * big.n_states + 16 * 4 * big.n_steps))
    sv = hg.Server(context(), hbm_budget_bytes=budget, max_inflight=4)
    log(f"[case] admission budget {budget} B")
    handles = [sv.submit(_problem(p), *_dev(p), p.dt, **_kw(p, "c64")) for p in reqs]
    seen = 0
    while not all(sv.poll(h) for h in handles):
        used, queued, running = sv.info()
        assert used <= budget
        seen = max(seen, running)
    for h in handles:
        sv.wait(h)
    # a request larger than the whole budget is refused at submit
    tiny = hg.Server(context(), hbm_budget_bytes=4096, max_inflight=1)
    with pytest.raises(L.HGError) as e:
        tiny.submit(_problem(big), *_dev(big), big.dt, **_kw(big, "c64"))
    assert e.value.status == L.HG_ERR_OUT_OF_MEMORY
    tiny.close()
    sv.close()


def test_cancel_queued_request():
    import paper_2304_06200_amd as hg
    from paper_2304_06200_amd import _lib as L
    reqs = _stream(4, seed=6)
    sv = hg.Server(context(), hbm_budget_bytes=4 << 30, max_inflight=1)
    hs = [sv.submit(_problem(p), *_dev(p), p.dt, **_kw(p, "c64")) for p in reqs]
    sv.cancel(hs[-1])
    for h in hs[:-1]:
        sv.wait(h)
    with pytest.raises(L.HGError) as e:
        sv.wait(hs[-1])
    assert e.value.status == L.HG_ERR_CANCELLED
    sv.close()


def test_dense_and_dia_problems_in_one_stream():
    """Requests on dense-storage problems (the MFMA path) and on DIA problems share
    one server; each result equals the same request evaluated alone."""
    import paper_2304_06200_amd as hg
    from workloads import make_config
    reqs = _stream(6, seed=8)
    dense_p = [make_config("gate3", d_t=4, N=2, random_amps=True, seed=s) for s in (1, 2)]
    dense_prob = hg.Problem(context(), dense_p[0].H0, dense_p[0].Hk, dense_p[0].omega, dense=True)
    sv = hg.Server(context(), hbm_budget_bytes=4 << 30, max_inflight=4)
    log("[case] serving: 6 DIA requests and 2 dense-storage gate requests")
    hs = [sv.submit(_problem(p), *_dev(p), p.dt, **_kw(p, "c64")) for p in reqs[:3]]
    hs += [sv.submit(dense_prob, *_dev(p), p.dt, **_kw(p, "c64")) for p in dense_p]
    hs += [sv.submit(_problem(p), *_dev(p), p.dt, **_kw(p, "c64")) for p in reqs[3:]]
    out = [sv.wait(h) for h in hs]
    sv.close()
    order = [(p, _problem(p)) for p in reqs[:3]] + [(p, dense_prob) for p in dense_p] + \
            [(p, _problem(p)) for p in reqs[3:]]
    for (p, prob), (r, lat, q) in zip(order, out):
        alone = hg.evaluate(prob, *_dev(p), p.dt, **_kw(p, "c64"))
        assert r.cost[0] == alone.cost[0], p.name
        assert np.array_equal(r.grad.cpu().numpy(), alone.grad.cpu().numpy()), p.name


def test_submit_waits_for_inputs_on_caller_stream():
    """Requests whose inputs are still being produced on torch's current
    stream when submit is called (a long GEMM chain first, then the amplitudes
    and states written by a kernel that depends on it), batched (B = 3) and
    with (S, d) states expanded by submit itself: every result equals the
    synchronous evaluate() of the same inputs, bitwise."""
    import torch
    import paper_2304_06200_amd as hg
    reqs = _stream(4, seed=11)
    sv = hg.Server(context(), hbm_budget_bytes=4 << 30, max_inflight=4)
    log("[case] serving: inputs produced on the caller's stream right before submit, B=3")
    rng = np.random.default_rng(12)
    side = torch.cuda.Stream()
    handles, inputs = [], []
    with torch.cuda.stream(side):
        for p in reqs:
            u_host = np.stack([p.u, p.u * 0.9, p.u * 1.1])
            u_src = torch.tensor(u_host, dtype=torch.float64, device="cuda")
            psi_src = torch.tensor(p.psi0, dtype=torch.complex128, device="cuda")
            tg_src = torch.tensor(p.targets, dtype=torch.complex128, device="cuda")
            torch.cuda.synchronize()
            big = torch.tensor(rng.standard_normal((2048, 2048)), dtype=torch.float32,
                               device="cuda")
            for _ in range(12):
                big = (big @ big) * (1.0 / 2048)
            zero = (big.sum() * 0.0).to(torch.float64)  # finite, depends on the chain
            u = torch.empty_like(u_src)
            u.copy_(u_src + zero)
            psi = torch.empty_like(psi_src)
            psi.copy_(psi_src + zero)
            h = sv.submit(_problem(p), u, psi, tg_src, p.dt, **_kw(p, "c64"))
            handles.append(h)
            inputs.append((u_src, psi_src, tg_src))
    out = [sv.wait(h) for h in handles]
    sv.close()
    torch.cuda.synchronize()
    for p, (u_src, psi_src, tg_src), (r, _, _) in zip(reqs, inputs, out):
        alone = hg.evaluate(_problem(p), u_src, psi_src, tg_src, p.dt, **_kw(p, "c64"))
        for b in range(3):
            assert r.cost[b] == alone.cost[b], (p.name, b)
        assert np.array_equal(r.grad.cpu().numpy(), alone.grad.cpu().numpy()), p.name


def test_spread_requests_equal_spread_alone():
    """Requests submitted with spread backward sweeps equal the same spread
    evaluation run alone (bitwise), while other requests run beside them."""
    import paper_2304_06200_amd as hg
    reqs = _stream(8, seed=21)
    sv = hg.Server(context(), hbm_budget_bytes=4 << 30, max_inflight=4)
    log("[case] serving 8 requests, spread on every other one, c64")
    hs = [sv.submit(_problem(p), *_dev(p), p.dt, spread=(i % 2 == 0), **_kw(p, "c64"))
          for i, p in enumerate(reqs)]
    out = [sv.wait(h) for h in hs]
    sv.close()
    for i, (p, (r, _, _)) in enumerate(zip(reqs, out)):
        alone = hg.evaluate(_problem(p), *_dev(p), p.dt, spread=(i % 2 == 0), **_kw(p, "c64"))
        assert r.cost[0] == alone.cost[0], p.name
        assert np.array_equal(r.grad.cpu().numpy(), alone.grad.cpu().numpy()), p.name

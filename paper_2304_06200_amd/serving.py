"""Serving wrapper: submit cost+gradient requests of any problem and shape to
libhgrape's server (continuous admission by HBM footprint, concurrent device
execution) and collect results with their latencies."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from . import _lib as L
from .api import Context, EvalResult, Problem, make_desc


@dataclass
class Handle:
    req_id: int
    n_batch: int
    keep: tuple          # device tensors and host arrays the request reads/writes
    results: object      # ctypes array of hg_result
    grad: object


class Server:
    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_inflight: int = 8):
        self.ctx = ctx
        self.handle = L.hg_server_create(ctx.handle, int(hbm_budget_bytes), int(max_inflight))

    def submit(self, problem: Problem, u, psi0, targets, dt: float, *, w_fid: float = 1.0,
               w_pen: float = 0.0, w_int: float = 0.0, tau: float = 1e-12, dtype: str = "c64",
               renorm_every: Optional[int] = None, mode: str = "reconstruct",
               ckpt_every: int = 0, spread: bool = False) -> Handle:
        """u: float64 device tensor (K, N) or (B, K, N); psi0, targets: complex128
        device tensors (S, d) or (B, S, d).  Returns a handle for wait().

        The inputs may still be being produced on torch's current stream: the
        request's device work waits for everything queued there up to this
        call (including the copies made here), so no synchronisation is needed
        before submit.  The gradient tensor is complete once wait() returns."""
        import torch
        if u.dim() == 2:
            u = u.unsqueeze(0)
        if psi0.dim() == 2:
            psi0 = psi0.unsqueeze(0)
        if targets.dim() == 2:
            targets = targets.unsqueeze(0)
        B, K, N = u.shape
        psi0 = psi0.expand(B, -1, -1).contiguous()
        targets = targets.expand(B, -1, -1).contiguous()
        u = u.contiguous()
        S = psi0.shape[1]
        code = {"c128": L.HG_C128, "c64": L.HG_C64}[dtype]
        if renorm_every is None:
            renorm_every = 1 if dtype == "c64" else 0
        mcode = {"reconstruct": L.HG_MODE_RECONSTRUCT, "checkpoint": L.HG_MODE_CHECKPOINT}[mode]
        desc = make_desc(N, B, dt, int(u.data_ptr()) if K > 0 else None, S, int(psi0.data_ptr()),
                         int(targets.data_ptr()), w_fid, w_pen, tau, code, renorm_every, None,
                         mode=mcode, ckpt_every=ckpt_every, w_int=w_int,
                         flags=L.HG_FLAG_SPREAD if spread else 0)
        grad = torch.empty((B, K, N), dtype=torch.float64, device=u.device) if K > 0 else None
        res = (L.hg_result * B)()
        rid = L.hg_server_submit(self.handle, problem.handle, desc, res,
                                 int(grad.data_ptr()) if grad is not None else None,
                                 torch.cuda.current_stream(u.device).cuda_stream)
        return Handle(rid, B, (u, psi0, targets, problem), res, grad)

    def poll(self, h: Handle) -> bool:
        return L.hg_server_poll(self.handle, h.req_id)

    def cancel(self, h: Handle) -> None:
        L.hg_server_cancel(self.handle, h.req_id)

    def wait(self, h: Handle):
        """(EvalResult, latency_ms, queued_ms); raises HGError on a failed request."""
        st, lat, q = L.hg_server_wait(self.handle, h.req_id)
        if st != L.HG_OK:
            raise L.HGError(st, "hg_server_wait", L.hg_last_error())
        r = h.results
        res = EvalResult(
            cost=np.array([x.cost for x in r]), infidelity=np.array([x.infidelity for x in r]),
            penalty=np.array([x.penalty for x in r]),
            overlap=np.array([complex(x.overlap_re, x.overlap_im) for x in r]),
            sum_mu=np.array([x.sum_mu for x in r], dtype=np.int64),
            max_theta=np.array([x.max_theta for x in r]), max_bound=np.array([x.max_bound for x in r]),
            drift=np.array([x.drift for x in r]), grad=h.grad,
            integrated_infidelity=np.array([x.integrated_infidelity for x in r]))
        return res, lat, q

    def info(self):
        """(device bytes admitted, queued, running)."""
        return L.hg_server_info(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            L.hg_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def percentiles(latencies_ms: List[float]):
    a = np.asarray(latencies_ms, dtype=np.float64)
    return {"p50_ms": float(np.percentile(a, 50)), "p99_ms": float(np.percentile(a, 99)),
            "mean_ms": float(a.mean()), "max_ms": float(a.max())}

"""Torch-facing wrapper around the C ABI (memory and streams only).

Every number is computed by libhgrape's HIP kernels and host planner; this
module only turns scipy/numpy operators into hg_csr structs and torch tensors
into device pointers on the current HIP stream.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import _lib as L


def _torch():
    import torch
    return torch


class Context:
    """One HIP device."""

    def __init__(self, device: int = 0):
        self.device = device
        self.handle = L.hg_create(device)

    def close(self):
        if self.handle:
            L.hg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _csr_struct(m, dim: int, keep: list) -> L.hg_csr:
    import scipy.sparse as sp
    m = sp.csr_matrix(m, dtype=np.complex128)
    indptr = np.ascontiguousarray(m.indptr, dtype=np.int64)
    indices = np.ascontiguousarray(m.indices, dtype=np.int32)
    values = np.ascontiguousarray(m.data.astype(np.complex128).view(np.float64))
    keep.extend([indptr, indices, values])
    return L.hg_csr(dim, indptr.ctypes.data_as(C.POINTER(C.c_int64)),
                    indices.ctypes.data_as(C.POINTER(C.c_int32)),
                    values.ctypes.data_as(C.POINTER(C.c_double)))


class Problem:
    """Drift H0, controls Hk and an optional diagonal penalty Omega, copied to
    the device (immutable; may be shared by concurrent evaluations).

    dense=False stores the operators by diagonals (sparse, banded problems);
    dense=True stores them as dense matrices and evaluations run the MFMA
    path (wide state blocks, dense operators)."""

    def __init__(self, ctx: Context, H0, Hk: Sequence, omega: Optional[np.ndarray] = None,
                 dense: bool = False):
        self.ctx = ctx
        dim = H0.shape[0]
        keep: list = []
        h0 = _csr_struct(H0, dim, keep)
        hk = [_csr_struct(h, dim, keep) for h in Hk]
        om = None if omega is None else np.ascontiguousarray(omega, dtype=np.float64)
        create = L.hg_problem_create_dense if dense else L.hg_problem_create
        self.handle = create(ctx.handle, dim, len(Hk), h0, hk, om)
        self.dense = dense
        self.info = L.hg_problem_info(self.handle)
        self.dim = dim
        self.n_ctrl = len(Hk)
        self.has_penalty = omega is not None

    def close(self):
        if getattr(self, "handle", None):
            L.hg_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class EvalResult:
    cost: np.ndarray        # (B,)
    infidelity: np.ndarray  # (B,)
    penalty: np.ndarray     # (B,)
    overlap: np.ndarray     # (B,) complex
    sum_mu: np.ndarray      # (B,) int
    max_theta: np.ndarray
    max_bound: np.ndarray
    drift: np.ndarray
    grad: object            # torch tensor (B, K, N) float64 on the device, or None
    ms_forward: float = 0.0   # kernel times of the whole batch (timing=True)
    ms_backward: float = 0.0
    integrated_infidelity: Optional[np.ndarray] = None  # (B,) C3 (w_int != 0)


def _ptr(t) -> int:
    return int(t.data_ptr())


def make_desc(n_steps, n_batch, dt, u, n_states, psi0, targets, w_fid, w_pen, tau, dtype,
              renorm_every, schedule=None, mode=L.HG_MODE_RECONSTRUCT, ckpt_every=0, flags=0,
              w_int=0.0, rule=L.HG_PLAN_SMALLEST_S, method=L.HG_METHOD_TAYLOR):
    d = L.hg_eval_desc()
    d.n_steps = n_steps
    d.n_batch = n_batch
    d.dt = dt
    d.u = u
    d.n_states = n_states
    d.psi0 = psi0
    d.targets = targets
    d.w_fid = w_fid
    d.w_pen = w_pen
    d.w_int = w_int
    d.tau = tau
    d.dtype = dtype
    d.mode = mode
    d.ckpt_every = ckpt_every
    d.renorm_every = renorm_every
    d.schedule = schedule
    d.flags = flags
    d.rule = rule
    d.method = method
    return d


RULES = {"smallest_s": L.HG_PLAN_SMALLEST_S, "min_mu": L.HG_PLAN_MIN_MU}
METHODS = {"taylor": L.HG_METHOD_TAYLOR, "diag": L.HG_METHOD_DIAG, "auto": L.HG_METHOD_AUTO}


def evaluate(problem: Problem, u, psi0, targets, dt: float, *, w_fid: float = 1.0,
             w_pen: float = 0.0, w_int: float = 0.0, tau: float = 1e-12, dtype: str = "c128",
             renorm_every: Optional[int] = None, schedule: Optional[np.ndarray] = None,
             want_grad: bool = True, timing: bool = False, mode: str = "reconstruct",
             ckpt_every: int = 0, stream=None, rule: str = "smallest_s",
             noalloc: bool = False, grad_out=None, spread: bool = False,
             method: str = "taylor") -> EvalResult:
    """Cost and gradient of B amplitude sets.

    u        torch float64 device tensor (K, N) or (B, K, N)
    psi0     torch complex128 device tensor (S, d) or (B, S, d), normalised rows
    targets  torch complex128 device tensor, same shape as psi0
    dtype    "c128" or "c64" (arithmetic of the Taylor products)
    schedule optional host int array (2, B, N) or (2, N) of frozen (m, s)
    mode     "reconstruct" (HG inverse propagation) or "checkpoint" (psi stored
             every ckpt_every steps, segments re-propagated in the backward sweep)
    w_int    weight of the time-integrated infidelity C3 (0 = off)
    rule     planner rule: "smallest_s" (the paper's) or "min_mu" (fewest products)
    noalloc  run through hg_eval_noalloc (the library's fixed scratch; no
             allocation in the call, one call at a time per device)
    grad_out optional preallocated float64 device tensor (B, K, N) for the gradient
    spread   let several workgroups share a column's backward sweep when the
             batch leaves compute units idle (lower latency, more total work)
    method   "taylor", "diag" (diagonalise H_n per step; dense storage) or "auto"
    """
    torch = _torch()
    if u.dim() == 2:
        u = u.unsqueeze(0)
    if psi0.dim() == 2:
        psi0 = psi0.unsqueeze(0)
    if targets.dim() == 2:
        targets = targets.unsqueeze(0)
    B, K, N = u.shape
    if psi0.shape[0] != B:
        psi0 = psi0.expand(B, -1, -1)
    if targets.shape[0] != B:
        targets = targets.expand(B, -1, -1)
    u = u.contiguous()
    psi0 = psi0.contiguous()
    targets = targets.contiguous()
    for name, t, dt_ in (("u", u, torch.float64), ("psi0", psi0, torch.complex128),
                         ("targets", targets, torch.complex128)):
        if t.dtype != dt_ or not t.is_cuda:
            raise TypeError(f"{name} must be a {dt_} device tensor")
    if K != problem.n_ctrl or psi0.shape[2] != problem.dim or targets.shape != psi0.shape:
        raise ValueError("shape mismatch between amplitudes, states and problem")
    S = psi0.shape[1]
    code = {"c128": L.HG_C128, "c64": L.HG_C64}[dtype]
    if renorm_every is None:
        renorm_every = 1 if dtype == "c64" else 0
    sched_p = None
    sched_arr = None
    if schedule is not None:
        sched_arr = np.asarray(schedule, dtype=np.int32)
        if sched_arr.ndim == 2:
            sched_arr = np.repeat(sched_arr[:, None, :], B, axis=1)
        sched_arr = np.ascontiguousarray(sched_arr.reshape(2, B, N))
        sched_p = sched_arr.ctypes.data_as(C.POINTER(C.c_int32))
    mcode = {"reconstruct": L.HG_MODE_RECONSTRUCT, "checkpoint": L.HG_MODE_CHECKPOINT}[mode]
    desc = make_desc(N, B, dt, _ptr(u) if K > 0 else None, S, _ptr(psi0), _ptr(targets),
                     w_fid, w_pen, tau, code, renorm_every, sched_p, mode=mcode,
                     ckpt_every=ckpt_every,
                     flags=(L.HG_FLAG_TIMING if timing else 0) | (L.HG_FLAG_SPREAD if spread else 0),
                     w_int=w_int, rule=RULES[rule], method=METHODS[method])
    if grad_out is not None:
        if grad_out.shape != (B, K, N) or grad_out.dtype != torch.float64 or not grad_out.is_contiguous():
            raise ValueError("grad_out must be a contiguous float64 tensor of shape (B, K, N)")
        grad = grad_out
    else:
        grad = torch.empty((B, K, N), dtype=torch.float64, device=u.device) if want_grad and K > 0 else None
    res = (L.hg_result * B)()
    st = stream if stream is not None else torch.cuda.current_stream(u.device).cuda_stream
    call = L.hg_eval_noalloc if noalloc else L.hg_eval
    call(problem.handle, desc, res, _ptr(grad) if grad is not None else None, st)
    return EvalResult(
        cost=np.array([r.cost for r in res]),
        infidelity=np.array([r.infidelity for r in res]),
        penalty=np.array([r.penalty for r in res]),
        overlap=np.array([complex(r.overlap_re, r.overlap_im) for r in res]),
        sum_mu=np.array([r.sum_mu for r in res], dtype=np.int64),
        max_theta=np.array([r.max_theta for r in res]),
        max_bound=np.array([r.max_bound for r in res]),
        drift=np.array([r.drift for r in res]),
        grad=grad, ms_forward=res[0].ms_forward, ms_backward=res[0].ms_backward,
        integrated_infidelity=np.array([r.integrated_infidelity for r in res]))


def step_norms(problem: Problem, u, dt: float, stream=None):
    """theta[b][n] = ||-i dt H_n||_1 on the device (FP64)."""
    torch = _torch()
    if u.dim() == 2:
        u = u.unsqueeze(0)
    u = u.contiguous()
    B, K, N = u.shape
    out = torch.empty((B, N), dtype=torch.float64, device=u.device)
    st = stream if stream is not None else torch.cuda.current_stream(u.device).cuda_stream
    L.hg_step_norms(problem.handle, _ptr(u), B, N, dt, _ptr(out), st)
    return out


def mem_pool_peak(ctx: Context, reset: bool = False) -> int:
    """Measured high-water mark (bytes) of the library's evaluation workspaces
    on the context's device since the last reset; reset=True restarts it."""
    return L.hg_mem_pool_peak(ctx.handle, reset)


def plan(theta: np.ndarray, sigma: int, tau: float, u: float = 2.0 ** -53,
         rule: str = "smallest_s"):
    """Host planner of the library (FP64): (m, s) arrays for the norms theta."""
    if rule == "smallest_s":
        return L.hg_plan(np.asarray(theta, dtype=np.float64), sigma, tau, u)
    return L.hg_plan_rule(np.asarray(theta, dtype=np.float64), sigma, tau, u, RULES[rule])

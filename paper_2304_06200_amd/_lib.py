"""ctypes binding of libhgrape.so: the C ABI of include/hgrape.h, same names.

Argument marshalling only.  Every function raises HGError with the status and
the library's detail message when the C call does not return HG_OK.  The
library must have been built (``python -m paper_2304_06200_amd.build``);
importing this module fails loudly otherwise -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhgrape.so")

HG_OK = 0
HG_ERR_INVALID_ARG = 1
HG_ERR_NOT_HERMITIAN = 2
HG_ERR_NONFINITE = 3
HG_ERR_TOLERANCE_UNREACHABLE = 4
HG_ERR_OUT_OF_MEMORY = 5
HG_ERR_DEVICE = 6
HG_ERR_BUSY = 7
HG_ERR_CANCELLED = 8
HG_ERR_UNSUPPORTED = 9

HG_C64 = 0
HG_C128 = 1
HG_FLAG_TIMING = 1
HG_FLAG_SPREAD = 2
HG_MODE_RECONSTRUCT = 0
HG_MODE_CHECKPOINT = 1
HG_PLAN_SMALLEST_S, HG_PLAN_MIN_MU = 0, 1
HG_METHOD_TAYLOR, HG_METHOD_DIAG, HG_METHOD_AUTO = 0, 1, 2


class HGError(RuntimeError):
    def __init__(self, status: int, func: str, detail: str):
        self.status = status
        super().__init__(f"{func}: {status_name(status)} ({status}): {detail}")


_NAMES = {0: "HG_OK", 1: "HG_ERR_INVALID_ARG", 2: "HG_ERR_NOT_HERMITIAN", 3: "HG_ERR_NONFINITE",
          4: "HG_ERR_TOLERANCE_UNREACHABLE", 5: "HG_ERR_OUT_OF_MEMORY", 6: "HG_ERR_DEVICE",
          7: "HG_ERR_BUSY", 8: "HG_ERR_CANCELLED", 9: "HG_ERR_UNSUPPORTED"}


def status_name(s: int) -> str:
    return _NAMES.get(s, f"status {s}")


class hg_csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("indptr", C.POINTER(C.c_int64)),
                ("indices", C.POINTER(C.c_int32)), ("values", C.POINTER(C.c_double))]


class hg_eval_desc(C.Structure):
    _fields_ = [("n_steps", C.c_int32), ("n_batch", C.c_int32), ("dt", C.c_double),
                ("u", C.c_void_p), ("n_states", C.c_int32), ("psi0", C.c_void_p),
                ("targets", C.c_void_p), ("w_fid", C.c_double), ("w_pen", C.c_double),
                ("w_int", C.c_double), ("tau", C.c_double), ("dtype", C.c_int), ("mode", C.c_int),
                ("ckpt_every", C.c_int32), ("renorm_every", C.c_int32),
                ("schedule", C.POINTER(C.c_int32)), ("flags", C.c_int32), ("rule", C.c_int32),
                ("method", C.c_int32)]


class hg_result(C.Structure):
    _fields_ = [("cost", C.c_double), ("infidelity", C.c_double), ("penalty", C.c_double),
                ("integrated_infidelity", C.c_double),
                ("overlap_re", C.c_double), ("overlap_im", C.c_double), ("sum_mu", C.c_int64),
                ("max_theta", C.c_double), ("max_bound", C.c_double), ("drift", C.c_double),
                ("ms_forward", C.c_double), ("ms_backward", C.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          f"`python paper_2304_06200_amd/build.py` (hipcc, gfx950)")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "hg_create": (C.c_int, [C.c_int, C.POINTER(P)]),
        "hg_destroy": (C.c_int, [P]),
        "hg_status_string": (C.c_char_p, [C.c_int]),
        "hg_last_error": (C.c_char_p, []),
        "hg_version": (C.c_int32, []),
        "hg_problem_create": (C.c_int, [P, C.c_int64, C.c_int32, C.POINTER(hg_csr),
                                        C.POINTER(hg_csr), C.POINTER(C.c_double), C.POINTER(P)]),
        "hg_problem_create_dense": (C.c_int, [P, C.c_int64, C.c_int32, C.POINTER(hg_csr),
                                              C.POINTER(hg_csr), C.POINTER(C.c_double),
                                              C.POINTER(P)]),
        "hg_problem_destroy": (C.c_int, [P]),
        "hg_problem_info": (C.c_int, [P, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int64)]),
        "hg_plan": (C.c_int, [C.POINTER(C.c_double), C.c_int64, C.c_int32, C.c_double,
                              C.c_double, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        "hg_error_bound": (C.c_double, [C.c_double, C.c_int32, C.c_int32, C.c_int32, C.c_double]),
        "hg_plan_rule": (C.c_int, [C.POINTER(C.c_double), C.c_int64, C.c_int32, C.c_double,
                                   C.c_double, C.c_int32, C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32)]),
        "hg_step_norms": (C.c_int, [P, P, C.c_int32, C.c_int32, C.c_double, P, P]),
        "hg_eval": (C.c_int, [P, C.POINTER(hg_eval_desc), C.POINTER(hg_result), P, P]),
        "hg_eval_footprint": (C.c_int, [P, C.POINTER(hg_eval_desc), C.POINTER(C.c_size_t)]),
        "hg_server_create": (C.c_int, [P, C.c_size_t, C.c_int32, C.POINTER(P)]),
        "hg_server_submit": (C.c_int, [P, P, C.POINTER(hg_eval_desc), C.POINTER(hg_result), P,
                                       P, C.POINTER(C.c_uint64)]),
        "hg_mem_pool_peak": (C.c_int, [P, C.c_int32, C.POINTER(C.c_size_t)]),
        "hg_eval_noalloc": (C.c_int, [P, C.POINTER(hg_eval_desc), C.POINTER(hg_result), P, P]),
        "hg_eval_noalloc_limits": (C.c_int, [C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
        "hg_server_poll": (C.c_int, [P, C.c_uint64, C.POINTER(C.c_int32)]),
        "hg_server_wait": (C.c_int, [P, C.c_uint64, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "hg_server_cancel": (C.c_int, [P, C.c_uint64]),
        "hg_server_info": (C.c_int, [P, C.POINTER(C.c_size_t), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32)]),
        "hg_server_destroy": (C.c_int, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()
EXPORTED = ("hg_create", "hg_destroy", "hg_status_string", "hg_last_error", "hg_version",
            "hg_problem_create", "hg_problem_create_dense", "hg_problem_destroy", "hg_problem_info", "hg_plan", "hg_plan_rule",
            "hg_error_bound", "hg_step_norms", "hg_eval", "hg_eval_footprint", "hg_mem_pool_peak",
            "hg_eval_noalloc", "hg_eval_noalloc_limits",
            "hg_server_create", "hg_server_submit", "hg_server_poll", "hg_server_wait",
            "hg_server_cancel", "hg_server_info", "hg_server_destroy")


def _check(status: int, func: str):
    if status != HG_OK:
        raise HGError(status, func, hg_last_error())


def hg_status_string(s: int) -> str:
    return _lib.hg_status_string(s).decode()


def hg_last_error() -> str:
    return _lib.hg_last_error().decode()


def hg_version() -> int:
    return int(_lib.hg_version())


def hg_create(device_ordinal: int = 0) -> int:
    out = C.c_void_p()
    _check(_lib.hg_create(device_ordinal, C.byref(out)), "hg_create")
    return out.value


def hg_destroy(ctx: int) -> None:
    _check(_lib.hg_destroy(ctx), "hg_destroy")


def hg_problem_create(ctx: int, dim: int, n_ctrl: int, H0: hg_csr, Hk, omega_diag) -> int:
    out = C.c_void_p()
    arr = (hg_csr * max(n_ctrl, 1))(*Hk) if n_ctrl > 0 else None
    om = omega_diag.ctypes.data_as(C.POINTER(C.c_double)) if omega_diag is not None else None
    _check(_lib.hg_problem_create(ctx, dim, n_ctrl, C.byref(H0), arr, om, C.byref(out)),
           "hg_problem_create")
    return out.value


def hg_problem_create_dense(ctx: int, dim: int, n_ctrl: int, H0: hg_csr, Hk, omega_diag) -> int:
    out = C.c_void_p()
    arr = (hg_csr * max(n_ctrl, 1))(*Hk) if n_ctrl > 0 else None
    om = omega_diag.ctypes.data_as(C.POINTER(C.c_double)) if omega_diag is not None else None
    _check(_lib.hg_problem_create_dense(ctx, dim, n_ctrl, C.byref(H0), arr, om, C.byref(out)),
           "hg_problem_create_dense")
    return out.value


def hg_problem_destroy(p: int) -> None:
    _check(_lib.hg_problem_destroy(p), "hg_problem_destroy")


def hg_problem_info(p: int) -> dict:
    dim, k, w, s, nnz = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
    _check(_lib.hg_problem_info(p, C.byref(dim), C.byref(k), C.byref(w), C.byref(s),
                                C.byref(nnz)), "hg_problem_info")
    return {"dim": dim.value, "n_ctrl": k.value, "ell_width": w.value, "sigma": s.value,
            "nnz": nnz.value}


def hg_plan(theta, sigma: int, tau: float, u: float):
    """theta: float64 numpy array (host).  Returns (m, s) int32 numpy arrays."""
    import numpy as np
    th = np.ascontiguousarray(theta, dtype=np.float64)
    m = np.zeros(th.shape, dtype=np.int32)
    s = np.zeros(th.shape, dtype=np.int32)
    _check(_lib.hg_plan(th.ctypes.data_as(C.POINTER(C.c_double)), th.size, sigma, tau, u,
                        m.ctypes.data_as(C.POINTER(C.c_int32)),
                        s.ctypes.data_as(C.POINTER(C.c_int32))), "hg_plan")
    return m, s


def hg_plan_rule(theta, sigma: int, tau: float, u: float, rule: int):
    import numpy as np
    th = np.ascontiguousarray(theta, dtype=np.float64)
    m = np.zeros(th.size, dtype=np.int32)
    s = np.zeros(th.size, dtype=np.int32)
    _check(_lib.hg_plan_rule(th.ctypes.data_as(C.POINTER(C.c_double)), th.size, sigma, tau, u,
                             rule, m.ctypes.data_as(C.POINTER(C.c_int32)),
                             s.ctypes.data_as(C.POINTER(C.c_int32))), "hg_plan_rule")
    return m, s


def hg_error_bound(theta: float, m: int, s: int, sigma: int, u: float) -> float:
    return float(_lib.hg_error_bound(theta, m, s, sigma, u))


def hg_step_norms(p: int, u_ptr: int, n_batch: int, n_steps: int, dt: float, theta_ptr: int,
                  stream: int) -> None:
    _check(_lib.hg_step_norms(p, u_ptr, n_batch, n_steps, dt, theta_ptr, stream),
           "hg_step_norms")


def hg_eval(p: int, desc: hg_eval_desc, results, grad_ptr, stream: int) -> None:
    _check(_lib.hg_eval(p, C.byref(desc), results, grad_ptr, stream), "hg_eval")


def hg_eval_noalloc(p: int, desc: hg_eval_desc, results, grad_ptr, stream: int) -> None:
    _check(_lib.hg_eval_noalloc(p, C.byref(desc), results, grad_ptr, stream), "hg_eval_noalloc")


def hg_eval_noalloc_limits():
    a, b = C.c_size_t(), C.c_size_t()
    _check(_lib.hg_eval_noalloc_limits(C.byref(a), C.byref(b)), "hg_eval_noalloc_limits")
    return int(a.value), int(b.value)


def hg_eval_footprint(p: int, desc: hg_eval_desc) -> int:
    out = C.c_size_t()
    _check(_lib.hg_eval_footprint(p, C.byref(desc), C.byref(out)), "hg_eval_footprint")
    return int(out.value)


def hg_server_create(ctx: int, hbm_budget_bytes: int, max_inflight: int) -> int:
    out = C.c_void_p()
    _check(_lib.hg_server_create(ctx, hbm_budget_bytes, max_inflight, C.byref(out)),
           "hg_server_create")
    return out.value


def hg_server_submit(sv: int, p: int, desc: hg_eval_desc, results, grad_ptr,
                     after_stream) -> int:
    rid = C.c_uint64()
    _check(_lib.hg_server_submit(sv, p, C.byref(desc), results, grad_ptr, after_stream,
                                 C.byref(rid)), "hg_server_submit")
    return int(rid.value)


def hg_mem_pool_peak(ctx: int, reset: bool = False) -> int:
    out = C.c_size_t()
    _check(_lib.hg_mem_pool_peak(ctx, 1 if reset else 0, C.byref(out)), "hg_mem_pool_peak")
    return int(out.value)


def hg_server_poll(sv: int, req_id: int) -> bool:
    done = C.c_int32()
    _check(_lib.hg_server_poll(sv, req_id, C.byref(done)), "hg_server_poll")
    return bool(done.value)


def hg_server_wait(sv: int, req_id: int):
    """Returns (status, latency_ms, queued_ms); the status is not raised."""
    lat, q = C.c_double(), C.c_double()
    st = _lib.hg_server_wait(sv, req_id, C.byref(lat), C.byref(q))
    return int(st), float(lat.value), float(q.value)


def hg_server_cancel(sv: int, req_id: int) -> None:
    _check(_lib.hg_server_cancel(sv, req_id), "hg_server_cancel")


def hg_server_info(sv: int):
    b, q, r = C.c_size_t(), C.c_int32(), C.c_int32()
    _check(_lib.hg_server_info(sv, C.byref(b), C.byref(q), C.byref(r)), "hg_server_info")
    return int(b.value), int(q.value), int(r.value)


def hg_server_destroy(sv: int) -> None:
    _check(_lib.hg_server_destroy(sv), "hg_server_destroy")

"""Shared helpers of the GPU tests: build the library objects from a workload
and compare with oracle values (tolerances of the parity bar)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")

# parity bar: relative error on cost and on the gradient (2-norm), and the
# elementwise gradient bound relative to the largest entry
TOL = {"c128": 1e-10, "c64": 1e-4}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


_ctx = None


def context():
    global _ctx
    import paper_2304_06200_amd as hg
    if _ctx is None:
        _ctx = hg.Context(0)
    return _ctx


def device_inputs(p, batch_u=None):
    import torch
    u = torch.tensor(p.u if batch_u is None else batch_u, dtype=torch.float64, device="cuda")
    psi0 = torch.tensor(p.psi0, dtype=torch.complex128, device="cuda")
    tg = torch.tensor(p.targets, dtype=torch.complex128, device="cuda")
    return u, psi0, tg


def make_problem(p):
    import paper_2304_06200_amd as hg
    return hg.Problem(context(), p.H0, p.Hk, p.omega)


def run(p, dtype="c128", prob=None, schedule=None, batch_u=None, **kw):
    import paper_2304_06200_amd as hg
    prob = prob or make_problem(p)
    u, psi0, tg = device_inputs(p, batch_u)
    return hg.evaluate(prob, u, psi0, tg, p.dt, w_fid=kw.pop("w_fid", p.w_fid),
                       w_pen=kw.pop("w_pen", p.w_pen), tau=kw.pop("tau", p.tau), dtype=dtype,
                       schedule=schedule, **kw)


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def assert_parity(res, ref, dtype, b=0, label=""):
    """Cost, infidelity, penalty and gradient of batch entry b against the oracle."""
    tol = TOL[dtype]
    g = res.grad[b].cpu().numpy()
    gr = np.asarray(ref["grad"])
    ec = rel(res.cost[b], float(ref["cost"]))
    # a gradient that vanishes exactly (e.g. an eigenstate with nothing to
    # steer) is compared in absolute terms
    scale2 = max(np.linalg.norm(gr), 1.0 if np.linalg.norm(gr) == 0 else 0.0)
    scalem = max(np.max(np.abs(gr)), 1.0 if np.max(np.abs(gr)) == 0 else 0.0)
    eg = np.linalg.norm(g - gr) / scale2
    emax = np.max(np.abs(g - gr)) / scalem
    log(f"[parity] {label} {dtype}: cost {res.cost[b]:.15g} ref {float(ref['cost']):.15g} "
        f"rel {ec:.2e}; grad rel {eg:.2e} max {emax:.2e}; sum_mu {res.sum_mu[b]}")
    assert ec <= tol, f"cost rel err {ec:.3e} > {tol}"
    assert eg <= tol, f"grad rel err {eg:.3e} > {tol}"
    assert emax <= tol, f"grad max err {emax:.3e} > {tol}"
    if "infidelity" in ref:
        assert abs(res.infidelity[b] - float(ref["infidelity"])) <= tol * max(1.0, abs(float(ref["infidelity"])))
        assert abs(res.penalty[b] - float(ref["penalty"])) <= tol * max(1.0, abs(float(ref["penalty"])))


def oracle_schedule(p, tau=None):
    """(m, s) per step from the oracle planner on oracle norms (never from the GPU)."""
    from oracle import planner
    import scipy.sparse as sp
    pat = abs(p.H0)
    for h in p.Hk:
        pat = pat + abs(h)
    sigma = int(np.max(np.diff(sp.csr_matrix(pat).indptr)))
    ms = np.zeros((2, p.n_steps), dtype=np.int32)
    for n in range(p.n_steps):
        H = p.H0 + sum(p.u[k, n] * p.Hk[k] for k in range(p.n_ctrl))
        theta = float(np.max(np.asarray(abs(-1j * p.dt * H).sum(axis=0))))
        ms[:, n] = planner.select(theta, sigma, tau or p.tau)
    return ms


def golden(name):
    path = os.path.join(GOLDEN, f"{name}_oracle.npz")
    if not os.path.exists(path):
        return None
    z = np.load(path, allow_pickle=False)
    return {k: z[k] for k in z.files}

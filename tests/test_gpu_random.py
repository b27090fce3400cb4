"""Seeded random problems against the exact oracle: random banded Hermitian
drifts and controls (union patterns of 1 to 13 diagonals, controls with up to
4), random sizes, state counts and step counts, both precisions and both
backward variants.  Covers pattern widths the named workloads do not reach."""
import numpy as np
import pytest
import scipy.sparse as sp

from gpu_common import assert_parity, log, run
from workloads.circuits import Problem

pytestmark = pytest.mark.gpu


def _herm_band(rng, d, offsets, scale):
    """Hermitian matrix with random entries on the diagonals +-offsets (0 = main)."""
    m = sp.lil_matrix((d, d), dtype=np.complex128)
    for o in offsets:
        if o == 0:
            m.setdiag(rng.uniform(-1, 1, d) * scale)
        elif o < d:
            v = (rng.standard_normal(d - o) + 1j * rng.standard_normal(d - o)) * scale / 2
            m.setdiag(v, o)
            m.setdiag(np.conj(v), -o)
    out = sp.csr_matrix(m)
    out.eliminate_zeros()
    return out


def _random_problem(seed):
    rng = np.random.default_rng(1000 + seed)
    d = int(rng.integers(2, 300))
    n_off = seed % 7                                     # 0..6 +- pairs: 1 to 13 diagonals
    pool = rng.permutation(np.arange(1, max(d, 2)))[:n_off]
    union = [0] + [int(o) for o in pool]
    K = int(rng.integers(0, 5))
    H0 = _herm_band(rng, d, union, 1.0)
    Hk = []
    for _ in range(K):
        own = [int(o) for o in rng.choice(union[1:], size=min(2, len(union) - 1), replace=False)] \
            if len(union) > 1 else [0]
        Hk.append(_herm_band(rng, d, own, 0.5))
    S = int(rng.integers(1, min(d, 6) + 1))
    N = int(rng.integers(1, 15))
    dt = float(rng.uniform(0.1, 0.6))
    u = rng.uniform(-1, 1, (K, N))
    q, _ = np.linalg.qr(rng.standard_normal((d, S)) + 1j * rng.standard_normal((d, S)))
    psi0 = q.T.copy()
    q2, _ = np.linalg.qr(rng.standard_normal((d, S)) + 1j * rng.standard_normal((d, S)))
    targets = q2.T.copy()
    om = (rng.uniform(size=d) < 0.3).astype(float) if rng.uniform() < 0.6 else None
    w_pen = float(rng.uniform(0.2, 1.0)) if om is not None else 0.0
    return Problem(f"rand{seed}", H0, Hk, dt, u, psi0, targets, om, w_fid=1.0, w_pen=w_pen)


@pytest.mark.parametrize("seed", range(12))
def test_random_problem(seed):
    from oracle import grape
    p = _random_problem(seed)
    w_int = 0.5 if seed % 3 == 0 else 0.0
    ref = grape.cost_and_grad(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets, omega=p.omega,
                              w_fid=p.w_fid, w_pen=p.w_pen, w_int=w_int)
    pattern = sp.csr_matrix(abs(p.H0) + sum(abs(h) for h in p.Hk)) if p.Hk else abs(p.H0)
    coo = sp.coo_matrix(pattern)
    W = len(set((coo.col - coo.row).tolist())) if coo.nnz else 1
    mode = "checkpoint" if seed % 2 else "reconstruct"
    log(f"[case] random seed={seed}: d={p.dim} K={p.n_ctrl} S={p.n_states} N={p.n_steps} "
        f"W={W} penalty={p.omega is not None} w_int={w_int} {mode}")
    kw = dict(mode=mode, ckpt_every=3) if mode == "checkpoint" else {}
    for dtype in ("c128", "c64"):
        r = run(p, dtype, w_int=w_int, **kw)
        if p.n_ctrl == 0:
            assert r.grad is None
            assert abs(r.cost[0] - ref["cost"]) <= (1e-10 if dtype == "c128" else 1e-4) * max(1, abs(ref["cost"]))
            continue
        assert_parity(r, ref, dtype, label=f"rand{seed}")

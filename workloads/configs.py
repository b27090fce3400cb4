"""The five benchmark workloads of the HG-GRAPE cost+gradient path (inputs only).

cfg1  single transmon, 4 levels, state transfer |0> -> |1>, N=200, dt=0.1 ns
cfg2  transmon(3) x cavity(20), d=60, 4 controls, N=1000, dt=1 ns, 4-state
      Haar target on the computational subspace, forbidden-level penalty
cfg3  transmon(4) x transmon(4) x cavity(100), d=1600, 6 controls, N=2000,
      dt=0.5 ns, 16 initial states (2-qubit basis x Fock 0..3), Haar target
cfg4  serving stream: transmon(3) x cavity(8..700), N in [200,2000], S in [1,8]
cfg5  transmon(8) x cavity(1024), d=8192, 4 controls, N=5000, dt=0.2 ns, S=4

Amplitudes are u = 2*pi*U[-0.05, 0.05] rad/ns from numpy's PCG64 with a fixed
seed per config.  Targets are phi_T^h = sum_j (U_T)_{jh} psi_0^j for a
Haar-random U_T on the span of the initial states (coherent subspace gate).
The penalty operator Omega is the diagonal 0/1 projector onto the top level of
every mode (the truncation edge), the forbidden-level occupation of the
paper's transmon-cavity benchmark.
"""
from __future__ import annotations

from typing import Dict, List, Optional

import numpy as np

from .circuits import (Problem, basis_state, haar_unitary, three_transmon_chain,
                       transmon_cavity_system,
                       two_transmon_cavity_system)

TWO_PI = 2.0 * np.pi
AMP = 0.05  # GHz; amplitudes are 2*pi*U[-AMP, AMP] rad/ns


def _amps(rng: np.random.Generator, K: int, N: int) -> np.ndarray:
    return TWO_PI * rng.uniform(-AMP, AMP, size=(K, N))


def _top_level_projector(dims) -> np.ndarray:
    """Diagonal of the projector onto 'any mode in its top level'."""
    idx = np.indices(dims).reshape(len(dims), -1)
    mask = np.zeros(idx.shape[1], dtype=bool)
    for j, d in enumerate(dims):
        mask |= idx[j] == d - 1
    return mask.astype(np.float64)


def _targets_from(psi0: np.ndarray, UT: np.ndarray) -> np.ndarray:
    # phi^h = sum_j UT[j, h] psi0^j   (rows are states)
    return UT.T @ psi0


def cfg1(N: int = 200, seed: int = 1) -> Problem:
    d = 4
    from .circuits import destroy, number
    import scipy.sparse as sp
    a = destroy(d)
    n = number(d)
    alpha = -TWO_PI * 0.225
    H0 = sp.csr_matrix(0.5 * alpha * (n @ (n - sp.identity(d, format="csr"))))
    H0.eliminate_zeros()
    hx = sp.csr_matrix(a + a.conj().T)
    hy = sp.csr_matrix(1j * (a.conj().T - a))
    for h in (hx, hy):
        h.eliminate_zeros()
        h.sort_indices()
    u = _amps(np.random.default_rng(seed), 2, 200)[:, :N]
    psi0 = basis_state(d, 0)[None, :]
    tgt = basis_state(d, 1)[None, :]
    return Problem("cfg1_transmon4", H0, [hx, hy], 0.1, u, psi0, tgt, None,
                   w_fid=1.0, w_pen=0.0, dims=(d,))


def cfg2(N: int = 1000, seed: int = 2, d_c: int = 20) -> Problem:
    d_t = 3
    H0, Hk, dims = transmon_cavity_system(d_t, d_c, -TWO_PI * 0.2, -TWO_PI * 0.002)
    d = d_t * d_c
    u = _amps(np.random.default_rng(seed), 4, 1000)[:, :N]
    idx = [t * d_c + c for t in (0, 1) for c in (0, 1)]
    psi0 = np.stack([basis_state(d, i) for i in idx])
    UT = haar_unitary(4, np.random.default_rng(1000 + seed))
    return Problem(f"cfg2_t3c{d_c}", H0, Hk, 1.0, u, psi0, _targets_from(psi0, UT),
                   _top_level_projector(dims), w_fid=1.0, w_pen=1.0, dims=dims)


def cfg3(N: int = 2000, seed: int = 3, d_c: int = 100, n_states: int = 16) -> Problem:
    d_t = 4
    H0, Hk, dims = two_transmon_cavity_system(d_t, d_c, -TWO_PI * 0.2, -TWO_PI * 0.002,
                                              TWO_PI * 0.005)
    d = d_t * d_t * d_c
    u = _amps(np.random.default_rng(seed), 6, 2000)[:, :N]
    idx = [(t1 * d_t + t2) * d_c + c for t1 in (0, 1) for t2 in (0, 1) for c in range(4)]
    idx = idx[:n_states]
    psi0 = np.stack([basis_state(d, i) for i in idx])
    UT = haar_unitary(len(idx), np.random.default_rng(1000 + seed))
    return Problem(f"cfg3_t4t4c{d_c}", H0, Hk, 0.5, u, psi0, _targets_from(psi0, UT),
                   _top_level_projector(dims), w_fid=1.0, w_pen=1.0, dims=dims)


def cfg5(N: int = 5000, seed: int = 5, d_c: int = 1024) -> Problem:
    d_t = 8
    H0, Hk, dims = transmon_cavity_system(d_t, d_c, -TWO_PI * 0.2, -TWO_PI * 0.002)
    d = d_t * d_c
    u = _amps(np.random.default_rng(seed), 4, 5000)[:, :N]
    idx = [t * d_c + c for t in (0, 1) for c in (0, 1)]
    psi0 = np.stack([basis_state(d, i) for i in idx])
    UT = haar_unitary(4, np.random.default_rng(1000 + seed))
    return Problem(f"cfg5_t8c{d_c}", H0, Hk, 0.2, u, psi0, _targets_from(psi0, UT),
                   _top_level_projector(dims), w_fid=1.0, w_pen=1.0, dims=dims)


def gate3(d_t: int = 4, N: int = 1, dt: float = 0.25, seed: int = 6,
          random_amps: bool = False) -> Problem:
    """Full-basis gate on three coupled transmons (Sec. IV.B, eq. gateH):
    alpha/2pi = -0.225 GHz, g/2pi = 0.1 GHz, drive amplitudes a/2pi = 0.1 GHz
    (constant, as in the paper's single-step benchmark, or seeded uniform in
    +-0.1 GHz with random_amps).  S = d initial states (the full product basis);
    target U_T = simultaneous Hadamards, each acting on levels {0, 1} of its
    transmon and as the identity on the levels above (reading for d_t > 2).
    dt = 0.25 ns (not stated for this benchmark): ||A||_1 grows as d_t^2 through
    the anharmonicity, and at d_t = 8 a longer step puts tau = 1e-12 below the
    floor of the App. C bound."""
    H0, Hk, dims = three_transmon_chain(d_t, -TWO_PI * 0.225, TWO_PI * 0.1)
    d = d_t ** 3
    if random_amps:
        u = TWO_PI * 0.1 * np.random.default_rng(seed).uniform(-1.0, 1.0, (3, N))
    else:
        u = np.full((3, N), TWO_PI * 0.1)
    h1 = np.eye(d_t, dtype=np.complex128)
    h1[:2, :2] = np.array([[1, 1], [1, -1]]) / np.sqrt(2)
    UT = np.kron(np.kron(h1, h1), h1)
    psi0 = np.eye(d, dtype=np.complex128)
    targets = (UT @ psi0.T).T.copy()
    return Problem(f"gate3_t{d_t}", H0, Hk, dt, u, psi0, targets, None, w_fid=1.0, w_pen=0.0,
                   dims=dims)


def serving_request(i: int, d_c: int, N: int, S: int) -> Problem:
    """One request of the serving stream: transmon(3) x cavity(d_c), dt = 1 ns."""
    d_t = 3
    H0, Hk, dims = transmon_cavity_system(d_t, d_c, -TWO_PI * 0.2, -TWO_PI * 0.002)
    d = d_t * d_c
    u = _amps(np.random.default_rng(40_000 + i), 4, N)
    order = [t * d_c + c for c in range(4) for t in range(2)]
    psi0 = np.stack([basis_state(d, j) for j in order[:S]])
    UT = haar_unitary(S, np.random.default_rng(50_000 + i))
    return Problem(f"cfg4_req{i}_c{d_c}_N{N}_S{S}", H0, Hk, 1.0, u, psi0,
                   _targets_from(psi0, UT), _top_level_projector(dims),
                   w_fid=1.0, w_pen=1.0, tau=1e-10, dims=dims, meta={"request": i})


def serving_stream(n_req: int = 256, seed: int = 4, d_c_max: int = 700,
                   n_max: int = 2000) -> List[Dict]:
    """Request shapes of the serving workload: d_c log-uniform in [8, d_c_max],
    N uniform in [200, n_max], S uniform in [1, 8].  Returns a list of dicts
    (index, d_c, N, S); build each request with ``serving_request``."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_req):
        d_c = int(round(np.exp(rng.uniform(np.log(8.0), np.log(float(d_c_max))))))
        N = int(rng.integers(200, n_max + 1))
        S = int(rng.integers(1, 9))
        out.append({"index": i, "d_c": d_c, "N": N, "S": S})
    return out


CONFIGS = {"cfg1": cfg1, "cfg2": cfg2, "cfg3": cfg3, "cfg5": cfg5, "gate3": gate3}


def make_config(name: str, **kw) -> Problem:
    return CONFIGS[name](**kw)


def problem_summary(p: Problem) -> Dict:
    import scipy.sparse as sp
    pattern = abs(p.H0)
    for h in p.Hk:
        pattern = pattern + abs(h)
    pattern = sp.csr_matrix(pattern)
    row_nnz = np.diff(pattern.indptr)
    return {"name": p.name, "dim": p.dim, "n_ctrl": p.n_ctrl, "n_steps": p.n_steps,
            "n_states": p.n_states, "dt": p.dt, "nnz_union": int(pattern.nnz),
            "sigma_max": int(row_nnz.max())}

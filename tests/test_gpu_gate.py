"""Full-basis gate optimisation on three coupled transmons (Sec. IV.B, eq.
gateH): S = d initial states (the product basis), target simultaneous
Hadamards, gate infidelity 1 - |tr(U_T^dag U)/d|^2 and its gradient against
the exact oracle.  Eleven union diagonals, so the 13-wide kernels run."""
import numpy as np
import pytest

from gpu_common import assert_parity, log, run
from workloads import make_config

pytestmark = pytest.mark.gpu


def _oracle(p):
    from oracle import grape
    return grape.cost_and_grad(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets)


@pytest.mark.parametrize("d_t,N,random_amps", [(3, 1, False), (4, 10, True), (6, 1, False)])
def test_gate3_full_basis(d_t, N, random_amps):
    p = make_config("gate3", d_t=d_t, N=N, random_amps=random_amps)
    ref = _oracle(p)
    log(f"[case] gate3 d_t={d_t} d={p.dim} S={p.n_states} N={N}")
    for dtype in ("c128", "c64"):
        r = run(p, dtype)
        assert_parity(r, ref, dtype, label=f"gate3-t{d_t}")


def test_gate3_cost_is_gate_infidelity():
    """The GPU overlap g equals tr(U_T^dag U)/d built from the oracle's propagator."""
    from oracle import grape
    p = make_config("gate3", d_t=3, N=3, random_amps=True)
    r = run(p, "c128")
    U = np.eye(p.dim, dtype=np.complex128)
    for n in range(p.n_steps):
        U = grape.propagator(grape.hamiltonian(grape._dense(p.H0), [grape._dense(h) for h in p.Hk],
                                               p.u[:, n]), p.dt) @ U
    UT = p.targets.T            # columns U_T e_h (psi0 = identity)
    g = np.trace(UT.conj().T @ U) / p.dim
    log(f"[case] gate3 overlap {r.overlap[0]:.15g} vs tr/d {g:.15g}")
    assert abs(r.overlap[0] - g) <= 1e-12

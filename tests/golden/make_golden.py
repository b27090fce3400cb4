"""Write oracle-computed expected values for the parity tests.

Calls only the FP64 oracle (oracle/grape.py) on inputs from workloads/.  Each
output is an .npz (no pickles) holding cost, infidelity, penalty, overlap and
the full gradient, plus the generating config name and sizes.

    python tests/golden/make_golden.py cfg1 cfg2            # seconds
    python tests/golden/make_golden.py cfg3 --threads 4     # several hours on 4 cores
    python tests/golden/make_golden.py cfg5:d_c=256 --discrete --threads 2   # ~10 min

The cfg3 file is the full-size d=1600, N=2000, S=16 oracle evaluation that the
GPU parity test compares against; it is too slow to recompute inside a test.

`--discrete` evaluates the Taylor-discretised problem instead (oracle/taylor.py,
sparse products, states stored, no reconstruction) with the (m, s) schedule of
the oracle planner at the config's tolerance; the schedule is saved with the
result.  A config name may carry keyword overrides: `cfg5:d_c=256,N=500`.
"""
import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("configs", nargs="+")
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--discrete", action="store_true")
    args = ap.parse_args()
    if args.threads:
        for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            os.environ[v] = str(args.threads)
    sys.path.insert(0, ROOT)
    import numpy as np
    from oracle import grape
    from workloads import make_config

    from oracle import planner, taylor

    for spec in args.configs:
        name, _, opts = spec.partition(":")
        kw = {k: int(v) for k, v in (o.split("=") for o in opts.split(",") if o)}
        p = make_config(name, **kw)
        t0 = time.time()
        extra = {}
        if args.discrete:
            # sigma' of the union pattern, exact column sums of |A_n| (sparse)
            pattern = abs(p.H0) + sum(abs(h) for h in p.Hk)
            sigma = int(np.max(np.diff(pattern.tocsr().indptr)))
            sched = np.zeros((2, p.n_steps), dtype=np.int32)
            for n in range(p.n_steps):
                A = -1j * p.dt * (p.H0 + sum(p.u[k, n] * p.Hk[k] for k in range(p.n_ctrl)))
                theta = float(np.max(np.asarray(abs(A).sum(axis=0))))
                sched[:, n] = planner.select(theta, sigma, p.tau)
            r = taylor.hg_discrete(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets, sched,
                                   omega=p.omega, w_fid=p.w_fid, w_pen=p.w_pen)
            final = np.asarray(r["final_states"])
            extra = {"schedule": sched}
            tag = p.name + "_discrete"
        else:
            r = grape.cost_and_grad(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets, omega=p.omega,
                                    w_fid=p.w_fid, w_pen=p.w_pen, want_states=True)
            final = r.pop("states")[-1].T.copy()      # psi_N^h as rows (S, d)
            tag = name
        el = time.time() - t0
        out = os.path.join(HERE, f"{tag}_oracle.npz")
        np.savez(out, cost=r["cost"], infidelity=r["infidelity"], penalty=r["penalty"],
                 overlap=np.array([r["overlap"].real, r["overlap"].imag]), grad=r["grad"],
                 final_states=final, name=p.name, dim=p.dim, n_steps=p.n_steps, n_states=p.n_states,
                 seconds=el, **extra)
        print(f"{name}: cost={r['cost']:.15g} |grad|={np.linalg.norm(r['grad']):.6g} "
              f"({el:.1f} s) -> {out}", flush=True)


if __name__ == "__main__":
    main()

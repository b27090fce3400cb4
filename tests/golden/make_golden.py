"""Write oracle-computed expected values for the parity tests.

Calls only the FP64 oracle (oracle/grape.py) on inputs from workloads/.  Each
output is an .npz (no pickles) holding cost, infidelity, penalty, overlap and
the full gradient, plus the generating config name and sizes.

    python tests/golden/make_golden.py cfg1 cfg2            # seconds
    python tests/golden/make_golden.py cfg3 --threads 4     # ~1.5-3 h on 4-8 cores

The cfg3 file is the full-size d=1600, N=2000, S=16 oracle evaluation that the
GPU parity test compares against; it is too slow to recompute inside a test.
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
    args = ap.parse_args()
    if args.threads:
        for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            os.environ[v] = str(args.threads)
    sys.path.insert(0, ROOT)
    import numpy as np
    from oracle import grape
    from workloads import make_config

    for name in args.configs:
        p = make_config(name)
        t0 = time.time()
        r = grape.cost_and_grad(p.H0, p.Hk, p.u, p.dt, p.psi0, p.targets, omega=p.omega,
                                w_fid=p.w_fid, w_pen=p.w_pen, want_states=True)
        final = r.pop("states")[-1].T.copy()      # psi_N^h as rows (S, d)
        el = time.time() - t0
        out = os.path.join(HERE, f"{name}_oracle.npz")
        np.savez(out, cost=r["cost"], infidelity=r["infidelity"], penalty=r["penalty"],
                 overlap=np.array([r["overlap"].real, r["overlap"].imag]), grad=r["grad"],
                 final_states=final, name=p.name, dim=p.dim, n_steps=p.n_steps, n_states=p.n_states,
                 seconds=el)
        print(f"{name}: cost={r['cost']:.15g} |grad|={np.linalg.norm(r['grad']):.6g} "
              f"({el:.1f} s) -> {out}", flush=True)


if __name__ == "__main__":
    main()

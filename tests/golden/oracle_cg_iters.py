"""Writes tests/golden/oracle_cgnr_iters_<config>.json: the number of iterations the
oracle's CG on Omega^dag Omega (the paper's fallback solver, Sec. IV) needs to reach the
true relative residual 1e-10 on the seeded Gaussian source of the workload (seed 123).
The CPU baseline of the benchmark times a few of these iterations and scales by this
count.  Calls only the oracle.

    OMP_NUM_THREADS=6 python tests/golden/oracle_cg_iters.py ns24_nt128
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def main(name):
    cfg = synth.CONFIGS[name]
    U = synth.gauge_field(cfg.ns, cfg.nt, cfg.eps, cfg.seed)
    eta = synth.random_spinor(cfg.ns, cfg.nt, 123)
    D = oracle.Dirac(U, cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    t0 = time.time()
    x, it, tr = D.solve(eta, tol=1e-10, maxiter=20000)
    rec = {"config": name, "m0": cfg.m0, "source": "Gaussian spinor, seed 123", "iterations": abs(it),
           "converged": it > 0, "true_resid": tr, "seconds": round(time.time() - t0, 1),
           "threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))}
    with open(os.path.join(ROOT, "tests", "golden", "oracle_cgnr_iters_%s.json" % name), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "ns24_nt128")

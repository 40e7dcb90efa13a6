"""Writes tests/golden/oracle_cgnr_iters_<config>[_laph].json: the number of iterations the
oracle's CG on Omega^dag Omega (the paper's fallback solver, Sec. IV) needs to reach the
true relative residual 1e-10 on the seeded Gaussian source of the workload (seed 123),
or with `laph` on the workload's first LapH source: projector b = 0 of its dilution
scheme applied to the Z4 noise (s, k) of the workload, V_s P^(0) rho (Sec. II), with the
oracle's own eigenvectors of the stout-smeared Laplacian on the source's time slice.
The CPU baseline of the benchmark times a few of these iterations and scales by this
count.  Calls only the oracle.

    OMP_NUM_THREADS=6 python tests/golden/oracle_cg_iters.py ns24_nt128 [laph]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def laph_source(cfg, U):
    """V_s P^(0) rho: with time dilution, projector 0 lives on the slices of b_T = 0 only;
    slice 0 belongs to it for every scheme of the workloads, and its eigenvectors are the
    only ones computed (other slices of the source are checked to be zero)."""
    import numpy as np

    S = oracle.stout_spatial(U, cfg.stout_rho, cfg.stout_steps)
    sch = oracle.parse_dilution(cfg.dilution, cfg.nt, cfg.nv)
    P = oracle.dilution_projector(sch, cfg.nt, cfg.nv, 0)
    slices = [t for t in range(cfg.nt) if P[t].any()]
    ev, V0 = oracle.laph_eigpairs(S, cfg.nv, slices=slices)
    V = np.zeros((cfg.nt, cfg.nv, cfg.ns, cfg.ns, cfg.ns, 3), dtype=np.complex128)
    V[slices] = V0
    rho = oracle.z4_noise(cfg.noise_s, cfg.noise_k, cfg.nt, cfg.nv)
    return oracle.source(V, rho, sch, 0), slices


def main(name, kind="gauss"):
    cfg = synth.CONFIGS[name]
    U = synth.gauge_field(cfg.ns, cfg.nt, cfg.eps, cfg.seed)
    if kind == "laph":
        eta, slices = laph_source(cfg, U)
        what = "LapH source b = 0 of (%s), noise (%d, %d), eigenvectors of slices %s" % (
            cfg.dilution, cfg.noise_s, cfg.noise_k, slices)
    else:
        eta = synth.random_spinor(cfg.ns, cfg.nt, 123)
        what = "Gaussian spinor, seed 123"
    D = oracle.Dirac(U, cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    t0 = time.time()
    x, it, tr = D.solve(eta, tol=1e-10, maxiter=20000)
    rec = {"config": name, "m0": cfg.m0, "source": what, "iterations": abs(it),
           "converged": it > 0, "true_resid": tr, "seconds": round(time.time() - t0, 1),
           "threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))}
    suffix = "_laph" if kind == "laph" else ""
    with open(os.path.join(ROOT, "tests", "golden", "oracle_cgnr_iters_%s%s.json" % (name, suffix)), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "ns24_nt128", sys.argv[2] if len(sys.argv) > 2 else "gauss")

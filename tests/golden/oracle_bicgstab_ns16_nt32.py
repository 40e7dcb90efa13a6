"""Writes tests/golden/oracle_bicgstab_ns16_nt32.json: the oracle's plain BiCGStab (the
paper's solver, Sec. IV) at the mass of the large workloads (m0 = -0.12) on the 16^3 x 32
field, on the even-odd system and on the full K x = gamma_4 eta, from the workload's first
LapH source (projector b = 0 of (TI16,SF,LI8) on the Z4 noise, oracle eigenvectors of the
slices it touches) and from a Gaussian source.  It records whether the iterated residual
reached 1e-10, the iteration count, the smallest residual seen and the history (every
tenth iteration), beside the oracle CG on the normal equations for the same sources.
Calls only the oracle.

    OMP_NUM_THREADS=6 python tests/golden/oracle_bicgstab_ns16_nt32.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

MAXITER = 1500


def laph_source(cfg, U):
    S = oracle.stout_spatial(U, cfg.stout_rho, cfg.stout_steps)
    sch = oracle.parse_dilution(cfg.dilution, cfg.nt, cfg.nv)
    P = oracle.dilution_projector(sch, cfg.nt, cfg.nv, 0)
    slices = [t for t in range(cfg.nt) if P[t].any()]
    ev, V0 = oracle.laph_eigpairs(S, cfg.nv, slices=slices)
    V = np.zeros((cfg.nt, cfg.nv, cfg.ns, cfg.ns, cfg.ns, 3), dtype=np.complex128)
    V[slices] = V0
    rho = oracle.z4_noise(cfg.noise_s, cfg.noise_k, cfg.nt, cfg.nv)
    return oracle.source(V, rho, sch, 0), slices


def main():
    cfg = synth.CONFIGS["ns16_nt32"]
    U = synth.gauge_field(cfg.ns, cfg.nt, cfg.eps, cfg.seed)
    D = oracle.Dirac(U, cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    eta_l, slices = laph_source(cfg, U)
    sources = {"laph_b0": eta_l, "gauss_seed123": synth.random_spinor(cfg.ns, cfg.nt, 123)}
    out = {"config": cfg.name, "m0": cfg.m0, "tol": 1e-10, "maxiter": MAXITER,
           "laph_source": "projector b = 0 of (%s), noise (%d, %d), oracle eigenvectors of slices %s" % (
               cfg.dilution, cfg.noise_s, cfg.noise_k, slices), "runs": []}
    for name, eta in sources.items():
        t0 = time.time()
        x, it, tr = D.solve(eta, tol=1e-10, maxiter=20000)
        out["runs"].append({"source": name, "solver": "cgnr (full system)", "iterations": int(it),
                            "true_resid": float(tr), "seconds": round(time.time() - t0, 1)})
        print(out["runs"][-1], flush=True)
        for eo in (True, False):
            t0 = time.time()
            x, k, hist, tr = oracle.bicgstab_solve(D, eta, tol=1e-10, maxiter=MAXITER, even_odd=eo)
            h = np.array(hist)
            rec = {"source": name, "solver": "bicgstab (%s)" % ("even-odd" if eo else "full K"),
                   "converged": bool(k > 0), "iterations": int(abs(k)), "min_resid": float(h.min()),
                   "min_at": int(h.argmin()), "final_resid": float(h[-1]), "true_resid": float(tr),
                   "history_every_10": [float(v) for v in h[::10]], "seconds": round(time.time() - t0, 1)}
            out["runs"].append(rec)
            print({k2: v for k2, v in rec.items() if k2 != "history_every_10"}, flush=True)
    out["threads"] = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))
    with open(os.path.join(ROOT, "tests", "golden", "oracle_bicgstab_ns16_nt32.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()

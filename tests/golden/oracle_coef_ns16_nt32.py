"""Writes tests/golden/oracle_coef_ns16_nt32.json: LapH sink coefficients of eight diluted
sources of the 16^3 x 32 workload (Sec. II: eta = V_s P^(b) rho with (TI16,SF,LI8)
dilution; Sec. IV: the coefficients V_s^dag Omega^-1 eta), computed by the oracle alone:
its stout smearing, its ARPACK eigenvectors of the slices the comparison uses (0, 5, 16,
21: the time-interlaced sources b_T = 0 and 5 live on {0, 16} and {5, 21}), its Z4 noise
and its CG on the normal equations solved to a true relative residual of 1e-12.

The GPU test recomputes the same oracle eigenvectors (ARPACK is deterministic here: two
runs at 1 and 8 BLAS threads agree to 3e-17, and the smallest eigenvalue gap below the
cut is 1.3e-4), hands them to the library and compares its coefficients on these slices.

    OMP_NUM_THREADS=6 python tests/golden/oracle_coef_ns16_nt32.py
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

SLICES = [0, 5, 16, 21]
SOURCES = [28, 29, 30, 31, 160, 161, 162, 163]  # b = (b_T * 4 + b_S) * 8 + b_L
TOL = 1e-12


def oracle_basis(cfg, U):
    """eigenvectors of the stout-smeared Laplacian on SLICES, zero elsewhere"""
    S = oracle.stout_spatial(U, cfg.stout_rho, cfg.stout_steps)
    ev, V0 = oracle.laph_eigpairs(S, cfg.nv, slices=SLICES)
    V = np.zeros((cfg.nt, cfg.nv, cfg.ns, cfg.ns, cfg.ns, 3), dtype=np.complex128)
    V[SLICES] = V0
    return ev, V


def main():
    cfg = synth.CONFIGS["ns16_nt32"]
    U = synth.gauge_field(cfg.ns, cfg.nt, cfg.eps, cfg.seed)
    ev, V = oracle_basis(cfg, U)
    sch = oracle.parse_dilution(cfg.dilution, cfg.nt, cfg.nv)
    rho = oracle.z4_noise(cfg.noise_s, cfg.noise_k, cfg.nt, cfg.nv)
    D = oracle.Dirac(U, cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    out = {"config": cfg.name, "dilution": cfg.dilution, "noise": [cfg.noise_s, cfg.noise_k],
           "slices": SLICES, "sources": SOURCES, "tol": TOL, "iterations": [], "true_resid": [],
           "coef": []}
    t0 = time.time()
    for b in SOURCES:
        P = oracle.dilution_projector(sch, cfg.nt, cfg.nv, b)
        assert all(t in SLICES for t in range(cfg.nt) if P[t].any()), b
        eta = oracle.source(V, rho, sch, b)
        x, it, tr = D.solve(eta, tol=TOL, maxiter=20000)
        assert it > 0 and tr <= TOL, (b, it, tr)
        c = oracle.sink_project(V, x)[SLICES]  # [4 slices, 4, nv]
        out["iterations"].append(int(it))
        out["true_resid"].append(float(tr))
        out["coef"].append([[float(v.real), float(v.imag)] for v in c.reshape(-1)])
        print("source", b, "iterations", it, "true residual %.2e" % tr, "%.0f s" % (time.time() - t0), flush=True)
    out["seconds"] = round(time.time() - t0, 1)
    out["threads"] = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))
    with open(os.path.join(ROOT, "tests", "golden", "oracle_coef_ns16_nt32.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()

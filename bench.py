#!/usr/bin/env python3
"""Benchmark: LapH sources solved per second on the 24^3 x 128 anisotropic lattice.

One step is one pass of the hot path over one batch of synthetic input: the 32 diluted
sources of one source time (4 spins x 8 LapH-interlace projectors of the (TF, SF, LI8)
scheme) are built from the LapH eigenvectors (make_diluted_source), solved to a true FP64
residual of 1e-10 (dirac_solve) and projected onto the LapH subspace (sink_project).
Setup that the paper also does once per configuration (stout smearing, the eigenvectors,
the clover term) runs before the timed region and is reported separately.

The headline value is the mixed-precision multi-right-hand-side form; the plain FP64
GPU solver (one right-hand side at a time) is timed on one batch beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# MI355X FP32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz;
# the library's kernels are compiled without packed FP32, so half of it is the attainable
# issue rate
FP32_VECTOR_PEAK_TFS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# counter summary of the multi-RHS hops on the 24^3 x 128 workload (R = 32, FP16 records)
TRAFFIC = "profiles/dslash_lds_f16_R32_24x24x24x128_traffic.json"


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (TRAFFIC: FETCH_SIZE x its copy-kernel scale + WRITE_SIZE), or None when there is none
    or the kernel's source has changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, TRAFFIC)
    if not kernel or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(kernel)
    if not rec:
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return {"bytes_per_launch": rec["bytes_per_launch"], "source": "%s (%s)" % (TRAFFIC, rec["profile"])}


def cpu_baseline(cfg, U, evecs_np, dil_text, iters_sample, log_fn):
    """The oracle timed on a bounded sample of the same workload: its CG on the normal
    equations of Omega for source b = 0, `iters_sample` iterations, extrapolated to the
    number of iterations the oracle needs for a full solve of that source."""
    import numpy as np

    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rho = oracle.z4_noise(cfg.noise_s, cfg.noise_k, cfg.nt, cfg.nv)
    sch = oracle.parse_dilution(dil_text, cfg.nt, cfg.nv)
    eta = oracle.source(evecs_np, rho, sch, 0)
    D = oracle.Dirac(U, cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    t0 = time.time()
    x, it, tr = D.solve(eta, tol=1e-10, maxiter=iters_sample)
    dt = time.time() - t0
    n = abs(it)
    per_iter = dt / max(n, 1)
    full = None
    path = os.path.join(ROOT, "tests", "golden", "oracle_cgnr_iters_%s.json" % cfg.name)
    if os.path.exists(path):
        with open(path) as f:
            rec = json.load(f)
        if abs(rec.get("m0", 1e9) - cfg.m0) < 1e-12:
            full = int(rec["iterations"])
    est_iters = full if full else None
    value = (1.0 / (per_iter * est_iters)) if est_iters else None
    log_fn("cpu oracle: %d CGNR iterations in %.1f s (%.2f s/iter), full solve %s iterations"
           % (n, dt, per_iter, est_iters))
    return {
        "value": value,
        "unit": "sources/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "%d iterations of the oracle's CG on Omega^dag Omega for source b=0 of the %s workload "
                  "(%.1f s, %.3f s/iteration), scaled by the %s iterations the oracle needs for that "
                  "source at true residual 1e-10" % (n, cfg.name, dt, per_iter,
                                                     est_iters if est_iters else "(unknown)"),
        "seconds_per_iteration": per_iter,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ns24_nt128")
    ap.add_argument("--precision", default="f16")
    ap.add_argument("--block", type=int, default=32)
    ap.add_argument("--solver", default="cgnr", choices=["cgnr", "bicgstab"],
                    help="Krylov method of both forms (BiCGStab breaks down near the critical mass "
                         "of this workload; CG on the normal equations is the paper's fallback)")
    ap.add_argument("--fp64-steps", type=int, default=1, help="batches timed with the plain FP64 solver")
    ap.add_argument("--cpu-iters", type=int, default=8, help="oracle CG iterations in the CPU sample (0: skip)")
    ap.add_argument("--m0", type=float, default=None)
    ap.add_argument("--reliable-delta", type=float, default=0.03,
                    help="reliable-update threshold (measured best on this workload; library default 0.1)")
    ap.add_argument("--reliable-every", type=int, default=50)
    ap.add_argument("--guess", default="none", choices=["none", "net"],
                    help="initial guess of the headline form: zero, or the trained network's N(gamma_4 eta)")
    ap.add_argument("--learned-mixed-steps", type=int, default=1,
                    help="steps of the headline form with the trained network's initial guess (0: skip)")
    ap.add_argument("--learned-sources", type=int, default=2,
                    help="sources solved with FGMRES and the learned preconditioner (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path (LapH sources "
              "are independent solves; several GPUs would each take their own share of the "
              "dilution indices)", file=sys.stderr)
        return 2

    import dataclasses

    import numpy as np
    import torch

    import paper_1104_3870_amd as P
    import synth

    cfg = synth.CONFIGS[args.workload]
    if args.m0 is not None:
        cfg = dataclasses.replace(cfg, m0=args.m0)
    torch.cuda.set_device(0)
    nsrc = 32  # sources of one source time: 4 spins x 8 LapH-interlace projectors
    times = [0, cfg.nt // 4, cfg.nt // 2, 3 * cfg.nt // 4]  # four source times

    t_setup = time.time()
    U = synth.gauge_field(cfg.ns, cfg.nt, cfg.eps, cfg.seed)
    log("gauge field generated in %.1f s" % (time.time() - t_setup))
    Ud = torch.from_numpy(U).cuda()
    L = P.Lattice(cfg.ns, cfg.nt)
    evals = np.zeros((cfg.nt, cfg.nv))
    evecs = torch.empty((cfg.nt, cfg.nv, cfg.ns, cfg.ns, cfg.ns, 3), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    t_eig = time.time()
    est = P.laph_eigvecs(L.ctx, Ud, cfg.stout_rho, cfg.stout_steps, cfg.nv, evals, evecs, krylov=cfg.krylov,
                         cheb_order=cfg.cheb_order, lam_l=cfg.lam_l, lam_c=cfg.lam_c, tol=cfg.eig_tol,
                         max_restarts=60)
    torch.cuda.synchronize()
    t_eig = time.time() - t_eig
    log("eigenvectors: %.1f s, restarts %d, matvecs %d, max residual %.2e, orth %.2e, gap %.2e"
        % (t_eig, est.restarts, est.matvecs, est.max_residual, est.max_orth, est.min_gap))

    dil = P.laph_parse_dilution(cfg.dilution, cfg.nt, cfg.nv)
    prm = P.laph_dirac(cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    shape = (nsrc, cfg.nt, cfg.ns, cfg.ns, cfg.ns, 4, 3)
    eta = torch.empty(shape, dtype=torch.complex128, device="cuda")
    x = torch.empty(shape, dtype=torch.complex128, device="cuda")
    coef = torch.empty((nsrc, cfg.nt, 4, cfg.nv), dtype=torch.complex128, device="cuda")

    def step(k, sv):
        t0 = times[k % len(times)]
        b_first = t0 * 4 * 8  # (t0 * n_S + 0) * n_L + 0
        P.make_diluted_source(L.ctx, evecs, cfg.nv, cfg.noise_s, cfg.noise_k, dil, b_first, nsrc, eta)
        st = P.dirac_solve(L.ctx, Ud, prm, eta, x, nsrc, sv)
        P.sink_project(L.ctx, evecs, cfg.nv, x, nsrc, coef)
        return st

    kind = P.LAPH_SOLVER_CGNR if args.solver == "cgnr" else P.LAPH_SOLVER_BICGSTAB
    guess_net, guess_meta = None, None
    if args.guess == "net":
        from paper_1104_3870_amd import train_ptnet as T

        w, guess_meta = T.load(os.path.join(ROOT, "paper_1104_3870_amd", "weights", "ptnet.npz"))
        guess_net = P.PTNet(L.ctx, guess_meta["channels"])
        guess_net.set_weights(w)
    best = P.solver_params(net=guess_net, tol=cfg.solve_tol, maxiter=6000, precision=args.precision, block_rhs=args.block,
                           solver=kind, reliable_every=args.reliable_every, reliable_delta=args.reliable_delta)
    plain = P.solver_params(tol=cfg.solve_tol, maxiter=6000, precision="f64", block_rhs=1, solver=kind)
    t_setup = time.time() - t_setup

    # ---------------- headline form: warmup, then exactly K timed steps
    for k in range(args.warmup):
        st = step(k, best)
        log("warmup %d: iters %s" % (k, sorted(s.iters for s in st)[::8]))
    torch.cuda.synchronize()
    P.laph_set_timing(L.ctx, True)
    P.laph_get_timing(L.ctx, reset=True)
    iters, resid = [], []
    torch.cuda.synchronize()
    t0 = time.time()
    for k in range(args.steps):
        st = step(args.warmup + k, best)
        iters += [s.iters for s in st]
        resid += [s.true_resid for s in st]
        log("step %d done (%.1f s): max true residual %.2e" % (k, time.time() - t0, max(s.true_resid for s in st)))
    torch.cuda.synchronize()
    elapsed = time.time() - t0
    tm = P.laph_get_timing(L.ctx, reset=True)
    P.laph_set_timing(L.ctx, False)
    value = nsrc * args.steps / elapsed

    # ---------------- plain FP64 solver, one right-hand side at a time
    fp64 = None
    if args.fp64_steps > 0:
        torch.cuda.synchronize()
        t1 = time.time()
        it64 = []
        for k in range(args.fp64_steps):
            st = step(k, plain)
            it64 += [s.iters for s in st]
            log("fp64 step %d done (%.1f s)" % (k, time.time() - t1))
        torch.cuda.synchronize()
        e64 = time.time() - t1
        fp64 = {"value": nsrc * args.fp64_steps / e64, "unit": "sources/s", "steps": args.fp64_steps,
                "ms_per_step": 1000 * e64 / args.fp64_steps, "mean_iters": float(np.mean(it64)),
                "form": "FP64 even-odd %s, one right-hand side at a time" % args.solver.upper()}

    # ---------------- learned + mixed + multi-RHS: the headline form started from N(gamma_4 eta)
    learned_mixed = None
    if args.learned_mixed_steps > 0 and guess_net is None:
        from paper_1104_3870_amd import train_ptnet as T

        w, meta = T.load(os.path.join(ROOT, "paper_1104_3870_amd", "weights", "ptnet.npz"))
        gnet = P.PTNet(L.ctx, meta["channels"])
        gnet.set_weights(w)
        svg = P.solver_params(net=gnet, tol=cfg.solve_tol, maxiter=6000, precision=args.precision,
                              block_rhs=args.block, solver=kind, reliable_every=args.reliable_every,
                              reliable_delta=args.reliable_delta)
        torch.cuda.synchronize()
        t3 = time.time()
        itg = []
        for k in range(args.learned_mixed_steps):
            st = step(k, svg)
            itg += [q.iters for q in st]
        torch.cuda.synchronize()
        eg = time.time() - t3
        learned_mixed = {"value": round(nsrc * args.learned_mixed_steps / eg, 4), "unit": "sources/s",
                         "steps": args.learned_mixed_steps, "mean_iters": float(np.mean(itg)),
                         "form": "headline form with the initial guess x0 = N(gamma_4 eta) of the trained PT-net"}
        log("learned + mixed: %.3f sources/s, %.1f iterations" % (learned_mixed["value"], learned_mixed["mean_iters"]))
        gnet.close()

    # ---------------- learned preconditioner: FGMRES with the trained PT-net, one source at a time
    learned = None
    if args.learned_sources > 0:
        from paper_1104_3870_amd import train_ptnet as T

        wpath = os.path.join(ROOT, "paper_1104_3870_amd", "weights", "ptnet.npz")
        t_tr = time.time()
        from_file = os.path.exists(wpath)
        if from_file:
            w, meta = T.load(wpath)
        else:
            w, meta = T.train(epochs=20, log=log)
        t_tr = time.time() - t_tr
        net = P.PTNet(L.ctx, meta["channels"])
        net.set_weights(w)
        nl = min(args.learned_sources, nsrc)
        svl = P.solver_params(tol=cfg.solve_tol, maxiter=3000, solver=P.LAPH_SOLVER_FGMRES, net=net, restart=32)
        P.make_diluted_source(L.ctx, evecs, cfg.nv, cfg.noise_s, cfg.noise_k, dil, 0, nl, eta[:nl])
        torch.cuda.synchronize()
        t2 = time.time()
        st = P.dirac_solve(L.ctx, Ud, prm, eta[:nl], x[:nl], nl, svl)
        P.sink_project(L.ctx, evecs, cfg.nv, x[:nl], nl, coef[:nl])
        torch.cuda.synchronize()
        el = time.time() - t2
        hist = meta.get("history", {})
        learned = {"value": round(nl / el, 4), "unit": "sources/s", "sources": nl,
                   "mean_iters": float(np.mean([q.iters for q in st])),
                   "fallbacks": int(sum(q.fallback_used for q in st)),
                   "max_true_resid": float(max(q.true_resid for q in st)),
                   "form": "even-odd FGMRES(32), FP64 basis, PT-net right preconditioner, channels %s "
                           "(BF16 weights, FP32 arithmetic)" % meta["channels"],
                   "training": {"pairs": meta["pairs_per_seed"] * (meta["train_seeds"][1] - meta["train_seeds"][0] + 1),
                                "lattice": meta["lattice"], "epochs": meta["epochs"],
                                "test_loss": hist.get("test", [None])[-1],
                                "untrained_test_loss": hist.get("test", [None])[0],
                                "data_s": meta["data_s"], "train_s": meta["train_s"],
                                "weights": "trained earlier with train_ptnet.py" if from_file else
                                           "trained in this run (%.1f s)" % t_tr}}
        log("learned: %d sources in %.2f s, iterations %s" % (nl, el, [q.iters for q in st]))
        net.close()

    # roofline of the dominant kernel (largest summed duration in the timed region)
    traffic = measured_traffic(tm[0]["kernel"] if tm else None)
    dom = tm[0] if tm else {"kernel": "none", "ms": 0.0, "launches": 0, "bytes": 0.0}
    avg_ms = dom["ms"] / max(dom["launches"], 1)
    bytes_per_launch = dom["bytes"] / max(dom["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic["bytes_per_launch"] if traffic else None,
                "traffic_source": traffic["source"] if traffic else None,
                "traffic_rate_frac": (round(traffic["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                                      if traffic and avg_ms > 0 else None),
                "kernel": dom["kernel"], "avg_launch_ms": round(avg_ms, 4), "launches": dom["launches"],
                "algorithmic_bytes_per_launch": bytes_per_launch,
                "share_of_timed_region": round(dom["ms"] / (1000 * elapsed), 3),
                "other_kernels": [{"kernel": k["kernel"], "launches": k["launches"],
                                   "avg_launch_ms": round(k["ms"] / max(k["launches"], 1), 4)} for k in tm[1:]]}

    # the same kernel against the FP32 vector peak: the multi-RHS hop is bound by VALU issue
    # (SQ counters), not by HBM. Algorithmic flops per output site and RHS: 1320 for the
    # hopping term, 504 per clover(-inverse) block application
    flops_site = {"plain": 1320, "plain_cg": 1320, "inv": 1824, "inv_dag": 2328}
    mode = dom["kernel"].split(",")[1] if dom["kernel"].count(",") >= 2 else None
    roofline_alu = None
    if mode in flops_site and dom["kernel"].startswith("dslash_lds") and avg_ms > 0:
        fl = flops_site[mode] * (cfg.ns ** 3 * cfg.nt // 2) * args.block
        tf = fl / (avg_ms * 1e-3) / 1e12
        roofline_alu = {"bound": "alu", "achieved": round(tf, 2), "peak": FP32_VECTOR_PEAK_TFS, "unit": "TFLOP/s",
                        "frac": round(tf / FP32_VECTOR_PEAK_TFS, 4), "flops_per_launch": fl,
                        "frac_of_unpacked_peak": round(tf / (FP32_VECTOR_PEAK_TFS / 2), 4),
                        "kernel": dom["kernel"]}

    cpu = None
    if args.cpu_iters > 0:
        cpu = cpu_baseline(cfg, U, evecs.cpu().numpy(), cfg.dilution, args.cpu_iters, log)

    out = {
        "metric": "LapH sources solved/s @ FP64 resid 1e-10",
        "value": round(value, 4),
        "unit": "sources/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000 * elapsed / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f16": "f16", "f32": "f32", "bf16": "bf16", "f64": "f64"}[args.precision] + "+f64",
        "data": "synthetic",
        "config": {"workload": "24^3x128 anisotropic Wilson-clover, xi=3.5, N_v=112, (TF,SF,LI8), "
                               "32 sources per step" if cfg.name == "ns24_nt128" else cfg.name,
                   "lattice": [cfg.ns, cfg.ns, cfg.ns, cfg.nt], "nv": cfg.nv, "m0": cfg.m0,
                   "dilution": cfg.dilution, "sources_per_step": nsrc,
                   "form": "even-odd %s, %s inner vectors, %d right-hand sides per batch, FP64 reliable "
                           "updates%s" % (args.solver.upper(), args.precision, args.block,
                                          ", initial guess from the trained PT-net" if guess_net else "")},
        "mean_iters": float(np.mean(iters)),
        "max_true_resid": float(max(resid)),
        "fp64_plain": fp64,
        "speedup_vs_fp64": round(value / fp64["value"], 3) if fp64 else None,
        "learned_mixed": learned_mixed,
        "learned": learned,
        "setup_s": {"total": round(t_setup, 2), "eigvecs": round(t_eig, 2), "eig_restarts": est.restarts},
        "roofline": roofline,
        "roofline_alu": roofline_alu,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    L.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())

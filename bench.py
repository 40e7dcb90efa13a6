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


def _golden_iters(cfg, suffix):
    path = os.path.join(ROOT, "tests", "golden", "oracle_cgnr_iters_%s%s.json" % (cfg.name, suffix))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if abs(rec.get("m0", 1e9) - cfg.m0) > 1e-12 or not rec.get("converged"):
        return None
    return rec


def _oracle_sample(cfg, U, evecs_np, iters):
    """Seconds per iteration of the oracle's CG on Omega^dag Omega for source b = 0."""
    import oracle

    rho = oracle.z4_noise(cfg.noise_s, cfg.noise_k, cfg.nt, cfg.nv)
    sch = oracle.parse_dilution(cfg.dilution, cfg.nt, cfg.nv)
    eta = oracle.source(evecs_np, rho, sch, 0)
    D = oracle.Dirac(U, cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    t0 = time.time()
    x, it, tr = D.solve(eta, tol=1e-10, maxiter=iters)
    dt = time.time() - t0
    return abs(it), dt


def cpu_baseline(cfg, U, evecs_np, iters_sample, iters_one_core, log_fn):
    """The oracle timed on a bounded sample of the same workload: its (unpreconditioned,
    full-lattice) CG on the normal equations of Omega for LapH source b = 0, a few
    iterations on all host threads (and, in a child process, on one), scaled by the
    iterations the oracle needs for a full solve of that source."""
    import subprocess

    import numpy as np

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n, dt = _oracle_sample(cfg, U, evecs_np, iters_sample)
    per_iter = dt / max(n, 1)
    rec = _golden_iters(cfg, "_laph")
    what = "that LapH source"
    if rec is None:
        rec = _golden_iters(cfg, "")
        what = "a Gaussian source of this workload (no count for the LapH source is stored)"
    full = int(rec["iterations"]) if rec else None
    value = (1.0 / (per_iter * full)) if full else None
    one = None
    if iters_one_core > 0:
        # one thread: a child process (the oracle's OpenMP pool is sized at load time)
        tmp = os.path.join("/tmp", "laph_oracle_sample_%d.npz" % os.getpid())
        np.savez(tmp, U=U, V=evecs_np)
        code = ("import sys, json, numpy as np; sys.path.insert(0, %r); import bench, synth; "
                "d = np.load(%r); cfg = synth.CONFIGS[%r]; "
                "print(json.dumps(bench._oracle_sample(cfg, d['U'], d['V'], %d)))" % (ROOT, tmp, cfg.name,
                                                                                      iters_one_core))
        env = dict(os.environ, OMP_NUM_THREADS="1")
        try:
            out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
            n1, dt1 = json.loads(out.stdout.strip().splitlines()[-1])
            one = {"value": (1.0 / (dt1 / max(n1, 1) * full)) if full else None, "cores": 1,
                   "seconds_per_iteration": dt1 / max(n1, 1), "sample_iterations": n1}
        except Exception as e:  # the one-core figure is context only
            log_fn("one-core oracle sample failed: %s" % e)
        finally:
            if os.path.exists(tmp):
                os.remove(tmp)
    log_fn("cpu oracle: %d CGNR iterations in %.1f s (%.2f s/iter), full solve %s iterations"
           % (n, dt, per_iter, full))
    return {
        "value": value,
        "unit": "sources/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "%d iterations of the oracle's CG on Omega^dag Omega (full lattice, no even-odd "
                  "preconditioning) for LapH source b=0 of the %s workload (%.1f s, %.3f s/iteration), "
                  "scaled by the %s iterations the oracle needs at true residual 1e-10 for %s; the GPU "
                  "solves the even-odd system, whose CG needs ~366 iterations" % (
                      n, cfg.name, dt, per_iter, full if full else "(unknown)", what),
        "seconds_per_iteration": per_iter,
        "one_core": one,
    }


def _oracle_path(cfg, slices, sources):
    """The oracle's whole path for the dilution indices `sources`: stout smearing, the
    eigenvectors of `slices` (those the sources and sinks use), then per source its
    construction, its CG solve to the workload's bar and its sink projection.  Seconds per
    part and the CG iterations."""
    import numpy as np

    import oracle
    import synth

    U = synth.gauge_field(cfg.ns, cfg.nt, cfg.eps, cfg.seed)
    t = {}
    t0 = time.time()
    S = oracle.stout_spatial(U, cfg.stout_rho, cfg.stout_steps)
    t["stout_s"] = time.time() - t0
    t0 = time.time()
    ev, V0 = oracle.laph_eigpairs(S, cfg.nv, slices=slices)
    t["eigvecs_s"] = time.time() - t0
    V = np.zeros((cfg.nt, cfg.nv, cfg.ns, cfg.ns, cfg.ns, 3), dtype=np.complex128)
    V[slices] = V0
    rho = oracle.z4_noise(cfg.noise_s, cfg.noise_k, cfg.nt, cfg.nv)
    sch = oracle.parse_dilution(cfg.dilution, cfg.nt, cfg.nv)
    D = oracle.Dirac(U, cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    t["source_s"] = t["solve_s"] = t["sink_s"] = 0.0
    its = []
    for b in sources:
        t0 = time.time()
        eta = oracle.source(V, rho, sch, b)
        t1 = time.time()
        x, it, tr = D.solve(eta, tol=cfg.solve_tol, maxiter=20000)
        t2 = time.time()
        oracle.sink_project(V, x)
        t3 = time.time()
        t["source_s"] += t1 - t0
        t["solve_s"] += t2 - t1
        t["sink_s"] += t3 - t2
        its.append(abs(it))
    t["iterations"] = its
    return t


def cpu_report(log_fn):
    """The oracle end to end on the host cores for the two smaller workloads: 4^3 x 8 in full
    (all 256 sources, all slices) on all cores, and on one core for 16 of its sources; for
    16^3 x 32 the eigenvectors of the two slices and the one source of dilution index 0,
    extrapolated to 32 slices and 512 sources (on one core: its CG iterations alone,
    extrapolated the same way)."""
    import subprocess

    import synth

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))

    def one_core(name, slices, sources):
        code = ("import sys, json; sys.path.insert(0, %r); import bench, synth; "
                "print(json.dumps(bench._oracle_path(synth.CONFIGS[%r], %r, %r)))" % (ROOT, name, slices, sources))
        out = subprocess.run([sys.executable, "-c", code], env=dict(os.environ, OMP_NUM_THREADS="1"),
                             capture_output=True, text=True, timeout=1200)
        return json.loads(out.stdout.strip().splitlines()[-1])

    rep = {"cores": threads}
    cfg = synth.CONFIGS["ns4_nt8"]
    nsrc = 256
    t = _oracle_path(cfg, list(range(cfg.nt)), list(range(nsrc)))
    tot = sum(t[k] for k in ("stout_s", "eigvecs_s", "source_s", "solve_s", "sink_s"))
    t1 = one_core(cfg.name, list(range(cfg.nt)), list(range(16)))
    tot1 = t1["stout_s"] + t1["eigvecs_s"] + (t1["source_s"] + t1["solve_s"] + t1["sink_s"]) * nsrc / 16
    rep[cfg.name] = {"measured": "all %d sources, all slices" % nsrc, "seconds": round(tot, 2),
                     "sources_per_s": round(nsrc / tot, 3), "mean_iterations": sum(t["iterations"]) / nsrc,
                     "parts_s": {k: round(v, 2) for k, v in t.items() if k.endswith("_s")},
                     "one_core": {"seconds": round(tot1, 2), "sources_per_s": round(nsrc / tot1, 3),
                                  "measured": "16 sources, scaled to 256"}}
    log_fn("cpu report %s: %.1f s all cores, %.1f s one core" % (cfg.name, tot, tot1))
    cfg = synth.CONFIGS["ns16_nt32"]
    nsrc = 512
    t = _oracle_path(cfg, [0, cfg.nt // 2], [0])
    tot = t["stout_s"] + t["eigvecs_s"] * cfg.nt / 2 + (t["source_s"] + t["solve_s"] + t["sink_s"]) * nsrc
    rep[cfg.name] = {"measured": "eigenvectors of 2 slices, source 0 (CG %d iterations); extrapolated to %d "
                                 "slices and %d sources" % (t["iterations"][0], cfg.nt, nsrc),
                     "seconds": round(tot, 1), "sources_per_s": round(nsrc / tot, 5),
                     "parts_s": {k: round(v, 2) for k, v in t.items() if k.endswith("_s")}}
    log_fn("cpu report %s: %.0f s all cores (extrapolated)" % (cfg.name, tot))
    return rep


def guess_weights():
    """weights of the network's initial guess: those trained on LapH sources when present
    (train_ptnet.py --sources laph), else the preconditioner's"""
    p = os.path.join(ROOT, "paper_1104_3870_amd", "weights", "ptnet_guess.npz")
    return p if os.path.exists(p) else os.path.join(ROOT, "paper_1104_3870_amd", "weights", "ptnet.npz")


def copy_peak_gbs(reps=10, nbytes=1 << 30):
    """Measured streaming rate of the box (read + write bytes over time, median of reps on
    1 GiB): the faster of a device-to-device copy and an elementwise kernel (out = 1.0 a,
    FP32), the attainable rate beside the nominal 8 TB/s.  Returns (GB/s, which)."""
    import torch

    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    best = (0.0, "")
    for name, fn in (("device-to-device copy", lambda: b.copy_(a)),
                     ("elementwise kernel", lambda: torch.mul(a, 1.0, out=b))):
        fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        gbs = 2.0 * nbytes / (sorted(ts)[len(ts) // 2] * 1e-3) / 1e9
        if gbs > best[0]:
            best = (gbs, name)
    del a, b
    return best


def hop_roofline(k):
    """HBM roofline of one kernel from the library's per-kernel event timing: algorithmic
    bytes per launch over the average launch duration, and the counter traffic when a
    summary for the kernel's current source exists."""
    avg_ms = k["ms"] / max(k["launches"], 1)
    bpl = k["bytes"] / max(k["launches"], 1)
    achieved = bpl / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic = measured_traffic(k["kernel"])
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic["bytes_per_launch"] if traffic else None,
            "traffic_source": traffic["source"] if traffic else None,
            "traffic_rate_frac": (round(traffic["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                                  if traffic and avg_ms > 0 else None),
            "kernel": k["kernel"], "avg_launch_ms": round(avg_ms, 4), "launches": k["launches"],
            "algorithmic_bytes_per_launch": bpl}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ns24_nt128")
    ap.add_argument("--precision", default="f16")
    ap.add_argument("--block", type=int, default=0, help="right-hand sides per batch (0: the autotuner's choice)")
    ap.add_argument("--graph", type=int, default=1, help="replay the Krylov iteration from HIP graphs")
    ap.add_argument("--solver", default="bicgstab", choices=["cgnr", "bicgstab"],
                    help="Krylov method of the headline and plain FP64 forms: the paper's even-odd "
                         "BiCGStab, or CG on the normal equations (its fallback)")
    ap.add_argument("--fp64-steps", type=int, default=1, help="batches timed with the plain FP64 solver")
    ap.add_argument("--cpu-iters", type=int, default=8, help="oracle CG iterations in the CPU sample (0: skip)")
    ap.add_argument("--cpu-iters-1core", type=int, default=2, help="oracle CG iterations on one thread (0: skip)")
    ap.add_argument("--hadron-reps", type=int, default=20, help="timed meson-function launches (0: skip)")
    ap.add_argument("--m0", type=float, default=None)
    ap.add_argument("--reliable-delta", type=float, default=0.1,
                    help="reliable-update threshold (the library default; measured best for BiCGStab here)")
    ap.add_argument("--reliable-every", type=int, default=50)
    ap.add_argument("--guess", default="none", choices=["none", "net"],
                    help="initial guess of the headline form: zero, or the trained network's N(gamma_4 eta)")
    ap.add_argument("--learned-mixed-steps", type=int, default=-1,
                    help="steps of the headline form with the trained network's initial guess (0: skip; "
                         "-1: as many as the headline)")
    ap.add_argument("--bicgstab-probe", type=int, default=0,
                    help="only run the paper's solver, FP64 BiCGStab on the even-odd system, on the first "
                         "LapH source with this many iterations at most, and print its outcome (with "
                         "LAPH_VERBOSE=1 the library logs the residual every 256 iterations)")
    ap.add_argument("--mass-scan", default="",
                    help="only solve the first LapH source with FP64 even-odd CGNR at each of these comma-"
                         "separated masses m0 (the workload's eigenvectors) and print the iteration counts")
    ap.add_argument("--cpu-report", action="store_true",
                    help="only time the oracle end to end on the host cores for the two smaller workloads "
                         "and print the figures (no GPU)")
    ap.add_argument("--learned-sources", type=int, default=2,
                    help="sources solved with FGMRES and the learned preconditioner (0: skip)")
    args = ap.parse_args()
    if args.cpu_report:
        print(json.dumps({"cpu_report": cpu_report(log)}))
        return 0
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

    if args.mass_scan:
        sv = P.solver_params(tol=cfg.solve_tol, maxiter=8000, precision="f64", block_rhs=1,
                             solver=P.LAPH_SOLVER_CGNR)
        P.make_diluted_source(L.ctx, evecs, cfg.nv, cfg.noise_s, cfg.noise_k, dil, 0, 1, eta[:1])
        scan = []
        for m0 in [float(v) for v in args.mass_scan.split(",")]:
            pm = P.laph_dirac(m0, cfg.xi, cfg.csw, cfg.bc_t)
            torch.cuda.synchronize()
            t0 = time.time()
            try:
                st = P.dirac_solve(L.ctx, Ud, pm, eta[:1], x[:1], 1, sv)
                rec = {"m0": m0, "iters": st[0].iters, "true_resid": st[0].true_resid, "status": st[0].status}
            except P.LaphError as e:
                rec = {"m0": m0, "error": str(e)}
            torch.cuda.synchronize()
            rec["seconds"] = round(time.time() - t0, 2)
            log("mass scan: %s" % rec)
            scan.append(rec)
        print(json.dumps({"mass_scan": {"workload": cfg.name, "source": "LapH source b = 0 of (%s)" % cfg.dilution,
                                        "solver": "FP64 CG on the normal equations of the even-odd system",
                                        "points": scan}}))
        return 0

    if args.bicgstab_probe > 0:
        sv = P.solver_params(tol=cfg.solve_tol, maxiter=args.bicgstab_probe, precision="f64", block_rhs=1,
                             solver=P.LAPH_SOLVER_BICGSTAB)
        P.make_diluted_source(L.ctx, evecs, cfg.nv, cfg.noise_s, cfg.noise_k, dil, 0, 1, eta[:1])
        torch.cuda.synchronize()
        t0 = time.time()
        st = P.dirac_solve(L.ctx, Ud, prm, eta[:1], x[:1], 1, sv)
        torch.cuda.synchronize()
        print(json.dumps({"bicgstab_probe": {
            "workload": cfg.name, "m0": cfg.m0, "source": "LapH source b = 0 of (%s)" % cfg.dilution,
            "iters": st[0].iters, "fallback_used": st[0].fallback_used, "status": st[0].status,
            "true_resid": st[0].true_resid, "seconds": round(time.time() - t0, 2),
            "note": "fallback_used = 1: BiCGStab diverged or stalled and CG on the normal equations finished"}}))
        return 0

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

        w, guess_meta = T.load(guess_weights())
        guess_net = P.PTNet(L.ctx, guess_meta["channels"])
        guess_net.set_weights(w)
    tune = None
    if args.block == 0:
        # the autotuner picks the block size and tile (the solve reuses its choice)
        t_tune = time.time()
        tune = P.laph_autotune(L.ctx, Ud, prm, args.precision)
        tune["seconds"] = round(time.time() - t_tune, 2)
        log("autotuner: R = %d, %d sites per block" % (tune["best_block_rhs"], tune["best_sites_per_block"]))
    block = args.block if args.block else tune["best_block_rhs"]
    best = P.solver_params(net=guess_net, tol=cfg.solve_tol, maxiter=6000, precision=args.precision,
                           block_rhs=args.block, solver=kind, reliable_every=args.reliable_every,
                           reliable_delta=args.reliable_delta, use_graph=args.graph)
    plain = P.solver_params(tol=cfg.solve_tol, maxiter=6000, precision="f64", block_rhs=1, solver=kind)
    t_setup = time.time() - t_setup

    # ---------------- headline form: warmup, then exactly K timed steps
    for k in range(args.warmup):
        st = step(k, best)
        log("warmup %d: iters %s" % (k, sorted(s.iters for s in st)[::8]))
    # the production form: no per-kernel events (they would also switch the graphs off)
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
    value = nsrc * args.steps / elapsed

    # ---------------- instrumented step: the same kernels and launch shapes with HIP events
    # around every hopping launch on the library's stream (graphs off), for the roofline
    P.laph_set_timing(L.ctx, True)
    P.laph_get_timing(L.ctx, reset=True)
    torch.cuda.synchronize()
    t_ins = time.time()
    step(args.warmup + args.steps, best)
    torch.cuda.synchronize()
    t_ins = time.time() - t_ins
    tm = P.laph_get_timing(L.ctx, reset=True)
    P.laph_set_timing(L.ctx, False)

    # ---------------- plain FP64 solver, one right-hand side at a time
    fp64 = None
    if args.fp64_steps > 0:
        # its hops are timed too (events cost far less than these latency-bound launches)
        P.laph_set_timing(L.ctx, True)
        P.laph_get_timing(L.ctx, reset=True)
        torch.cuda.synchronize()
        t1 = time.time()
        it64, r64 = [], []
        for k in range(args.fp64_steps):
            st = step(k, plain)
            it64 += [s.iters for s in st]
            r64 += [s.true_resid for s in st]
            log("fp64 step %d done (%.1f s)" % (k, time.time() - t1))
        torch.cuda.synchronize()
        e64 = time.time() - t1
        tm64 = P.laph_get_timing(L.ctx, reset=True)
        P.laph_set_timing(L.ctx, False)
        fp64 = {"value": nsrc * args.fp64_steps / e64, "unit": "sources/s", "steps": args.fp64_steps,
                "ms_per_step": 1000 * e64 / args.fp64_steps, "mean_iters": float(np.mean(it64)),
                "max_true_resid": float(max(r64)),
                "form": "FP64 even-odd %s, one right-hand side at a time" % args.solver.upper(),
                "roofline": hop_roofline(tm64[0]) if tm64 else None}

    # ---------------- learned + mixed + multi-RHS: the headline form started from N(gamma_4 eta)
    learned_mixed = None
    if args.learned_mixed_steps != 0 and guess_net is None:
        from paper_1104_3870_amd import train_ptnet as T

        w, meta = T.load(guess_weights())
        gnet = P.PTNet(L.ctx, meta["channels"])
        gnet.set_weights(w)
        svg = P.solver_params(net=gnet, tol=cfg.solve_tol, maxiter=6000, precision=args.precision,
                              block_rhs=args.block, solver=kind, reliable_every=args.reliable_every,
                              reliable_delta=args.reliable_delta, use_graph=args.graph)
        nlm = args.learned_mixed_steps if args.learned_mixed_steps > 0 else args.steps
        step(0, svg)  # warm-up of the network's path
        torch.cuda.synchronize()
        t3 = time.time()
        itg, rg = [], []
        for k in range(nlm):
            st = step(args.warmup + k, svg)
            itg += [q.iters for q in st]
            rg += [q.true_resid for q in st]
        torch.cuda.synchronize()
        eg = time.time() - t3
        learned_mixed = {"value": round(nsrc * nlm / eg, 4), "unit": "sources/s",
                         "steps": nlm, "mean_iters": float(np.mean(itg)), "max_true_resid": float(max(rg)),
                         "form": "headline form with the initial guess x0 = N(gamma_4 eta) of the trained PT-net",
                         "weights": "%s (trained on %s sources)" % (os.path.relpath(guess_weights(), ROOT),
                                                                     meta.get("sources", "gauss"))}
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

    # ---------------- hadron functions on the last step's quark lines (Sec. III.B): the
    # meson function of the barred sinks with themselves and of the barred sources, then
    # the connected correlator; timed with events on the library's (torch's current) stream
    hadron = None
    if args.hadron_reps > 0:
        nv, nt = cfg.nv, cfg.nt
        t_src = times[(args.warmup + args.steps) % len(times)]
        b0 = t_src * 4 * 8
        g5 = np.diag([1.0, 1.0, -1.0, -1.0]).astype(np.complex128)
        g5g4 = g5 @ np.array([[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]], dtype=np.complex128)
        sbar = torch.empty_like(coef)
        P.laph_spin_apply(L.ctx, g5g4, coef, nsrc, nv, sbar)
        rbar = torch.empty_like(coef)
        r2 = torch.empty_like(coef)
        P.laph_quark_source(L.ctx, nv, cfg.noise_s, cfg.noise_k, dil, b0, nsrc, rbar, bar=True)
        P.laph_quark_source(L.ctx, nv, cfg.noise_s, cfg.noise_k, dil, b0, nsrc, r2)
        msnk = torch.empty((nt, nsrc, nsrc), dtype=torch.complex128, device="cuda")
        msrc = torch.empty_like(msnk)
        corr = torch.empty(nt, dtype=torch.complex128, device="cuda")
        P.laph_meson_function(L.ctx, g5, sbar, nsrc, coef, nsrc, nv, msnk)  # warm-up
        # the kernel's own duration (HIP events around each launch on the library's stream);
        # the calls back to back also give the per-call time with the host's launch path
        P.laph_set_timing(L.ctx, True)
        P.laph_get_timing(L.ctx, reset=True)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(args.hadron_reps):
            P.laph_meson_function(L.ctx, g5, sbar, nsrc, coef, nsrc, nv, msnk)
        ev1.record()
        torch.cuda.synchronize()
        ms_call = ev0.elapsed_time(ev1) / args.hadron_reps
        tmm = [k for k in P.laph_get_timing(L.ctx, reset=True) if k["kernel"] == "meson_function"]
        P.laph_set_timing(L.ctx, False)
        ms_m = tmm[0]["ms"] / max(tmm[0]["launches"], 1) if tmm else ms_call
        P.laph_meson_function(L.ctx, g5, rbar, nsrc, r2, nsrc, nv, msrc)
        P.laph_meson_correlator(L.ctx, msnk, msrc, nsrc, nsrc, t_src, corr)
        torch.cuda.synchronize()
        mbytes = (2 * nsrc * nt * 4 * nv + nt * nsrc * nsrc) * 16.0
        mflops = 8.0 * nt * nsrc * nsrc * 4 * nv + 2 * 4 * 4 * 8.0 * nsrc * nt * nv
        hadron = {"kernel": "meson_function (%d x %d quark lines, Nt = %d, N_v = %d)" % (nsrc, nsrc, nt, nv),
                  "avg_launch_ms": round(ms_m, 4),
                  "ms_per_call_with_host_launch": round(ms_call, 4),
                  "roofline": {"bound": "hbm", "achieved": round(mbytes / (ms_m * 1e-3) / 1e9, 1),
                               "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(mbytes / (ms_m * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                               "algorithmic_bytes_per_launch": mbytes},
                  "gflops": round(mflops / (ms_m * 1e-3) / 1e9, 1),
                  "fp64_frac": round(mflops / (ms_m * 1e-3) / 78.6e12, 4)}
        log("meson function: %.4f ms per launch (%.4f ms per call with the host's launch path)" % (ms_m, ms_call))
        # displaced LapH vectors and their momentum overlaps (Sec. II displacement types,
        # Sec. III.B momentum projection) on the stout-smeared field
        Usm = torch.empty_like(Ud)
        P.laph_stout_smear(L.ctx, Ud, cfg.stout_rho, cfg.stout_steps, Usm)
        Vdisp = torch.empty_like(evecs)
        O = torch.empty((nt, nv, nv), dtype=torch.complex128, device="cuda")
        P.laph_displace(L.ctx, Usm, 0, 1, 3, evecs, nv, Vdisp)  # warm-up
        P.laph_mom_overlap(L.ctx, evecs, nv, Vdisp, nv, (1, 0, 0), O)
        ev0.record()
        P.laph_displace(L.ctx, Usm, 0, 1, 3, evecs, nv, Vdisp)
        ev1.record()
        ev2 = torch.cuda.Event(enable_timing=True)
        P.laph_mom_overlap(L.ctx, evecs, nv, Vdisp, nv, (1, 0, 0), O)
        ev2.record()
        torch.cuda.synchronize()
        ms_d, ms_o = ev0.elapsed_time(ev1), ev1.elapsed_time(ev2)
        V3 = cfg.ns ** 3
        dbytes = nt * V3 * (2 * nv * 48.0 + 3 * 144.0)  # vectors in and out, three links per site once
        obytes = 2 * nt * nv * V3 * 48.0 + nt * nv * nv * 16.0
        oflops = 8.0 * nt * nv * nv * 3 * V3
        hadron["displace"] = {"kernel": "displace (%d vectors per slice, 3 links)" % nv, "ms": round(ms_d, 3),
                              "roofline": {"bound": "hbm", "achieved": round(dbytes / (ms_d * 1e-3) / 1e9, 1),
                                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                           "frac": round(dbytes / (ms_d * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}
        hadron["mom_overlap"] = {"kernel": "mom_overlap (%d x %d per slice, K = 3 Ns^3)" % (nv, nv),
                                 "ms": round(ms_o, 3),
                                 "roofline": {"bound": "fp64", "achieved": round(oflops / (ms_o * 1e-3) / 1e12, 2),
                                              "peak": 78.6, "unit": "TFLOP/s",
                                              "frac": round(oflops / (ms_o * 1e-3) / 78.6e12, 4)},
                                 "hbm_GBs": round(obytes / (ms_o * 1e-3) / 1e9, 1)}
        log("displace %.3f ms, overlap %.3f ms" % (ms_d, ms_o))
        del Usm, Vdisp, O
        # baryon functions (Sec. III.A): the eigenvector tensor once, then the sink
        # functions of the step's 32 quark lines taken as all three quarks
        T = torch.empty((nt, nv, nv, nv), dtype=torch.complex128, device="cuda")
        cb = np.zeros((4, 4, 4), dtype=np.complex128)
        cb[0, 1, 0], cb[1, 0, 0] = 1.0, -1.0
        nbq = nsrc
        Bout = torch.empty((nt, nbq, nbq, nbq), dtype=torch.complex128, device="cuda")
        ev0.record()
        P.laph_baryon_tensor(L.ctx, evecs, nv, (0, 0, 0), T)
        ev1.record()
        P.laph_baryon_function(L.ctx, T, nv, cb, coef, nbq, coef, nbq, coef, nbq, Bout)
        ev2.record()
        torch.cuda.synchronize()
        ms_t, ms_b = ev0.elapsed_time(ev1), ev1.elapsed_time(ev2)
        tflops = 8.0 * nt * (nv * (nv - 1) * (nv - 2) / 6.0) * 3 * V3  # useful: n1 < n2 < n3
        bflops = 8.0 * nt * (nv * nv * nv * 4 * nbq + nv * nv * 16 * nbq * nbq + 4 * nbq * nv * 16 * nbq * nbq)
        hadron["baryon_tensor"] = {"kernel": "baryon_tensor (N_v = %d, K = 3 Ns^3)" % nv, "ms": round(ms_t, 2),
                                   "roofline": {"bound": "fp64", "achieved": round(tflops / (ms_t * 1e-3) / 1e12, 2),
                                                "peak": 78.6, "unit": "TFLOP/s",
                                                "frac": round(tflops / (ms_t * 1e-3) / 78.6e12, 4)}}
        hadron["baryon_function"] = {"kernel": "baryon_function (%d^3 dilution triples, N_v = %d)" % (nbq, nv),
                                     "ms": round(ms_b, 2),
                                     "roofline": {"bound": "fp64",
                                                  "achieved": round(bflops / (ms_b * 1e-3) / 1e12, 2),
                                                  "peak": 78.6, "unit": "TFLOP/s",
                                                  "frac": round(bflops / (ms_b * 1e-3) / 78.6e12, 4)}}
        log("baryon tensor %.1f ms, baryon function %.1f ms" % (ms_t, ms_b))
        del T, Bout

    # roofline of the dominant kernel (largest summed duration in the instrumented step)
    dom = tm[0] if tm else {"kernel": "none", "ms": 0.0, "launches": 0, "bytes": 0.0}
    roofline = hop_roofline(dom)
    roofline["measured"] = ("HIP events around every hopping launch on the library's stream during one "
                            "instrumented step after the timed region (same kernels and launch shapes; "
                            "graphs off in that step)")
    roofline["share_of_instrumented_step"] = round(dom["ms"] / (1000 * t_ins), 3) if t_ins > 0 else None
    # the same against the measured streaming rate of the box (a plain device copy)
    cp, cp_how = copy_peak_gbs()
    roofline["copy_peak"] = {"achieved": round(cp, 1), "unit": "GB/s",
                             "measured": "median of 10 passes over 1 GiB (read + write bytes), the faster of a "
                                         "device-to-device copy and an elementwise kernel: %s" % cp_how}
    roofline["frac_of_copy_peak"] = round(roofline["achieved"] / cp, 4) if cp > 0 else None
    if fp64 and fp64.get("roofline"):
        fp64["roofline"]["frac_of_copy_peak"] = round(fp64["roofline"]["achieved"] / cp, 4) if cp > 0 else None
    roofline["other_kernels"] = [{"kernel": k["kernel"], "launches": k["launches"],
                                  "avg_launch_ms": round(k["ms"] / max(k["launches"], 1), 4)} for k in tm[1:]]

    # the same kernel against the FP32 vector peak: the multi-RHS hop is bound by VALU issue
    # (SQ counters), not by HBM. Algorithmic flops per output site and RHS: 1320 for the
    # hopping term, 504 per clover(-inverse) block application, 144 for the inner products
    # <y, out> and |out|^2 of the BiCGStab epilogue
    avg_ms = roofline["avg_launch_ms"]
    flops_site = {"plain": 1320, "plain_cg": 1320, "inv": 1824, "inv_dag": 2328, "inv_dot": 1968}
    mode = dom["kernel"].split(",")[1] if dom["kernel"].count(",") >= 2 else None
    rb = int(dom["kernel"].rsplit("R", 1)[1].rstrip(">")) if "R" in dom["kernel"] else block
    roofline_alu = None
    if mode in flops_site and dom["kernel"].startswith("dslash_lds") and avg_ms > 0:
        fl = flops_site[mode] * (cfg.ns ** 3 * cfg.nt // 2) * rb
        tf = fl / (avg_ms * 1e-3) / 1e12
        roofline_alu = {"bound": "alu", "achieved": round(tf, 2), "peak": FP32_VECTOR_PEAK_TFS, "unit": "TFLOP/s",
                        "frac": round(tf / FP32_VECTOR_PEAK_TFS, 4), "flops_per_launch": fl,
                        "frac_of_unpacked_peak": round(tf / (FP32_VECTOR_PEAK_TFS / 2), 4),
                        "kernel": dom["kernel"]}

    cpu = None
    if args.cpu_iters > 0:
        cpu = cpu_baseline(cfg, U, evecs.cpu().numpy(), args.cpu_iters, args.cpu_iters_1core, log)

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
                   "form": "even-odd %s, %s inner vectors, %d right-hand sides per batch (%s), FP64 reliable "
                           "updates, iteration %s%s" % (
                               args.solver.upper(), args.precision, block,
                               "autotuned" if args.block == 0 else "fixed",
                               "replayed from HIP graphs" if args.graph else "launched eagerly",
                               ", initial guess from the trained PT-net" if guess_net else "")},
        "mean_iters": float(np.mean(iters)),
        "max_true_resid": float(max(resid)),
        "fp64_plain": fp64,
        "speedup_vs_fp64": round(value / fp64["value"], 3) if fp64 else None,
        "learned_mixed": learned_mixed,
        "learned": learned,
        "ms_per_step_instrumented": round(1000 * t_ins, 2),
        "autotune": tune,
        "setup_s": {"total": round(t_setup, 2), "eigvecs": round(t_eig, 2), "eig_restarts": est.restarts},
        "roofline": roofline,
        "roofline_alu": roofline_alu,
        "hadron_functions": hadron,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    L.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())

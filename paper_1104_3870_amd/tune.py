"""Workload tuning utility (run on a GPU).

tune_m0: choose the bare mass m0 so that CG on the normal equations of the full system,
Omega^dag Omega x = Omega^dag eta (the paper's fallback solver, Sec. IV), needs a target
number of iterations to reach the true residual 1e-10 on a seeded Gaussian source.  The
workloads name their conditioning by such an iteration count; the synthetic near-unit
fields are smoother than the paper's ensembles, so the mass, not the field, sets it.

Omega is applied by the library (laph_dirac_apply); the CG vector algebra of this
tuning aid uses torch.  The search stays on the physical side of the critical mass: the
count rises as m0 falls towards it, and m0 is not taken below the point where the count
stops rising (further down lie the doubler branches of the Wilson operator).

    python -m paper_1104_3870_amd.tune m0 ns24_nt128 1000
"""
from __future__ import annotations

import json
import math
import sys
import time


def full_cg_iters(P, L, Ud, cfg, m0, eta, tol=1e-10, maxiter=20000):
    """Iterations of CG on Omega^dag Omega (full lattice) to |eta - Omega x| <= tol |eta|."""
    import torch

    prm = P.laph_dirac(m0, cfg.xi, cfg.csw, cfg.bc_t)

    def omega(v):
        out = torch.empty_like(v)
        P.laph_dirac_apply(L.ctx, Ud, prm, P.LAPH_OP_OMEGA, v, out)
        return out

    def omega_dag(v):  # Omega^dag = K^dag gamma_4; gamma_4 swaps the spin pairs
        g = v[..., [2, 3, 0, 1], :].contiguous()
        out = torch.empty_like(v)
        P.laph_dirac_apply(L.ctx, Ud, prm, P.LAPH_OP_KDAG, g, out)
        return out

    x = torch.zeros_like(eta)
    res = eta.clone()
    r = omega_dag(res)
    p = r.clone()
    rr = torch.vdot(r.flatten(), r.flatten()).real
    en = torch.linalg.vector_norm(eta).item()
    for it in range(1, maxiter + 1):
        q = omega(p)
        alpha = rr / torch.vdot(q.flatten(), q.flatten()).real
        x += alpha * p
        res -= alpha * q
        if it % 10 == 0 and torch.linalg.vector_norm(res).item() <= tol * en:
            break
        r -= alpha * omega_dag(q)
        rr_new = torch.vdot(r.flatten(), r.flatten()).real
        p = r + (rr_new / rr) * p
        rr = rr_new
    true = torch.linalg.vector_norm(eta - omega(x)).item() / en
    return it, true


def tune_m0(cfg, target, start=0.2, step=0.04, seed=123, log=print):
    import torch

    import paper_1104_3870_amd as P
    import synth

    U = synth.gauge_field(cfg.ns, cfg.nt, cfg.eps, cfg.seed)
    Ud = torch.from_numpy(U).cuda()
    del U
    L = P.Lattice(cfg.ns, cfg.nt)
    eta = torch.from_numpy(synth.random_spinor(cfg.ns, cfg.nt, seed)).cuda()
    cache = {}

    def f(m0):
        m0 = round(m0, 6)
        if m0 not in cache:
            t0 = time.time()
            it, tr = full_cg_iters(P, L, Ud, cfg, m0, eta)
            cache[m0] = it
            log(json.dumps({"m0": m0, "cg_iters": it, "true_resid": tr, "s": round(time.time() - t0, 2)}))
        return cache[m0]

    # walk down from the heavy side until the target is passed or the count stops rising
    hi, prev = start, f(start)
    lo = None
    m = start
    while m > -3.0:
        m -= step
        v = f(m)
        if v >= target:
            lo = m
            break
        if v < prev:  # passed the critical region without reaching the target
            lo = None
            break
        hi, prev = m, v
    if lo is None:
        best = max(cache, key=lambda k: cache[k] if k >= m else -1)
    else:
        for _ in range(12):
            mid = 0.5 * (lo + hi)
            v = f(mid)
            if abs(math.log(v / target)) < 0.03:
                lo = hi = mid
                break
            if v > target:
                lo = mid
            else:
                hi = mid
        best = min(cache, key=lambda k: abs(math.log(cache[k] / target)))
    L.close()
    return best, cache[best]


def main(argv):
    import synth

    if len(argv) >= 3 and argv[0] == "m0":
        cfg = synth.CONFIGS[argv[1]]
        target = int(argv[2])
        m0, it = tune_m0(cfg, target)
        print(json.dumps({"config": cfg.name, "target": target, "m0": m0, "cg_iters": it}), flush=True)
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))

"""Train the parallel-transport preconditioner network on the GPU with the library's own
forward / backward / Adam kernels.

Data: for each gauge seed a field of the workload's generator (near-unit SU(3) links,
eps 0.4) on a small lattice, and `pairs` sources b with their solutions x = K^-1 b
(dirac_solve with eta = gamma_4 b, since Omega = gamma_4 K).  The network is translation
invariant and local (four nearest-neighbour hops), so weights trained on the small
lattice apply unchanged to 24^3 x 128.  Two source distributions, one per use:
* gauss (FGMRES preconditioner): Gaussian sources on odd sites, the vectors the
  preconditioner is applied to in the even-odd solve;
* laph (initial guess of the solve): b = gamma_4 eta for LapH sources eta = V_s P^(b) rho
  (Sec. II) of (TF,SF,LI8) dilution built on the field's own stout-smeared LapH vectors,
  the input the solver gives the network for its guess.
The loss is taken on odd sites (only the odd part of the output is used).

    python -m paper_1104_3870_amd.train_ptnet --out paper_1104_3870_amd/weights/ptnet.npz
    python -m paper_1104_3870_amd.train_ptnet --sources laph --out paper_1104_3870_amd/weights/ptnet_guess.npz
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_CHANNELS = (1, 2, 2, 2, 1)


def _odd_mask(ns, nt):
    t, z, y, x = np.meshgrid(*[np.arange(n) for n in (nt, ns, ns, ns)], indexing="ij")
    return (((t + z + y + x) & 1) == 1)[..., None, None]


LAPH_NV = 16  # LapH vectors per slice of the small training lattice


def make_pairs(P, L, cfg, ns, nt, seed, pairs, block=32, kind="gauss"):
    """(U, b, x) on the device for one gauge seed."""
    import torch

    import synth

    U = synth.gauge_field(ns, nt, cfg.eps, seed)
    Ud = torch.from_numpy(U).cuda()
    P.laph_forget_gauge(L.ctx)
    if kind == "laph":
        nv = LAPH_NV
        evals = np.zeros((nt, nv))
        evecs = torch.empty((nt, nv, ns, ns, ns, 3), dtype=torch.complex128, device="cuda")
        P.laph_eigvecs(L.ctx, Ud, cfg.stout_rho, cfg.stout_steps, nv, evals, evecs, krylov=60, lam_c=1.0, tol=1e-9,
                       max_restarts=200)
        dil = P.laph_parse_dilution("TF,SF,LI8", nt, nv)
        nb = P.laph_dilution_count(dil, nt, nv)
        b0 = int(np.random.default_rng(seed).integers(0, nb - pairs + 1))
        etad = torch.empty((pairs, nt, ns, ns, ns, 4, 3), dtype=torch.complex128, device="cuda")
        P.make_diluted_source(L.ctx, evecs, nv, seed & 0xFFFF, 1, dil, b0, pairs, etad)
        bd = etad[..., [2, 3, 0, 1], :].contiguous()  # gamma_4 eta (chiral basis)
    else:
        b = synth.random_spinor(ns, nt, 1_000_003 * seed + 17, nrhs=pairs) * _odd_mask(ns, nt)
        bd = torch.from_numpy(np.ascontiguousarray(b)).cuda()
        etad = bd[..., [2, 3, 0, 1], :].contiguous()  # gamma_4 b
    xd = torch.empty_like(bd)
    prm = P.laph_dirac(cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    sv = P.solver_params(tol=1e-9, maxiter=6000, precision="f32", solver=P.LAPH_SOLVER_CGNR,
                         block_rhs=min(block, 32))
    P.dirac_solve(L.ctx, Ud, prm, etad, xd, pairs, sv)
    return Ud, bd, xd


def eval_loss(P, L, net, data, mask_dev, bc_t):
    """Mean relative odd-site error |N(b) - x|^2 / |x|^2 over the pairs."""
    import torch

    tot, n = 0.0, 0
    for Ud, bd, xd in data:
        out = torch.empty_like(bd)
        P.laph_ptnet_forward(L.ctx, net.handle, Ud, bc_t, bd, out, bd.shape[0])
        d = (out - xd) * mask_dev
        num = (d.abs() ** 2).flatten(1).sum(1)
        den = ((xd * mask_dev).abs() ** 2).flatten(1).sum(1)
        tot += float((num / den).sum())
        n += bd.shape[0]
    return tot / n


def train(workload="ns24_nt128", ns=8, nt=16, train_seeds=range(100, 200), test_seeds=range(200, 210), pairs=20,
          epochs=60, lr=2e-3, channels=DEFAULT_CHANNELS, seed=0, log=print, kind="gauss"):
    import torch

    import paper_1104_3870_amd as P
    import synth

    cfg = synth.CONFIGS[workload]
    torch.cuda.set_device(0)
    L = P.Lattice(ns, nt)
    t0 = time.time()
    data = [make_pairs(P, L, cfg, ns, nt, s, pairs, kind=kind) for s in train_seeds]
    test = [make_pairs(P, L, cfg, ns, nt, s, pairs, kind=kind) for s in test_seeds]
    t_data = time.time() - t0
    log("data: %d train pairs, %d test pairs in %.1f s" % (pairs * len(data), pairs * len(test), t_data))
    mask = torch.from_numpy(np.ascontiguousarray(_odd_mask(ns, nt))).cuda()
    net = P.PTNet(L.ctx, channels, seed=seed)
    hist = {"train": [], "test": [eval_loss(P, L, net, test, mask, cfg.bc_t)]}
    log("epoch 0: test loss %.4f" % hist["test"][-1])
    rng = np.random.default_rng(seed)
    t1 = time.time()
    for ep in range(epochs):
        lr_ep = lr * 0.5 * (1 + np.cos(np.pi * ep / epochs))  # cosine schedule
        losses = []
        for i in rng.permutation(len(data)):
            Ud, bd, xd = data[i]
            losses.append(P.laph_ptnet_train_step(L.ctx, net.handle, Ud, cfg.bc_t, bd, xd, pairs, lr=lr_ep,
                                                  loss_parity=1))
        hist["train"].append(float(np.mean(losses)))
        if (ep + 1) % max(1, epochs // 10) == 0 or ep == epochs - 1:
            hist["test"].append(eval_loss(P, L, net, test, mask, cfg.bc_t))
            log("epoch %d: train loss %.4f, test loss %.4f (%.1f s)" % (ep + 1, hist["train"][-1], hist["test"][-1],
                                                                     time.time() - t1))
    t_train = time.time() - t1
    w = net.get_weights()
    meta = {"channels": list(channels), "workload": workload, "lattice": [ns, nt], "m0": cfg.m0, "sources": kind,
            "train_seeds": [min(train_seeds), max(train_seeds)], "test_seeds": [min(test_seeds), max(test_seeds)],
            "pairs_per_seed": pairs, "epochs": epochs, "lr": lr, "data_s": round(t_data, 1),
            "train_s": round(t_train, 1), "history": hist}
    net.close()
    L.close()
    return w, meta


def save(path, w, meta):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, weights=np.asarray(w, dtype=np.complex128), meta=json.dumps(meta))


def load(path):
    with np.load(path, allow_pickle=False) as f:
        return f["weights"], json.loads(str(f["meta"]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="default: weights/ptnet.npz (gauss), weights/ptnet_guess.npz (laph)")
    ap.add_argument("--sources", default="gauss", choices=["gauss", "laph"])
    ap.add_argument("--workload", default="ns24_nt128")
    ap.add_argument("--ns", type=int, default=8)
    ap.add_argument("--nt", type=int, default=16)
    ap.add_argument("--pairs", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--channels", default=",".join(map(str, DEFAULT_CHANNELS)))
    a = ap.parse_args()
    ch = tuple(int(c) for c in a.channels.split(","))
    w, meta = train(a.workload, a.ns, a.nt, pairs=a.pairs, epochs=a.epochs, lr=a.lr, channels=ch,
                    log=lambda *x: print(*x, flush=True), kind=a.sources)
    out = a.out or os.path.join(ROOT, "paper_1104_3870_amd", "weights",
                                "ptnet_guess.npz" if a.sources == "laph" else "ptnet.npz")
    save(out, w, meta)
    print(json.dumps({k: v for k, v in meta.items() if k != "history"}))
    return 0


if __name__ == "__main__":
    sys.exit(main())

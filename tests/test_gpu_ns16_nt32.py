"""The 16^3 x 32 workload end to end on the GPU against the oracle: stout smearing and the
N_v = 48 LapH eigenpairs of every slice (Sec. II, Sec. IV Lanczos settings), all 512
(TI16,SF,LI8) diluted sources solved by the production form (even-odd BiCGStab, FP16 inner
vectors, blocks of 32) and judged by the oracle's Omega, and the LapH coefficients of eight
sources against the oracle's own solution on shared (oracle) eigenvectors.

* Eigenvalues to 1e-9 on four slices; each eigenvector within the Davis-Kahan bound
  2 |(-Lap) v - lambda v| / gap of the oracle's (gap: distance to the rest of the oracle
  spectrum); every slice satisfies the oracle Laplacian's eigen-equation.
* Every solution's true relative residual, computed by the oracle, <= 1e-10.
* Coefficients within 1e-8 of the largest coefficient of the source: the solve's bar
  times the condition number of Omega on this field (<= 100) bounds the difference.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host, say

pytestmark = pytest.mark.gpu

CFG = synth.CONFIGS["ns16_nt32"]
NS, NT, NV = CFG.ns, CFG.nt, CFG.nv
SLICES = [0, 5, 16, 21]
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_coef_ns16_nt32.json")


@pytest.fixture(scope="module")
def P():
    import paper_1104_3870_amd as P

    P.lib()
    return P


@pytest.fixture(scope="module")
def field():
    return synth.gauge_field(NS, NT, CFG.eps, CFG.seed)


@pytest.fixture(scope="module")
def smeared(field):
    return oracle.stout_spatial(field, CFG.stout_rho, CFG.stout_steps)


@pytest.fixture(scope="module")
def dirac(field):
    return oracle.Dirac(field, CFG.m0, CFG.xi, CFG.csw, CFG.bc_t)


@pytest.fixture(scope="module")
def gpu_eig(P, field):
    """GPU eigenpairs of all 32 slices with the workload's Lanczos settings; the device
    tensor stays resident for the source tests"""
    import torch

    say("GPU eigenpairs at 16^3 x 32, N_v = 48")
    L = P.Lattice(NS, NT)
    evals = np.zeros((NT, NV))
    evecs = torch.empty((NT, NV, NS, NS, NS, 3), dtype=torch.complex128, device="cuda")
    st = P.laph_eigvecs(L.ctx, dev(field), CFG.stout_rho, CFG.stout_steps, NV, evals, evecs, krylov=CFG.krylov,
                        cheb_order=CFG.cheb_order, lam_l=CFG.lam_l, lam_c=CFG.lam_c, tol=CFG.eig_tol,
                        max_restarts=100)
    say("  restarts", st.restarts, "max residual", st.max_residual, "orth", st.max_orth)
    return L, st, evals, evecs


def test_eigpairs_ns16_nt32(P, smeared, gpu_eig):
    L, st, evals, evecs = gpu_eig
    # the eigensolver's bar is relative to the Laplacian's norm (<= lambda_L)
    assert st.max_residual < CFG.eig_tol * CFG.lam_l and st.max_orth < 1e-12
    V = host(evecs)
    res = np.empty((NT, NV))
    for n in range(NV):
        v = np.ascontiguousarray(V[:, n])
        r = -oracle.laplacian(smeared, v) - evals[:, n][:, None, None, None, None] * v
        res[:, n] = np.linalg.norm(r.reshape(NT, -1), axis=1)
    say("  max |(-Lap) v - lambda v| over all slices", res.max())
    assert res.max() < 1e-8
    extra = 8
    ev_ref, V_ref = oracle.laph_eigpairs(smeared, NV + extra, slices=SLICES)
    worst_val, worst_ratio = 0.0, 0.0
    for si, t in enumerate(SLICES):
        w = ev_ref[si]
        worst_val = max(worst_val, float(np.abs(evals[t] - w[:NV]).max()))
        for n in range(NV):
            gap = min(abs(evals[t, n] - w[m]) for m in range(NV + extra) if m != n)
            a = V[t, n].reshape(-1)
            b = V_ref[si, n].reshape(-1)
            d = np.linalg.norm(a - b * (np.vdot(b, a) / abs(np.vdot(b, a))))
            bound = 2.0 * res[t, n] / gap + 1e-10
            worst_ratio = max(worst_ratio, d / bound)
            assert d <= bound, (t, n, d, bound)
    say("  eigenvalue max abs err", worst_val, "worst vector difference / Davis-Kahan bound", worst_ratio)
    assert worst_val < 1e-9


@pytest.mark.parametrize("part", range(4))
def test_all_sources_solved_ns16_nt32(P, field, dirac, gpu_eig, part):
    """Sources 128 part .. 128 part + 127 of the 512, in four blocks of 32 (FP16 inner
    vectors, FP64 reliable updates), each judged by the oracle's Omega."""
    import torch

    L, st, evals, evecs = gpu_eig
    dil = P.laph_parse_dilution(CFG.dilution, NT, NV)
    assert P.laph_dilution_count(dil, NT, NV) == 512
    prm = P.laph_dirac(CFG.m0, CFG.xi, CFG.csw, CFG.bc_t)
    sv = P.solver_params(tol=CFG.solve_tol, maxiter=6000, precision="f16", block_rhs=32,
                         solver=P.LAPH_SOLVER_BICGSTAB, use_graph=1)
    Ud = dev(field)
    worst, its = 0.0, []
    for blk in range(4):
        b0 = 128 * part + 32 * blk
        say("  sources", b0, "..", b0 + 31)
        eta = torch.empty((32, NT, NS, NS, NS, 4, 3), dtype=torch.complex128, device="cuda")
        P.make_diluted_source(L.ctx, evecs, NV, CFG.noise_s, CFG.noise_k, dil, b0, 32, eta)
        x = torch.empty_like(eta)
        sts = P.dirac_solve(L.ctx, Ud, prm, eta, x, 32, sv)
        assert all(q.status == 0 and q.fallback_used == 0 for q in sts)
        its += [q.iters for q in sts]
        eh, xh = host(eta), host(x)
        del eta, x
        for r in range(32):
            tr = dirac.true_residual(eh[r], xh[r])
            worst = max(worst, tr)
            assert tr <= 1e-10, (b0 + r, tr)
            assert abs(tr - sts[r].true_resid) <= 1e-12
    say("  worst oracle true residual", worst, "iterations", min(its), "-", max(its))


def test_coefficients_vs_oracle_ns16_nt32(P, field, smeared):
    """Eight sources (b_T = 0 and 5) on the oracle's eigenvectors of the slices they touch:
    the library's source, FP16 solve and sink projection against the coefficients the
    oracle computed with its own CG (true residual 1e-12), stored by
    tests/golden/oracle_coef_ns16_nt32.py."""
    import torch

    with open(GOLDEN) as f:
        g = json.load(f)
    assert g["slices"] == SLICES
    ev, V0 = oracle.laph_eigpairs(smeared, NV, slices=SLICES)  # the golden script's call
    V = np.zeros((NT, NV, NS, NS, NS, 3), dtype=np.complex128)
    V[SLICES] = V0
    L = P.Lattice(NS, NT)
    Vd = dev(V)
    dil = P.laph_parse_dilution(CFG.dilution, NT, NV)
    src = g["sources"]
    n = len(src)
    eta = torch.empty((n, NT, NS, NS, NS, 4, 3), dtype=torch.complex128, device="cuda")
    # two contiguous runs of four dilution indices
    for i0 in range(0, n, 4):
        assert src[i0:i0 + 4] == list(range(src[i0], src[i0] + 4))
        P.make_diluted_source(L.ctx, Vd, NV, CFG.noise_s, CFG.noise_k, dil, src[i0], 4, eta[i0:i0 + 4])
    x = torch.empty_like(eta)
    prm = P.laph_dirac(CFG.m0, CFG.xi, CFG.csw, CFG.bc_t)
    sv = P.solver_params(tol=CFG.solve_tol, maxiter=6000, precision="f16", block_rhs=8,
                         solver=P.LAPH_SOLVER_BICGSTAB)
    sts = P.dirac_solve(L.ctx, dev(field), prm, eta, x, n, sv)
    assert all(q.status == 0 for q in sts)
    coef = torch.empty((n, NT, 4, NV), dtype=torch.complex128, device="cuda")
    P.sink_project(L.ctx, Vd, NV, x, n, coef)
    got = host(coef)[:, SLICES]
    L.close()
    worst = 0.0
    for i in range(n):
        ref = np.array(g["coef"][i]).view(np.complex128).reshape(len(SLICES), 4, NV)
        err = np.abs(got[i] - ref).max() / np.abs(ref).max()
        worst = max(worst, err)
        say("  source", src[i], "iters", sts[i].iters, "coefficient max rel err", err)
        assert err <= 1e-8
    say("  worst", worst)

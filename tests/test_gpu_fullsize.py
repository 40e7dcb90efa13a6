"""Parity at the production size, 24^3 x 128 (the benchmark's workload and launch
configuration), against the oracle.

At this size the oracle computes what it can in seconds and checks the rest by properties
that hold at any size:
* noise and dilution are bit-exact (Sec. IV noise, Sec. II dilution);
* the FP64 even-odd Dirac operator matches the oracle's K on the whole lattice to 1e-13;
* sources built from the GPU's own LapH eigenvectors match the oracle's sources on them;
* the benchmark's solve (FP16 inner vectors, 32 right-hand sides, FP64 reliable updates)
  of those sources reaches the true residual 1e-10 measured by the oracle's own Omega on
  every one of the 32;
* sink projection on those eigenvectors matches the oracle's sums;
* the LapH eigenpairs (stout smearing, Chebyshev-accelerated Lanczos) match the oracle's
  on a sampled slice, and every slice's eigenvectors satisfy the oracle Laplacian's
  eigen-equation.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host, rel_err, say

pytestmark = pytest.mark.gpu

CFG = synth.CONFIGS["ns24_nt128"]
NS, NT, NV = CFG.ns, CFG.nt, CFG.nv


@pytest.fixture(scope="module")
def P():
    import paper_1104_3870_amd as P

    P.lib()
    return P


@pytest.fixture(scope="module")
def field():
    say("generating the 24^3 x 128 field")
    return synth.gauge_field(NS, NT, CFG.eps, CFG.seed)


@pytest.fixture(scope="module")
def dirac(field):
    say("oracle Dirac operator at 24^3 x 128")
    return oracle.Dirac(field, CFG.m0, CFG.xi, CFG.csw, CFG.bc_t)


@pytest.fixture(scope="module")
def gpu_eig(P, field):
    """Stout smearing (10 steps) and the N_v = 112 lowest eigenpairs of every slice with the
    paper's Lanczos settings (Krylov 160, Chebyshev T_8, lambda_L = 15, lambda_C = 0.5,
    tol 1e-9); the device tensor stays resident, its host copy serves the oracle."""
    import torch

    say("GPU eigenvectors at 24^3 x 128")
    L = P.Lattice(NS, NT)
    evals = np.zeros((NT, NV))
    evecs = torch.empty((NT, NV, NS, NS, NS, 3), dtype=torch.complex128, device="cuda")
    st = P.laph_eigvecs(L.ctx, dev(field), CFG.stout_rho, CFG.stout_steps, NV, evals, evecs, krylov=CFG.krylov,
                        cheb_order=CFG.cheb_order, lam_l=CFG.lam_l, lam_c=CFG.lam_c, tol=CFG.eig_tol,
                        max_restarts=60)
    say("  restarts", st.restarts, "max residual", st.max_residual, "orth", st.max_orth)
    return L, st, evals, evecs, host(evecs)


def test_noise_bitexact_fullsize(P):
    import torch

    L = P.Lattice(NS, NT)
    rho = torch.empty((NT, 4, NV), dtype=torch.complex128, device="cuda")
    P.laph_z4_noise(L.ctx, CFG.noise_s, CFG.noise_k, NV, rho)
    ref = oracle.z4_noise(CFG.noise_s, CFG.noise_k, NT, NV)
    assert np.array_equal(host(rho), ref)


def test_dirac_apply_fullsize(P, field, dirac):
    import torch

    say("FP64 K at 24^3 x 128")
    L = P.Lattice(NS, NT)
    psi = synth.random_spinor(NS, NT, 5)
    out = torch.empty(psi.shape, dtype=torch.complex128, device="cuda")
    prm = P.laph_dirac(CFG.m0, CFG.xi, CFG.csw, CFG.bc_t)
    P.laph_dirac_apply(L.ctx, dev(field), prm, P.LAPH_OP_K, dev(psi), out, 1)
    ref = dirac.K(psi)
    err = np.abs(host(out) - ref).max() / np.abs(ref).max()
    say("  max rel err", err)
    assert err < 1e-13


def test_source_solve_sink_fullsize(P, field, dirac, gpu_eig):
    """The benchmark's step on sources of source time 0: 4 spins x 8 LapH-interlace
    projectors on the GPU eigenvectors, FP16 inner vectors, 32 right-hand sides, solved by
    the production BiCGStab and by CG on the normal equations."""
    import torch

    L, _, _, Vd, basis = gpu_eig
    dil = P.laph_parse_dilution(CFG.dilution, NT, NV)
    nsrc = 32
    eta = torch.empty((nsrc, NT, NS, NS, NS, 4, 3), dtype=torch.complex128, device="cuda")
    P.make_diluted_source(L.ctx, Vd, NV, CFG.noise_s, CFG.noise_k, dil, 0, nsrc, eta)
    rho = oracle.z4_noise(CFG.noise_s, CFG.noise_k, NT, NV)
    sch = oracle.parse_dilution(CFG.dilution, NT, NV)
    eta_h = host(eta)
    for b in (0, 13, 31):
        ref = oracle.source(basis, rho, sch, b)
        err = np.abs(eta_h[b] - ref).max() / np.abs(ref).max()
        say("  source b", b, "max rel err", err)
        assert err < 1e-14
    prm = P.laph_dirac(CFG.m0, CFG.xi, CFG.csw, CFG.bc_t)
    # the production form (BiCGStab, the benchmark's settings), then CG on the normal equations
    for name, kind, delta in (("bicgstab", P.LAPH_SOLVER_BICGSTAB, 0.1), ("cgnr", P.LAPH_SOLVER_CGNR, 0.03)):
        say("solve 32 sources (f16, R = 32, %s)" % name)
        x = torch.empty_like(eta)
        sv = P.solver_params(tol=CFG.solve_tol, maxiter=6000, precision="f16", block_rhs=32, solver=kind,
                             reliable_delta=delta, use_graph=1)
        st = P.dirac_solve(L.ctx, dev(field), prm, eta, x, nsrc, sv)
        assert all(q.status == 0 and q.fallback_used == 0 for q in st)
        xh = host(x)
        del x
        worst = 0.0
        for r in range(nsrc):
            tr = dirac.true_residual(eta_h[r], xh[r])
            worst = max(worst, tr)
            assert tr <= 1e-10, (name, r, tr)
            assert abs(tr - st[r].true_resid) <= 1e-12
        say("  oracle true residual of all 32: max", worst, "iterations", [q.iters for q in st])
        del xh
    del eta_h, eta
    # sink projection on synthetic solutions (both sides get the same host data)
    X = synth.random_spinor(NS, NT, 9, nrhs=2)
    coef = torch.empty((2, NT, 4, NV), dtype=torch.complex128, device="cuda")
    P.sink_project(L.ctx, Vd, NV, dev(X), 2, coef)
    ref = np.stack([oracle.sink_project(basis, X[r]) for r in range(2)])
    err = rel_err(host(coef), ref)
    say("  sink rel err", err)
    assert err < 1e-13


def test_eigvecs_fullsize(P, field, gpu_eig):
    """The eigenpairs of the fixture: smeared field, eigen-equation on every slice,
    orthonormality and slice 0 against the oracle."""
    import torch

    L, st, evals, evecs, V = gpu_eig
    S = oracle.stout_spatial(field, CFG.stout_rho, CFG.stout_steps)
    # smeared field: GPU against oracle
    Sd = torch.empty_like(dev(field))
    P.laph_stout_smear(L.ctx, dev(field), CFG.stout_rho, CFG.stout_steps, Sd)
    serr = np.abs(host(Sd) - S).max()
    say("  stout max abs err", serr)
    assert serr < 1e-12
    # every slice: eigen-equation of the oracle Laplacian; orthonormality on sampled slices
    worst = 0.0
    for n in range(NV):
        v = np.ascontiguousarray(V[:, n])
        res = -oracle.laplacian(S, v) - evals[:, n][:, None, None, None, None] * v
        worst = max(worst, float(np.abs(res).max()))
    say("  max |(-Lap) v - lambda v| over all slices", worst)
    assert worst < 1e-6
    for t in (0, 63, 127):
        Vt = V[t].reshape(NV, -1)
        assert np.abs(Vt.conj() @ Vt.T - np.eye(NV)).max() < 1e-10
    # slice 0 against the oracle's eigenpairs (ARPACK on the oracle Laplacian)
    ev_ref, _ = oracle.laph_eigpairs(S, NV, slices=[0], extra=1)
    err = np.abs(evals[0] - ev_ref[0, :NV]).max()
    say("  slice 0 eigenvalue max abs err", err)
    assert err < 1e-7

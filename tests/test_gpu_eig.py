"""GPU LapH eigenvectors (Sec. IV: KSRL with Chebyshev acceleration) against the plain
definition (Sec. II: the N_v lowest eigenpairs of -Lap per slice of the stout-smeared
field), computed by the oracle with dense LAPACK eigh.

Eigenvalues must agree to 1e-9 (relative to |Lap| <= 12).  Eigenvectors are compared
after the phase convention where the neighbouring gaps exceed 1e-6; inside a
near-degenerate cluster the cluster projectors are compared instead (the vectors
themselves are not unique); where the N_v cut falls inside a cluster, the GPU's vectors of
that cluster must lie in the space of the oracle's whole cluster."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1104_3870_amd as P

    P.lib()
    return P


def _compare(ev_gpu, V_gpu, ev_ref, V_ref, nv, tol_val=1e-9, tol_vec=1e-6):
    """ev_ref, V_ref hold nv + extra oracle pairs, so that the cluster the N_v cut falls in
    is complete on the oracle side."""
    assert np.abs(ev_gpu - ev_ref[:nv]).max() < tol_val
    m = len(ev_ref)
    # clusters by gap 1e-6 over all oracle pairs
    edges = [0] + [i for i in range(1, m) if ev_ref[i] - ev_ref[i - 1] > 1e-6] + [m]
    cut = 0
    for a, b in zip(edges, edges[1:]):
        if a >= nv:
            break
        A = V_gpu[a:min(b, nv)].reshape(min(b, nv) - a, -1)
        B = V_ref[a:b].reshape(b - a, -1)
        if b <= nv:
            if b - a == 1:
                assert np.linalg.norm(A - B) < tol_vec
            else:
                PA = A.T @ A.conj()
                PB = B.T @ B.conj()
                assert np.linalg.norm(PA - PB) < tol_vec
        else:
            # the cut at N_v falls inside this cluster: the GPU's vectors of it must lie in
            # the space of the oracle's whole cluster, |(1 - P_cluster) V_gpu| small
            assert b < m, "cluster at the cut not closed by the extra oracle pairs"
            resid = A.T - B.T @ (B.conj() @ A.T)
            assert np.linalg.norm(resid) < tol_vec
            cut += 1
    return cut


@pytest.mark.parametrize("ns,nt,eps,nv,m,lamc,steps", [(4, 8, 0.3, 8, 48, 2.5, 2), (6, 4, 0.5, 12, 40, 1.5, 2),
                                                       (8, 4, 0.4, 20, 60, 1.0, 3)])
def test_eigvecs_parity(P, ns, nt, eps, nv, m, lamc, steps):
    import torch

    say("eig", ns, nt, eps, nv, m)
    U = synth.gauge_field(ns, nt, eps, 1)
    S = oracle.stout_spatial(U, 0.1, steps)
    ev_ref, V_ref = oracle.laph_eigpairs(S, nv + 12)
    L = P.Lattice(ns, nt)
    evals = np.zeros((nt, nv))
    evecs = torch.empty((nt, nv, ns, ns, ns, 3), dtype=torch.complex128, device="cuda")
    st = P.laph_eigvecs(L.ctx, dev(U), 0.1, steps, nv, evals, evecs, krylov=m, lam_c=lamc, tol=1e-12,
                        max_restarts=200)
    say("  restarts", st.restarts, "matvecs", st.matvecs, "max_res", st.max_residual, "orth", st.max_orth,
        "gap", st.min_gap)
    assert st.max_residual < 1e-9
    assert st.max_orth < 1e-12
    V = host(evecs)
    cut = sum(_compare(evals[t], V[t], ev_ref[t], V_ref[t], nv) for t in range(nt))
    say("  slices whose N_v cut falls inside a cluster", cut)


def test_eigvecs_cut_cluster(P):
    """Free field under a random SU(3) gauge transformation: -Lap is unitarily equivalent
    to the free one, with exact shells (eigenvalue 0 three times, then 2 eighteen times on
    4^3), so N_v = 8 cuts the first excited shell.  Its five GPU vectors must lie in the
    oracle's 18-dimensional eigenspace; the three below the cut are compared as a
    projector."""
    import torch

    ns, nt, nv = 4, 4, 8
    U = synth.unit_gauge_field(ns, nt)
    G = synth.gauge_transform_field(ns, nt, 3)
    for mu, ax in enumerate((3, 2, 1, 0)):  # U'_mu(x) = G(x) U_mu(x) G(x + mu)^dag
        Gn = np.roll(G, -1, axis=ax)
        U[..., mu, :, :] = G @ U[..., mu, :, :] @ np.conj(np.swapaxes(Gn, -1, -2))
    S = oracle.stout_spatial(U, 0.1, 1)
    ev_ref, V_ref = oracle.laph_eigpairs(S, nv + 16)
    assert np.abs(ev_ref[:, 3:21] - 2.0).max() < 1e-12 and ev_ref[:, 21].min() > 2.5
    L = P.Lattice(ns, nt)
    evals = np.zeros((nt, nv))
    evecs = torch.empty((nt, nv, ns, ns, ns, 3), dtype=torch.complex128, device="cuda")
    st = P.laph_eigvecs(L.ctx, dev(U), 0.1, 1, nv, evals, evecs, krylov=48, lam_c=2.5, tol=1e-12,
                        max_restarts=200)
    say("  restarts", st.restarts, "max_res", st.max_residual, "orth", st.max_orth)
    assert st.max_residual < 1e-9 and st.max_orth < 1e-12
    V = host(evecs)
    cut = sum(_compare(evals[t], V[t], ev_ref[t], V_ref[t], nv) for t in range(nt))
    assert cut == nt

"""GPU parity of the baryon functions (Sec. III.A, Eq. baryonfunc) and the baryon
correlator with its six noise orderings (Eq. baryoncorr) against the oracle, through the
C-ABI; FP64 throughout.

Bars: the eigenvector tensor and the baryon functions against the oracle's full-field
definition within 1e-12 relative; the correlator contraction against the oracle's within
1e-13; the whole path on 4^3 x 8 with full dilution (three LapH vectors) within 1e-8 of
the brute-force six-term Wick contraction of the dense quark line (the solves stop at
true residual 1e-10)."""
import itertools

import numpy as np
import pytest

import oracle
import synth
import wick
from gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1104_3870_amd as P

    P.lib()
    return P


def _basis(ns, nt, nv, seed):
    rng = np.random.default_rng(seed)
    n = ns ** 3 * 3
    V = np.empty((nt, nv, ns, ns, ns, 3), dtype=np.complex128)
    for t in range(nt):
        q, _ = np.linalg.qr(rng.normal(size=(n, nv)) + 1j * rng.normal(size=(n, nv)))
        V[t] = q.T.reshape(nv, ns, ns, ns, 3)
    return V


def _tensor(seed, sparse=False):
    r = np.random.default_rng(seed)
    c = r.normal(size=(4, 4, 4)) + 1j * r.normal(size=(4, 4, 4))
    if sparse:
        mask = np.zeros((4, 4, 4), dtype=bool)
        for idx in r.choice(64, size=2, replace=False):
            mask.flat[idx] = True
        c = np.where(mask, c, 0)
    return c


def _unit_coef(nt, nv, n):
    """coefficients of V_n placed in spin 0 on every slice"""
    f = np.zeros((nt, 4, nv), dtype=np.complex128)
    f[:, 0, n] = 1.0
    return f


@pytest.mark.parametrize("ns,nt,nv,k", [(4, 2, 5, (1, 0, 2)), (4, 2, 19, (0, 0, 0)), (4, 2, 100, (0, 1, 3)),
                                        (4, 2, 140, (1, 1, 0))])
def test_baryon_tensor_parity(P, ns, nt, nv, k):
    """T[t][n1][n2][n3] against Eq. baryonfunc with single-vector fields V_n in spin 0
    and c = delta at (0, 0, 0); nv = 19 spans two 16-wide tiles with a ragged tail, nv = 100
    seven tiles whose pairs take two blocks per n1 (the kernel form that loads each stage
    one stage ahead), nv = 140 nine tiles (more than 128 rows: the form that stages
    directly); sampled triples in every order, with repeated indices (zero) among them."""
    import torch

    say("baryon tensor", ns, nt, nv, k)
    V = _basis(ns, nt, nv, 1)
    L = P.Lattice(ns, nt)
    T = torch.empty((nt, nv, nv, nv), dtype=torch.complex128, device="cuda")
    P.laph_baryon_tensor(L.ctx, dev(V), nv, k, T)
    got = host(T)
    L.close()
    c = np.zeros((4, 4, 4))
    c[0, 0, 0] = 1.0
    if nv < 10:
        trip = list(itertools.product(range(nv), repeat=3))
    elif nv < 40:
        trip = [(0, 5, 17), (18, 3, 16), (16, 17, 18), (7, 7, 2), (4, 18, 0)]
    else:
        base = [(0, 15, 16), (99, 50, 1), (31, 32, 95), (96, 97, 98), (14, 99, 60), (63, 64, 65), (5, 5, 40)]
        if nv > 128:
            base += [(0, 128, 139), (130, 131, 17), (127, 128, 129), (112, 139, 138)]
        trip = sorted({q for b in base for q in itertools.permutations(b)})
    need = sorted({n for q in trip for n in q})
    fields = {n: oracle.smeared_field(V, _unit_coef(nt, nv, n)) for n in need}
    scale = np.abs(got).max()
    for n1, n2, n3 in trip:
        ref = oracle.baryon_function(fields[n1], fields[n2], fields[n3], c, k)
        assert np.abs(got[:, n1, n2, n3] - ref).max() <= 1e-12 * scale, (n1, n2, n3)


@pytest.mark.parametrize("n1,n2,n3", [(2, 3, 2), (1, 1, 1), (5, 2, 3)])
def test_baryon_function_parity(P, n1, n2, n3):
    import torch

    ns, nt, nv, k = 4, 4, 6, (2, 1, 0)
    V = _basis(ns, nt, nv, 2)
    r = np.random.default_rng(3)
    f = [r.normal(size=(n, nt, 4, nv)) + 1j * r.normal(size=(n, nt, 4, nv)) for n in (n1, n2, n3)]
    c = _tensor(4)
    L = P.Lattice(ns, nt)
    T = torch.empty((nt, nv, nv, nv), dtype=torch.complex128, device="cuda")
    P.laph_baryon_tensor(L.ctx, dev(V), nv, k, T)
    out = torch.empty((nt, n1, n2, n3), dtype=torch.complex128, device="cuda")
    P.laph_baryon_function(L.ctx, T, nv, c, dev(f[0]), n1, dev(f[1]), n2, dev(f[2]), n3, out)
    got = host(out)
    L.close()
    full = [[oracle.smeared_field(V, fk[i]) for i in range(fk.shape[0])] for fk in f]
    ref = np.empty_like(got)
    for i, j, l in itertools.product(range(n1), range(n2), range(n3)):
        ref[:, i, j, l] = oracle.baryon_function(full[0][i], full[1][j], full[2][l], c, k)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_baryon_correlator_contraction(P):
    import torch

    nt, n, t0 = 4, 5, 2
    r = np.random.default_rng(5)
    snk = r.normal(size=(nt, n, n, n)) + 1j * r.normal(size=(nt, n, n, n))
    src = r.normal(size=(6, nt, n, n, n)) + 1j * r.normal(size=(6, nt, n, n, n))
    L = P.Lattice(4, nt)
    out = torch.empty(nt, dtype=torch.complex128, device="cuda")
    P.laph_baryon_correlator(L.ctx, dev(snk), dev(src), n, t0, out)
    ref = oracle.baryon_correlator(snk, list(src), t0)
    assert np.abs(host(out) - ref).max() <= 1e-13 * np.abs(ref).max()
    L.close()


def test_baryon_correlator_end_to_end_exact(P):
    """GPU path (diluted sources for three noises, FP16 multi-RHS solves, sink projections,
    the eigenvector tensor, baryon functions of the sinks and of the sources in the six
    noise orderings, the correlator) with full dilution against the six-term Wick
    contraction of the dense quark line S Omega^-1 S."""
    import torch

    cfg = synth.CONFIGS["ns4_nt8"]
    nv, nt, ns = 3, cfg.nt, cfg.ns
    U = synth.gauge_field(ns, nt, cfg.eps, cfg.seed)
    S = oracle.stout_spatial(U, cfg.stout_rho, cfg.stout_steps)
    ev, V = oracle.laph_eigpairs(S, nv)
    D = oracle.Dirac(U, cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    B = oracle.laph_basis(V)
    Q = B @ (B.conj().T @ oracle.dense_solve(D, B)) @ B.conj().T
    t0, k = 3, (1, 0, 0)
    c, cp = _tensor(8, sparse=True), _tensor(9, sparse=True)
    L = P.Lattice(ns, nt)
    Ud, Vd = dev(U), dev(V)
    dil = P.laph_parse_dilution("TF,SF,LF", nt, nv)
    n0 = 4 * nv
    b0 = t0 * n0
    prm = P.laph_dirac(cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    shape = (n0, nt, ns, ns, ns, 4, 3)
    sinks, srcs = [], []
    for s in (1, 2, 3):
        eta = torch.empty(shape, dtype=torch.complex128, device="cuda")
        x = torch.empty_like(eta)
        P.make_diluted_source(L.ctx, Vd, nv, s, 5, dil, b0, n0, eta)
        st = P.dirac_solve(L.ctx, Ud, prm, eta, x, n0, P.solver_params(precision="f16", block_rhs=16,
                                                                        solver=P.LAPH_SOLVER_CGNR))
        assert all(q.status == 0 for q in st)
        co = torch.empty((n0, nt, 4, nv), dtype=torch.complex128, device="cuda")
        P.sink_project(L.ctx, Vd, nv, x, n0, co)
        sinks.append(co)
        q = torch.empty_like(co)
        P.laph_quark_source(L.ctx, nv, s, 5, dil, b0, n0, q)
        srcs.append(q)
    T = torch.empty((nt, nv, nv, nv), dtype=torch.complex128, device="cuda")
    P.laph_baryon_tensor(L.ctx, Vd, nv, k, T)
    snk = torch.empty((nt, n0, n0, n0), dtype=torch.complex128, device="cuda")
    P.laph_baryon_function(L.ctx, T, nv, c, sinks[0], n0, sinks[1], n0, sinks[2], n0, snk)
    src = torch.empty((6, nt, n0, n0, n0), dtype=torch.complex128, device="cuda")
    for p, (order, sign) in enumerate(oracle.BARYON_PERMUTATIONS):
        P.laph_baryon_function(L.ctx, T, nv, cp, srcs[order[0]], n0, srcs[order[1]], n0, srcs[order[2]], n0, src[p])
    corr = torch.empty(nt, dtype=torch.complex128, device="cuda")
    P.laph_baryon_correlator(L.ctx, snk, src, n0, t0, corr)
    got = host(corr)
    L.close()
    ref = wick.baryon_wick(Q, ns, nt, t0, c, cp, k)
    assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max()

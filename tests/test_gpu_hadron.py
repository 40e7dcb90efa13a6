"""GPU parity of the hadron building blocks (Sec. II: quark sources, the gamma_5-Hermitian
estimate; Sec. III.B: meson functions, the meson correlator and its internal-line term)
against the oracle, through the C-ABI.

Bars: the quark-source coefficients (signs and Z4 values times 0/1) bit-exact; meson
functions from coefficients against the oracle's definition on full fields within 1e-12
relative (FP64; the reduction to the LapH index uses only the orthonormality of V_s);
the end-to-end correlator on 4^3 x 8 with full dilution, from the GPU's own sources,
mixed-precision solves and sink projections, within 1e-8 of the brute-force Wick
contraction of the dense quark line (the solves stop at true residual 1e-10)."""
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


def _basis(ns, nt, nv, seed):
    rng = np.random.default_rng(seed)
    n = ns ** 3 * 3
    V = np.empty((nt, nv, ns, ns, ns, 3), dtype=np.complex128)
    for t in range(nt):
        q, _ = np.linalg.qr(rng.normal(size=(n, nv)) + 1j * rng.normal(size=(n, nv)))
        V[t] = q.T.reshape(nv, ns, ns, ns, 3)
    return V


def _coefs(n, nt, nv, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, nt, 4, nv)) + 1j * rng.normal(size=(n, nt, 4, nv))


def _g5g4():
    return oracle.gamma(4) @ oracle.gamma(3)


@pytest.mark.parametrize("spec,nt,nv,bar", [("TF,SF,LI4", 8, 8, 0), ("TI4,SB2,LF", 8, 12, 1), ("TB2,S1,LI3", 4, 9, 1)])
def test_quark_source_bitexact(P, spec, nt, nv, bar):
    import torch

    L = P.Lattice(4, nt)
    dil = P.laph_parse_dilution(spec, nt, nv)
    nb = P.laph_dilution_count(dil, nt, nv)
    out = torch.empty((nb, nt, 4, nv), dtype=torch.complex128, device="cuda")
    P.laph_quark_source(L.ctx, nv, 9, 4, dil, 0, nb, out, bar=bar)
    got = host(out)
    rho = oracle.z4_noise(9, 4, nt, nv)
    sch = oracle.parse_dilution(spec, nt, nv)
    for b in range(nb):
        ref = oracle.dilution_projector(sch, nt, nv, b) * rho
        if bar:
            ref = -oracle.spin_apply(_g5g4(), ref)
        assert np.array_equal(got[b], ref), b
    L.close()


def test_spin_apply(P):
    import torch

    L = P.Lattice(4, 8)
    a = _coefs(3, 8, 7, 1)
    S = np.random.default_rng(2).normal(size=(4, 4)) + 0j
    out = torch.empty(a.shape, dtype=torch.complex128, device="cuda")
    P.laph_spin_apply(L.ctx, S, dev(a), 3, 7, out)
    ref = oracle.spin_apply(S, a)
    assert np.abs(host(out) - ref).max() <= 1e-14 * np.abs(ref).max()
    ad = dev(a)
    P.laph_spin_apply(L.ctx, _g5g4(), ad, 3, 7, ad)  # in place
    assert np.abs(host(ad) - oracle.spin_apply(_g5g4(), a)).max() == 0
    L.close()


@pytest.mark.parametrize("ns,nt,nv,n1,n2", [(4, 8, 8, 21, 18), (6, 4, 12, 5, 33), (4, 2, 3, 1, 1)])
def test_meson_function_parity(P, ns, nt, nv, n1, n2):
    """M[t][i][j] from coefficients (LDS-tiled product, ragged 16 x 16 tiles) against the
    oracle's Eq. mesonfunc on the full fields V_s a_i and V_s b_j."""
    import torch

    say("meson", ns, nt, nv, n1, n2)
    V = _basis(ns, nt, nv, 3)
    a = _coefs(n1, nt, nv, 4)
    b = _coefs(n2, nt, nv, 5)
    c = np.random.default_rng(6).normal(size=(4, 4)) + 1j * np.random.default_rng(7).normal(size=(4, 4))
    L = P.Lattice(ns, nt)
    out = torch.empty((nt, n1, n2), dtype=torch.complex128, device="cuda")
    P.laph_meson_function(L.ctx, c, dev(a), n1, dev(b), n2, nv, out)
    got = host(out)
    fa = [oracle.smeared_field(V, a[i]) for i in range(n1)]
    fb = [oracle.smeared_field(V, b[j]) for j in range(n2)]
    ref = np.empty((nt, n1, n2), dtype=np.complex128)
    for i in range(n1):
        for j in range(n2):
            ref[:, i, j] = oracle.meson_function(fa[i], fb[j], c)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    n = min(n1, n2)  # diagonal form on the first n fields of each side
    d = torch.empty((nt, n), dtype=torch.complex128, device="cuda")
    P.laph_meson_function(L.ctx, c, dev(a[:n]), n, dev(b[:n]), n, nv, d, diag=True)
    refd = np.stack([ref[:, i, i] for i in range(n)], axis=1)
    assert np.abs(host(d) - refd).max() <= 1e-12 * np.abs(refd).max()
    L.close()


def test_correlator_terms(P):
    """Eq. mesoncorr's two terms from given meson functions (definition written out)."""
    import torch

    nt, n1, n2, t0 = 8, 13, 7, 3
    rng = np.random.default_rng(8)
    snk = rng.normal(size=(nt, n1, n2)) + 1j * rng.normal(size=(nt, n1, n2))
    src = rng.normal(size=(nt, n1, n2)) + 1j * rng.normal(size=(nt, n1, n2))
    L = P.Lattice(4, nt)
    out = torch.empty(nt, dtype=torch.complex128, device="cuda")
    P.laph_meson_correlator(L.ctx, dev(snk), dev(src), n1, n2, t0, out)
    ref = -np.einsum("tij,ij->t", snk, src[t0].conj())
    assert np.abs(host(out) - ref).max() <= 1e-13 * np.abs(ref).max()
    ds, dr = snk[:, :, 0].copy(), src[:, :, 0].copy()
    P.laph_meson_correlator(L.ctx, dev(ds), dev(dr), n1, n1, t0, out, diag=True)
    ref = ds.sum(axis=1) * np.conj(dr[t0].sum())
    assert np.abs(host(out) - ref).max() <= 1e-13 * np.abs(ref).max()
    L.close()


@pytest.fixture(scope="module")
def exact_ns4(P):
    cfg = synth.CONFIGS["ns4_nt8"]
    U = synth.gauge_field(cfg.ns, cfg.nt, cfg.eps, cfg.seed)
    S = oracle.stout_spatial(U, cfg.stout_rho, cfg.stout_steps)
    ev, V = oracle.laph_eigpairs(S, cfg.nv)
    D = oracle.Dirac(U, cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    B = oracle.laph_basis(V)
    tau = B.conj().T @ oracle.dense_solve(D, B)
    Q = B @ tau @ B.conj().T
    return cfg, U, V, Q


def _gpu_sinks(P, L, cfg, Ud, Vd, dil, s, k, b_first, n):
    """Sink coefficients of n diluted sources (FP16 inner solves, 32 right-hand sides)."""
    import torch

    shape = (n, cfg.nt, cfg.ns, cfg.ns, cfg.ns, 4, 3)
    eta = torch.empty(shape, dtype=torch.complex128, device="cuda")
    x = torch.empty_like(eta)
    coef = torch.empty((n, cfg.nt, 4, cfg.nv), dtype=torch.complex128, device="cuda")
    P.make_diluted_source(L.ctx, Vd, cfg.nv, s, k, dil, b_first, n, eta)
    prm = P.laph_dirac(cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    st = P.dirac_solve(L.ctx, Ud, prm, eta, x, n, P.solver_params(precision="f16", block_rhs=32,
                                                                   solver=P.LAPH_SOLVER_CGNR))
    assert all(q.status == 0 and q.true_resid <= 1e-10 for q in st)
    P.sink_project(L.ctx, Vd, cfg.nv, x, n, coef)
    return coef


@pytest.mark.parametrize("gam", ["g5", "random"])
def test_meson_correlator_end_to_end_exact(P, exact_ns4, gam):
    """The GPU path (diluted sources, FP16 multi-RHS solves, sink projections, barred
    sources and sinks, meson functions, correlator) with full dilution against the
    brute-force Wick contraction of S Omega^-1 S: connected term for every sink slice and
    the internal-line term of isoscalars."""
    import torch

    cfg, U, V, Q = exact_ns4
    nt, nv, V3 = cfg.nt, cfg.nv, cfg.ns ** 3
    c = oracle.gamma(4) if gam == "g5" else np.random.default_rng(3).normal(size=(4, 4)) + 0.5j
    cp = oracle.gamma(4) if gam == "g5" else np.random.default_rng(4).normal(size=(4, 4)) - 0.3j
    t0 = 2
    L = P.Lattice(cfg.ns, nt)
    Ud, Vd = dev(U), dev(V)
    dil = P.laph_parse_dilution(cfg.dilution, nt, nv)
    nb = P.laph_dilution_count(dil, nt, nv)
    n0 = 4 * nv  # projectors of one source time
    b0 = t0 * n0
    # connected: noise 1 (barred, gamma_5-Hermitian line) and noise 2, sources on t0
    phi1 = _gpu_sinks(P, L, cfg, Ud, Vd, dil, 1, 7, b0, n0)
    phi2 = _gpu_sinks(P, L, cfg, Ud, Vd, dil, 2, 7, b0, n0)
    P.laph_spin_apply(L.ctx, _g5g4(), phi1, n0, nv, phi1)  # varphi-bar_1
    rb1 = torch.empty((n0, nt, 4, nv), dtype=torch.complex128, device="cuda")
    r2 = torch.empty_like(rb1)
    P.laph_quark_source(L.ctx, nv, 1, 7, dil, b0, n0, rb1, bar=True)
    P.laph_quark_source(L.ctx, nv, 2, 7, dil, b0, n0, r2)
    msnk = torch.empty((nt, n0, n0), dtype=torch.complex128, device="cuda")
    msrc = torch.empty_like(msnk)
    P.laph_meson_function(L.ctx, c, phi1, n0, phi2, n0, nv, msnk)
    P.laph_meson_function(L.ctx, cp, rb1, n0, r2, n0, nv, msrc)
    conn = torch.empty(nt, dtype=torch.complex128, device="cuda")
    P.laph_meson_correlator(L.ctx, msnk, msrc, n0, n0, t0, conn)
    # internal line: every projector, noise 1 at the sink slices and noise 2 at t0
    f1 = _gpu_sinks(P, L, cfg, Ud, Vd, dil, 1, 7, 0, nb)
    f2 = _gpu_sinks(P, L, cfg, Ud, Vd, dil, 2, 7, 0, nb)
    q1 = torch.empty((nb, nt, 4, nv), dtype=torch.complex128, device="cuda")
    q2 = torch.empty_like(q1)
    P.laph_quark_source(L.ctx, nv, 1, 7, dil, 0, nb, q1)
    P.laph_quark_source(L.ctx, nv, 2, 7, dil, 0, nb, q2)
    dsnk = torch.empty((nt, nb), dtype=torch.complex128, device="cuda")
    dsrc = torch.empty_like(dsnk)
    P.laph_meson_function(L.ctx, c, q1, nb, f1, nb, nv, dsnk, diag=True)
    P.laph_meson_function(L.ctx, cp, f2, nb, q2, nb, nv, dsrc, diag=True)
    disc = torch.empty(nt, dtype=torch.complex128, device="cuda")
    P.laph_meson_correlator(L.ctx, dsnk, dsrc, nb, nb, t0, disc, diag=True)
    L.close()
    Qr = Q.reshape(nt, V3, 4, 3, nt, V3, 4, 3)
    conn_bf = np.array([-np.einsum("ab,cd,ucvxaw,xbwudv->", c, cp.conj(), Qr[t0, :, :, :, tf], Qr[tf, :, :, :, t0])
                        for tf in range(nt)])
    tr_snk = np.array([np.einsum("ab,xbwxaw->", c, Qr[tf, :, :, :, tf]) for tf in range(nt)])
    tr_src = np.einsum("cd,xcwxdw->", cp.conj(), Qr[t0, :, :, :, t0])
    for got, ref in ((host(conn), conn_bf), (host(disc), tr_snk * tr_src)):
        assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max()


@pytest.mark.parametrize("name,spec,bs", [("ns4_nt8", "TI4,SF,LI4", (0, 9, 63)), ("ns16_nt32", "TI16,SF,LI8", (5, 300))])
def test_same_time_lines_parity(P, name, spec, bs):
    """Same-time (t_F -> t_F) quark lines of an interlaced time dilution (Sec. II; the
    paper's (TI16, SF, LI8) on the 16^3 x 32 workload): the internal-line meson function
    M^[bb](varrho^[b], varphi^[b]; t) of sampled projectors b from the GPU path against the
    oracle's, which solves the same sources with its own CG (true residual 1e-12) and
    evaluates Eq. mesonfunc on the full fields; both sides use the same basis V_s (the
    oracle's eigenvectors on 4^3 x 8, an orthonormal random basis per slice on 16^3 x 32)."""
    import torch

    cfg = synth.CONFIGS[name]
    say("same-time", name, spec, bs)
    U = synth.gauge_field(cfg.ns, cfg.nt, cfg.eps, cfg.seed)
    if cfg.ns == 4:
        S = oracle.stout_spatial(U, cfg.stout_rho, cfg.stout_steps)
        ev, V = oracle.laph_eigpairs(S, cfg.nv)
    else:  # any orthonormal basis per slice serves the parity check (eigensolves are slow here)
        V = _basis(cfg.ns, cfg.nt, cfg.nv, 12)
    D = oracle.Dirac(U, cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    rho = oracle.z4_noise(cfg.noise_s, cfg.noise_k, cfg.nt, cfg.nv)
    sch = oracle.parse_dilution(spec, cfg.nt, cfg.nv)
    c = oracle.gamma(4)
    L = P.Lattice(cfg.ns, cfg.nt)
    Ud, Vd = dev(U), dev(V)
    dil = P.laph_parse_dilution(spec, cfg.nt, cfg.nv)
    for b in bs:
        coef = _gpu_sinks(P, L, cfg, Ud, Vd, dil, cfg.noise_s, cfg.noise_k, b, 1)
        q = torch.empty_like(coef)
        P.laph_quark_source(L.ctx, cfg.nv, cfg.noise_s, cfg.noise_k, dil, b, 1, q)
        d = torch.empty((cfg.nt, 1), dtype=torch.complex128, device="cuda")
        P.laph_meson_function(L.ctx, c, q, 1, coef, 1, cfg.nv, d, diag=True)
        eta = oracle.source(V, rho, sch, b)
        x, it, tr = D.solve(eta, tol=1e-12)
        ref = oracle.meson_function(oracle.quark_source(V, rho, sch, b), oracle.quark_sink(V, x), c)
        got = host(d)[:, 0]
        assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max(), b
    L.close()

"""Pins of the oracle's hadron functions (Sec. II: quark sources and sinks and the
gamma_5-Hermitian estimate; Sec. III.B: the meson function and the meson correlator).

The strongest pin: with full time x spin x LapH dilution the stochastic LapH estimate of
every quark line is exact for any noise (Sec. II), so the meson correlator assembled from
meson functions of quark sources and sinks (Eq. mesoncorr) must equal the Wick contraction
of the smeared quark line Q = S Omega^-1 S computed by brute force in the full lattice
space from a dense LU inverse (the sums over sites, colours and spins written out), on the
4^3 x 8 workload.  A wrong conjugation, sign of the barred fields, spin index order or
pairing fails it.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = []


@pytest.fixture(scope="module")
def setup():
    cfg = synth.CONFIGS["ns4_nt8"]
    U = synth.gauge_field(cfg.ns, cfg.nt, cfg.eps, cfg.seed)
    S = oracle.stout_spatial(U, cfg.stout_rho, cfg.stout_steps)
    ev, V = oracle.laph_eigpairs(S, cfg.nv)
    D = oracle.Dirac(U, cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    B = oracle.laph_basis(V)  # [12 V, Nt 4 Nv]
    X = oracle.dense_solve(D, B)  # Omega^-1 V_s
    tau = B.conj().T @ X
    Q = B @ tau @ B.conj().T  # S Omega^-1 S with S = V_s V_s^dag
    sch = oracle.parse_dilution(cfg.dilution, cfg.nt, cfg.nv)
    return cfg, U, V, D, B, X, Q, sch


def _shape(cfg):
    return (cfg.nt, cfg.ns, cfg.ns, cfg.ns, 4, 3)


def _sink(cfg, V, X, rho, b, bar=False):
    """Quark sink of projector b for full dilution: X^[b] = Omega^-1 V_s e_b rho_b."""
    xb = (X[:, b] * rho.ravel()[b]).reshape(_shape(cfg))
    return oracle.quark_sink(V, xb, bar=bar)


def _rand_gamma(seed):
    r = np.random.default_rng(seed)
    return r.normal(size=(4, 4)) + 1j * r.normal(size=(4, 4))


def test_gamma5_hermitian_estimates_agree(setup):
    """Eqs. laphprop and laphpropg5: with full dilution sum_b varphi^[b] varrho^[b]dag and
    sum_b varrho-bar^[b] varphi-bar^[b]dag both equal S Omega^-1 S (one noise)."""
    cfg, U, V, D, B, X, Q, sch = setup
    rho = oracle.z4_noise(3, 1, cfg.nt, cfg.nv)
    n = 12 * cfg.ns ** 3 * cfg.nt
    Q1 = np.zeros((n, n), dtype=np.complex128)
    Q2 = np.zeros_like(Q1)
    phis, rhos, phib, rhob = [], [], [], []
    for b in range(oracle.dilution_count(sch, cfg.nt, cfg.nv)):
        phis.append(_sink(cfg, V, X, rho, b).ravel())
        phib.append(_sink(cfg, V, X, rho, b, bar=True).ravel())
        rhos.append(oracle.quark_source(V, rho, sch, b).ravel())
        rhob.append(oracle.quark_source(V, rho, sch, b, bar=True).ravel())
    F, R, Fb, Rb = (np.array(a).T for a in (phis, rhos, phib, rhob))
    Q1 = F @ R.conj().T
    Q2 = Rb @ Fb.conj().T
    scale = np.abs(Q).max()
    assert np.abs(Q1 - Q).max() <= 1e-12 * scale
    assert np.abs(Q2 - Q).max() <= 1e-12 * scale


def test_meson_function_conjugate_and_gauge(setup):
    """conj M(f1, f2; c, k) = M(f2, f1; c^dag, -k), and M is unchanged when both fields are
    rotated by the same site-local SU(3) matrices (colours contracted with delta_ab)."""
    cfg = setup[0]
    f1 = synth.random_spinor(cfg.ns, cfg.nt, 5)
    f2 = synth.random_spinor(cfg.ns, cfg.nt, 6)
    c = _rand_gamma(1)
    for k in ((0, 0, 0), (1, 0, 2)):
        m12 = oracle.meson_function(f1, f2, c, k=k)
        m21 = oracle.meson_function(f2, f1, c.conj().T, k=tuple(-q for q in k))
        assert np.abs(m12.conj() - m21).max() <= 1e-13 * np.abs(m12).max()
    G = synth.gauge_transform_field(cfg.ns, cfg.nt, 4)
    g1 = np.einsum("tzyxab,tzyxsb->tzyxsa", G, f1)
    g2 = np.einsum("tzyxab,tzyxsb->tzyxsa", G, f2)
    m = oracle.meson_function(f1, f2, c, k=(1, 1, 0))
    mg = oracle.meson_function(g1, g2, c, k=(1, 1, 0))
    assert np.abs(m - mg).max() <= 1e-12 * np.abs(m).max()


def test_meson_function_momentum_and_displacement(setup):
    """A plane wave exp(i q.x) in the second field shifts the momentum: M(f1, e^{iq.x} f2; k)
    = M(f1, f2; k - q); displacements d1, d2 multiply by exp(-i p.(d1 + d2)/2); the spin
    matrix enters as c_{alpha beta} with alpha on f1 (a single unit entry picks one spin pair)."""
    cfg = setup[0]
    ns = cfg.ns
    f1 = synth.random_spinor(ns, cfg.nt, 7)
    f2 = synth.random_spinor(ns, cfg.nt, 8)
    c = _rand_gamma(2)
    t, z, y, x = np.meshgrid(*(np.arange(n) for n in (cfg.nt, ns, ns, ns)), indexing="ij")
    q = (1, 2, 3)
    wave = np.exp(2j * np.pi * (q[0] * x + q[1] * y + q[2] * z) / ns)[..., None, None]
    for k in ((1, 2, 3), (0, 1, 1)):
        lhs = oracle.meson_function(f1, wave * f2, c, k=k)
        rhs = oracle.meson_function(f1, f2, c, k=tuple(a - b for a, b in zip(k, q)))
        assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()
    k, d1, d2 = (1, 0, 2), (3, 0, 0), (0, -3, 3)
    ph = np.exp(-1j * 2 * np.pi / ns * sum(kk * (a + b) / 2 for kk, a, b in zip(k, d1, d2)))
    m0 = oracle.meson_function(f1, f2, c, k=k)
    md = oracle.meson_function(f1, f2, c, k=k, d1=d1, d2=d2)
    assert np.abs(md - ph * m0).max() <= 1e-12 * np.abs(m0).max()
    e = np.zeros((4, 4))
    e[1, 2] = 1.0
    direct = np.einsum("tzyxa,tzyxa->t", f1[..., 1, :].conj(), f2[..., 2, :])
    assert np.abs(oracle.meson_function(f1, f2, e) - direct).max() <= 1e-13 * np.abs(direct).max()


@pytest.mark.parametrize("gam", ["g5", "random"])
def test_meson_correlator_full_dilution_is_exact(setup, gam):
    """Eq. mesoncorr with full dilution equals the brute-force Wick contraction of
    Q = S Omega^-1 S: connected term -sum c_ab c'*_cd Q(t0 c, tF a) Q(tF b, t0 d), and the
    internal-line term [sum c_ab Tr Q(tF b, tF a)] [sum c'*_cd Tr Q(t0 c, t0 d)] (traces over
    sites and colours), for every sink slice tF."""
    cfg, U, V, D, B, X, Q, sch = setup
    if gam == "g5":
        c = oracle.gamma(4)
        cp = oracle.gamma(4)
    else:
        c, cp = _rand_gamma(3), _rand_gamma(4)
    t0 = 2
    nt, V3, nv = cfg.nt, cfg.ns ** 3, cfg.nv
    rho1 = oracle.z4_noise(1, 7, nt, nv)
    rho2 = oracle.z4_noise(2, 7, nt, nv)
    # projectors whose sources live on t0 (b_T = t0 for full time dilution): others give
    # source meson functions that vanish identically at t0
    bs = [b for b in range(oracle.dilution_count(sch, nt, nv)) if b // (4 * nv) == t0]
    sink_bar1 = {b: _sink(cfg, V, X, rho1, b, bar=True) for b in bs}
    sink2 = {b: _sink(cfg, V, X, rho2, b) for b in bs}
    src_bar1 = {b: oracle.quark_source(V, rho1, sch, b, bar=True) for b in bs}
    src2 = {b: oracle.quark_source(V, rho2, sch, b) for b in bs}
    conn = np.zeros(nt, dtype=np.complex128)
    for b1 in bs:
        for b2 in bs:
            msnk = oracle.meson_function(sink_bar1[b1], sink2[b2], c)
            msrc = oracle.meson_function(src_bar1[b1], src2[b2], cp)
            conn += -msnk * np.conj(msrc[t0])
    # internal-line term: sum over every projector (same noise at both ends of a line)
    all_b = range(oracle.dilution_count(sch, nt, nv))
    dsnk = sum(oracle.meson_function(oracle.quark_source(V, rho1, sch, b), _sink(cfg, V, X, rho1, b), c)
               for b in all_b)
    dsrc = sum(oracle.meson_function(_sink(cfg, V, X, rho2, b), oracle.quark_source(V, rho2, sch, b), cp)
               for b in all_b)
    disc = dsnk * np.conj(dsrc[t0])
    # brute force in the full space
    Qr = Q.reshape(nt, V3, 4, 3, nt, V3, 4, 3)
    conn_bf = np.empty(nt, dtype=np.complex128)
    trace_snk = np.empty(nt, dtype=np.complex128)
    for tf in range(nt):
        A = Qr[t0, :, :, :, tf]  # [x0, c, a0, x, a, col]
        Bq = Qr[tf, :, :, :, t0]  # [x, b, col, x0, d, a0]
        conn_bf[tf] = -np.einsum("ab,cd,ucvxaw,xbwudv->", c, cp.conj(), A, Bq)
        trace_snk[tf] = np.einsum("ab,xbwxaw->", c, Qr[tf, :, :, :, tf])
    trace_src = np.einsum("cd,xcwxdw->", cp.conj(), Qr[t0, :, :, :, t0])
    disc_bf = trace_snk * trace_src
    assert np.abs(conn - conn_bf).max() <= 1e-10 * np.abs(conn_bf).max()
    assert np.abs(disc - disc_bf).max() <= 1e-10 * np.abs(disc_bf).max()

"""Pins of the oracle's Dirac operator, solve, source and sink projection (CPU only).

The paper names the operator (an improved anisotropic clover action, Omega = gamma_4 K,
Sec. II) but does not print it; the frozen reading (chiral basis, anisotropic Wilson
hop with w_4 = 1 and w_k = 1/xi, clover with c_s = c_sw/xi and c_t = c_sw(1+1/xi)/2,
antiperiodic time) is pinned here by the free-field momentum-space form,
gamma_5-hermiticity (Sec. II, K^dag = gamma_5 K gamma_5), gauge covariance, the
abelian closed form of the clover term and dense LU.  The quark-line pins follow
Sec. II (exact zeros of full dilution: the diluted estimator of V^dag Omega^-1 V is
exact for any single noise) and Sec. IV (coefficients are gauge invariant).
"""
import numpy as np
import pytest

import oracle
import synth

XI = 3.5


def _transform_links(U, G):
    out = np.empty_like(U)
    for mu in range(4):
        Gp = np.roll(G, -1, axis=3 - mu)
        out[..., mu, :, :] = G @ U[..., mu, :, :] @ np.conj(np.swapaxes(Gp, -1, -2))
    return out


def _g(mu, psi):
    return np.einsum("ab,...bc->...ac", oracle.gamma(mu), psi)


def test_gamma_algebra():
    g = [oracle.gamma(m) for m in range(5)]
    for m in range(4):
        assert np.abs(g[m] - g[m].conj().T).max() == 0
        for n in range(4):
            anti = g[m] @ g[n] + g[n] @ g[m]
            assert np.abs(anti - 2 * (m == n) * np.eye(4)).max() < 1e-15
    assert np.abs(g[4] - np.diag([1, 1, -1, -1])).max() < 1e-15
    assert np.abs(g[0] @ g[1] @ g[2] @ g[3] - g[4]).max() < 1e-15


@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 0, 0, 0), (1, 2, 3, 1), (3, 1, 0, 2)])
def test_free_field_momentum_space(n):
    """U = 1: K u e^{ipx} = K(p) u e^{ipx}, K(p) = M(p) + i sum_mu gamma_mu w_mu sin p_mu,
    M(p) = m0 + sum_mu w_mu (1 - cos p_mu), antiperiodic p_4 = (2 n_4 + 1) pi / N_t."""
    ns, nt, m0 = 4, 6, -0.07
    U = synth.unit_gauge_field(ns, nt)
    D = oracle.Dirac(U, m0, XI, 1.0)
    w = np.array([1 / XI, 1 / XI, 1 / XI, 1.0])
    p = np.array([2 * np.pi * n[0] / ns, 2 * np.pi * n[1] / ns, 2 * np.pi * n[2] / ns,
                  (2 * n[3] + 1) * np.pi / nt])
    rng = np.random.default_rng(1)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    t, z, y, x = np.meshgrid(np.arange(nt), np.arange(ns), np.arange(ns), np.arange(ns), indexing="ij")
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    psi = ph[..., None, None] * u
    Kp = (m0 + np.sum(w * (1 - np.cos(p)))) * np.eye(4, dtype=complex)
    for mu in range(4):
        Kp = Kp + 1j * w[mu] * np.sin(p[mu]) * oracle.gamma(mu)
    ref = ph[..., None, None] * (Kp @ u)
    assert np.abs(D.K(psi) - ref).max() < 1e-13
    # K(p)^dag K(p) = M^2 + |s|^2 (gamma_mu Hermitian and anticommuting)
    s2 = np.sum((w * np.sin(p)) ** 2)
    M = m0 + np.sum(w * (1 - np.cos(p)))
    KK = D.K(D.K(psi), dagger=True)
    assert np.abs(KK - (M * M + s2) * psi).max() < 1e-12


def test_clover_zero_at_unit_field():
    A = oracle.clover(synth.unit_gauge_field(4, 4), -0.1, XI, 1.0)
    d = -0.1 + 1 + 3 / XI
    assert np.abs(A - d * np.eye(12)).max() < 1e-15


def test_clover_hermitian_and_chiral():
    U = synth.gauge_field(4, 4, 0.6, 2)
    A = oracle.clover(U, -0.1, XI, 1.0)
    assert np.abs(A - np.conj(np.swapaxes(A, -1, -2))).max() < 1e-15
    g5 = np.kron(oracle.gamma(4), np.eye(3))
    assert np.abs(A @ g5 - g5 @ A).max() < 1e-15
    assert np.abs(np.trace(A, axis1=-2, axis2=-1) - 12 * (-0.1 + 1 + 3 / XI)).max() < 1e-13


@pytest.mark.parametrize("plane", [(0, 1), (0, 3), (1, 2), (2, 3)])
def test_clover_abelian_closed_form(plane):
    """Constant abelian field strength in the (mu,nu) plane with colour charges (1,-1,0):
    every leaf equals e^{i q phi}, so F_mu,nu = diag(sin phi, -sin phi, 0) exactly and
    A = d - 1/2 c sigma_mu,nu (x) F_mu,nu with sigma_mu,nu = (i/2)[gamma_mu, gamma_nu]."""
    mu, nu = plane
    ns, nt = 4, 4
    L = nt if mu == 3 else ns
    phi = 2 * np.pi / L
    coords = np.meshgrid(np.arange(nt), np.arange(ns), np.arange(ns), np.arange(ns), indexing="ij")
    xmu = coords[3 - mu]
    phases = np.zeros((nt, ns, ns, ns, 4))
    phases[..., nu] = phi * xmu
    q = np.array([1.0, -1.0, 0.0])
    U = synth.unit_gauge_field(ns, nt)
    for a in range(3):
        U[..., a, a] = np.exp(1j * q[a] * phases)
    m0 = -0.05
    A = oracle.clover(U, m0, XI, 1.0)
    g = [oracle.gamma(m) for m in range(4)]
    sig = 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])
    c = (1 + 1 / XI) / 2 if nu == 3 else 1 / XI
    F = np.diag(q * np.sin(phi))
    ref = (m0 + 1 + 3 / XI) * np.eye(12) - 0.5 * c * np.kron(sig, F)
    assert np.abs(A - ref).max() < 1e-14


def test_gamma5_hermiticity_and_adjoint():
    U = synth.gauge_field(4, 4, 0.6, 2)
    D = oracle.Dirac(U, -0.1, XI, 1.0)
    a = synth.random_spinor(4, 4, 1)
    b = synth.random_spinor(4, 4, 2)
    lhs = np.vdot(a, _g(4, D.K(_g(4, b))))
    rhs = np.vdot(D.K(a), b)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    assert abs(np.vdot(a, D.K(b)) - np.vdot(D.K(a, dagger=True), b)) < 1e-13 * abs(lhs)
    assert abs(np.vdot(a, D.omega(b)) - np.vdot(D.omega(a, dagger=True), b)) < 1e-13 * abs(lhs)


def test_dirac_gauge_covariance():
    U = synth.gauge_field(4, 4, 0.6, 2)
    G = synth.gauge_transform_field(4, 4, 7)
    psi = synth.random_spinor(4, 4, 3)
    D1 = oracle.Dirac(_transform_links(U, G), -0.1, XI, 1.0)
    D0 = oracle.Dirac(U, -0.1, XI, 1.0)
    Gpsi = np.einsum("...ab,...sb->...sa", G, psi)
    a = D1.K(Gpsi)
    b = np.einsum("...ab,...sb->...sa", G, D0.K(psi))
    assert np.abs(a - b).max() < 1e-13


def test_antiperiodic_time_boundary():
    """Constant-in-space field on the last slice: the forward time hop across the
    boundary carries the factor -1 (free field, so only the hop term is involved)."""
    ns, nt = 2, 4
    U = synth.unit_gauge_field(ns, nt)
    D = oracle.Dirac(U, 0.0, XI, 0.0)
    psi = np.zeros((nt, ns, ns, ns, 4, 3), dtype=complex)
    psi[0, ..., 0, 0] = 1.0  # only t = 0
    out = D.K(psi)
    # at t = nt-1 the forward hop reaches t = 0: -1/2 (1 - gamma_4) psi * (-1)
    P = np.eye(4) - oracle.gamma(3)
    assert np.abs(out[nt - 1, 0, 0, 0, :, 0] - 0.5 * P[:, 0]).max() < 1e-15
    # at t = 1 the backward hop reaches t = 0 with no sign: -1/2 (1 + gamma_4) psi
    Pb = np.eye(4) + oracle.gamma(3)
    assert np.abs(out[1, 0, 0, 0, :, 0] + 0.5 * Pb[:, 0]).max() < 1e-15


def test_solve_matches_dense_lu_4x4():
    """Dense LU on a 4^4 lattice: the CGNR solution agrees within cond * tol."""
    U = synth.gauge_field(4, 4, 0.3, 1)
    D = oracle.Dirac(U, -0.02, XI, 1.0)
    M = D.dense(omega=True)
    eta = synth.random_spinor(4, 4, 4)
    x_lu = np.linalg.solve(M, eta.reshape(-1))
    x, it, tr = D.solve(eta, tol=1e-12)
    assert it > 0 and tr <= 1e-12
    s = np.linalg.svd(M, compute_uv=False)
    cond = s[0] / s[-1]
    assert np.linalg.norm(x.reshape(-1) - x_lu) / np.linalg.norm(x_lu) <= cond * 1e-12
    # the dense matrix is the operator: application agrees with the stencil
    assert np.abs(M @ eta.reshape(-1) - D.omega(eta).reshape(-1)).max() < 1e-13


# --------------------------------------------------------------- quark lines

@pytest.fixture(scope="module")
def ns4_nt8_setup():
    cfg = synth.CONFIGS["ns4_nt8"]
    U = synth.gauge_field(cfg.ns, cfg.nt, cfg.eps, cfg.seed)
    S = oracle.stout_spatial(U, cfg.stout_rho, cfg.stout_steps)
    ev, V = oracle.laph_eigpairs(S, cfg.nv)
    D = oracle.Dirac(U, cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    tau = oracle.perambulator(D, V)
    return cfg, U, V, D, tau


def test_source_recovers_diluted_noise(ns4_nt8_setup):
    cfg, U, V, D, tau = ns4_nt8_setup
    rho = oracle.z4_noise(cfg.noise_s, cfg.noise_k, cfg.nt, cfg.nv)
    sch = oracle.parse_dilution("TI4,SB2,LI4", cfg.nt, cfg.nv)
    for b in (0, 5, 31):
        eta = oracle.source(V, rho, sch, b)
        P = oracle.dilution_projector(sch, cfg.nt, cfg.nv, b)
        c = oracle.sink_project(V, eta)
        assert np.abs(c - P * rho).max() < 1e-14
        # support: zero outside T(b_T) x S(b_S)
        supp = (P.sum(axis=2) > 0)  # [t, alpha]
        mask = np.broadcast_to(supp[:, None, None, None, :, None], eta.shape)
        assert np.abs(eta[~mask]).max() == 0


def test_full_dilution_reproduces_perambulator(ns4_nt8_setup):
    """Sec. II: with full T x S x L dilution, sum_b c^[b] (P_b rho)^dag equals
    V^dag Omega^-1 V exactly for a single noise.  Checked source by source on a
    sample of b: c^[b] = tau[:, b] rho_b (CGNR solve vs dense LU)."""
    cfg, U, V, D, tau = ns4_nt8_setup
    rho = oracle.z4_noise(cfg.noise_s, cfg.noise_k, cfg.nt, cfg.nv)
    sch = oracle.parse_dilution(cfg.dilution, cfg.nt, cfg.nv)
    assert oracle.dilution_count(sch, cfg.nt, cfg.nv) == 256
    for b in (0, 37, 128, 255):
        eta = oracle.source(V, rho, sch, b)
        x, it, tr = D.solve(eta, tol=1e-12)
        assert tr <= 1e-12
        c = oracle.sink_project(V, x).ravel()
        ref = tau[:, b] * rho.ravel()[b]
        assert np.linalg.norm(c - ref) / np.linalg.norm(ref) < 1e-9


def test_coefficients_gauge_invariant(ns4_nt8_setup):
    """Sec. IV: coefficients are gauge invariant when the eigenvector phases are carried
    along (V -> G V)."""
    cfg, U, V, D, tau = ns4_nt8_setup
    G = synth.gauge_transform_field(cfg.ns, cfg.nt, 11)
    UG = _transform_links(U, G)
    VG = np.einsum("tzyxab,tnzyxb->tnzyxa", G, V)
    DG = oracle.Dirac(UG, cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    rho = oracle.z4_noise(0, 1, cfg.nt, cfg.nv)
    sch = oracle.parse_dilution("TI2,SF,LI2", cfg.nt, cfg.nv)
    c0 = oracle.sink_project(V, D.solve(oracle.source(V, rho, sch, 3), tol=1e-12)[0])
    c1 = oracle.sink_project(VG, DG.solve(oracle.source(VG, rho, sch, 3), tol=1e-12)[0])
    assert np.linalg.norm(c1 - c0) / np.linalg.norm(c0) < 1e-10


def test_undiluted_estimator_statistics(ns4_nt8_setup):
    """Sec. II: Omega^-1 ~ N_R^-1 sum_r X^r eta^r dag; without dilution the error of the
    estimate of tau falls like 1/sqrt(N).  Uses c = tau rho (exact for each noise)."""
    cfg, U, V, D, tau = ns4_nt8_setup
    errs = []
    for N in (16, 256):
        est = np.zeros_like(tau)
        for s in range(N):
            rho = oracle.z4_noise(s, 1, cfg.nt, cfg.nv).ravel()
            est += np.outer(tau @ rho, rho.conj())
        errs.append(np.linalg.norm(est / N - tau) / np.linalg.norm(tau))
    ratio = errs[0] / errs[1]
    assert 2.5 < ratio < 6.5  # sqrt(256/16) = 4

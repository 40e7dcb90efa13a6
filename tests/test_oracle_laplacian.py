"""Pins of the oracle's stout smearing, Laplacian, Chebyshev map and LapH eigenpairs.

Sec. II: spatial stout links (spatial staples only, temporal links untouched); the
gauge-covariant Laplacian, Hermitian and block diagonal in time, eigenvalues of
-Lap non-negative.  Sec. IV: the Chebyshev transform B = 1 + 2/(lamL-lamC)(Lap+lamC)
and A = T_n(B) by the three-term recurrence; the eigenvector phase convention.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth


def _transform_links(U, G):
    """U^G_mu(x) = G(x) U_mu(x) G(x+mu)^dag."""
    out = np.empty_like(U)
    for mu in range(4):
        axis = 3 - mu  # array axes are [t, z, y, x]
        Gp = np.roll(G, -1, axis=axis)
        out[..., mu, :, :] = G @ U[..., mu, :, :] @ np.conj(np.swapaxes(Gp, -1, -2))
    return out


# ---------------------------------------------------------------------- stout

def test_stout_unit_is_fixed_point():
    U = synth.unit_gauge_field(4, 4)
    assert np.abs(oracle.stout_spatial(U, 0.1, 3) - U).max() < 1e-15


def test_stout_preserves_su3_and_leaves_time_links():
    U = synth.gauge_field(4, 4, 0.5, 3)
    S = oracle.stout_spatial(U, 0.1, 4)
    I3 = np.eye(3)
    assert np.abs(np.conj(np.swapaxes(S, -1, -2)) @ S - I3).max() < 1e-13
    assert np.abs(np.linalg.det(S) - 1).max() < 1e-13
    assert np.array_equal(S[..., 3, :, :], U[..., 3, :, :])


def test_stout_rho_zero_is_identity():
    U = synth.gauge_field(4, 4, 0.5, 3)
    assert np.abs(oracle.stout_spatial(U, 0.0, 2) - U).max() < 1e-14


def test_stout_gauge_covariance():
    U = synth.gauge_field(4, 4, 0.6, 5)
    G = synth.gauge_transform_field(4, 4, 9)
    a = oracle.stout_spatial(_transform_links(U, G), 0.1, 2)
    b = _transform_links(oracle.stout_spatial(U, 0.1, 2), G)
    assert np.abs(a[..., :3, :, :] - b[..., :3, :, :]).max() < 1e-13


def test_stout_raises_plaquette():
    U = synth.gauge_field(4, 4, 0.6, 5)
    p = [oracle.plaquette_spatial(oracle.stout_spatial(U, 0.1, n)) for n in range(4)]
    assert all(b > a for a, b in zip(p, p[1:]))


def test_stout_abelian_closed_form():
    """For links diag(e^{i phi}, e^{-i phi}, 1) everything is diagonal and one step
    reduces to phase arithmetic: Q_aa = Im(w_a) - (1/3) sum_b Im(w_b) with
    w_a = rho * (staple sum)_aa * conj(u_a), and u_a' = exp(i Q_aa) u_a."""
    ns, nt, rho = 4, 2, 0.13
    rng = np.random.default_rng(2)
    phi = rng.uniform(-1, 1, (nt, ns, ns, ns, 4))
    q = np.array([1.0, -1.0, 0.0])
    U = synth.unit_gauge_field(ns, nt)
    for a in range(3):
        U[..., a, a] = np.exp(1j * q[a] * phi)
    S = oracle.stout_spatial(U, rho, 1)
    u = np.stack([U[..., a, a] for a in range(3)], -1)  # [t,z,y,x,mu,a]
    new = u.copy()
    for k in range(3):
        C = np.zeros(u.shape[:4] + (3,), dtype=complex)
        for j in range(3):
            if j == k:
                continue
            ax_j, ax_k = 3 - j, 3 - k
            uj, uk = u[..., j, :], u[..., k, :]
            C += uj * np.roll(uk, -1, ax_j) * np.conj(np.roll(uj, -1, ax_k))
            ujm = np.roll(uj, 1, ax_j)
            C += np.conj(ujm) * np.roll(uk, 1, ax_j) * np.roll(ujm, -1, ax_k)
        w = rho * C * np.conj(uk)
        Q = w.imag - w.imag.sum(-1, keepdims=True) / 3
        new[..., k, :] = np.exp(1j * Q) * uk
    for a in range(3):
        assert np.abs(S[..., a, a] - new[..., a]).max() < 1e-14
    off = S.copy()
    for a in range(3):
        off[..., a, a] = 0
    assert np.abs(off).max() < 1e-15


# ------------------------------------------------------------------ Laplacian

def test_free_laplacian_plane_waves():
    """U = 1: Lap e^{ipx} = -sum_k 4 sin^2(p_k/2) e^{ipx}, p_k = 2 pi n_k / L."""
    ns, nt = 6, 2
    U = synth.unit_gauge_field(ns, nt)
    x = np.arange(ns)
    for n in [(0, 0, 0), (1, 0, 0), (1, 2, 3), (5, 5, 1)]:
        p = 2 * np.pi * np.array(n) / ns
        ph = np.exp(1j * (p[0] * x[None, None, :] + p[1] * x[None, :, None] + p[2] * x[:, None, None]))
        v = np.zeros((nt, ns, ns, ns, 3), dtype=complex)
        v[0, ..., 1] = ph
        v[1, ..., 0] = 2 * ph
        lam = -np.sum(4 * np.sin(p / 2) ** 2)
        assert np.abs(oracle.laplacian(U, v) - lam * v).max() < 1e-13


def test_free_laplacian_spectrum():
    ns = 4
    U = synth.unit_gauge_field(ns, 1)
    w = np.linalg.eigvalsh(oracle.laplacian_slice_matrix(U, 0))
    ref = sorted(3 * [sum(4 * np.sin(np.pi * n / ns) ** 2 for n in ns3)
                      for ns3 in itertools.product(range(ns), repeat=3)])
    assert np.abs(np.sort(w) - np.array(ref)).max() < 1e-12


def test_laplacian_hermitian_and_bounded():
    U = synth.gauge_field(4, 2, 0.7, 4)
    a = synth.random_colour_field(4, 2, 1)
    b = synth.random_colour_field(4, 2, 2)
    lhs = np.vdot(a, oracle.laplacian(U, b))
    rhs = np.vdot(oracle.laplacian(U, a), b)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    M = oracle.laplacian_slice_matrix(U, 1)
    assert np.abs(M - M.conj().T).max() < 1e-14
    w = np.linalg.eigvalsh(M)
    assert w.min() >= -1e-12 and w.max() <= 12 + 1e-12


def test_laplacian_block_diagonal_in_time():
    U = synth.gauge_field(4, 3, 0.5, 4)
    v = np.zeros((3, 4, 4, 4, 3), dtype=complex)
    v[1] = synth.random_colour_field(4, 1, 3)[0]
    out = oracle.laplacian(U, v)
    assert np.abs(out[0]).max() == 0 and np.abs(out[2]).max() == 0
    assert np.abs(out[1] - oracle.laplacian_slice(U, 1, v[1])).max() == 0


def test_laplacian_gauge_covariance():
    U = synth.gauge_field(4, 2, 0.7, 4)
    G = synth.gauge_transform_field(4, 2, 5)
    v = synth.random_colour_field(4, 2, 6)
    a = oracle.laplacian(_transform_links(U, G), np.einsum("...ab,...b->...a", G, v))
    b = np.einsum("...ab,...b->...a", G, oracle.laplacian(U, v))
    assert np.abs(a - b).max() < 1e-13


# ------------------------------------------------------------------ Chebyshev

def test_chebyshev_endpoints_and_value():
    lamL, lamC = 15.0, 0.5
    B = lambda mu: 1 + 2 * (lamC - mu) / (lamL - lamC)  # B on an eigenvalue mu of -Lap
    assert B(lamL) == -1.0 and B(lamC) == 1.0
    # T_8(B(0)) = cosh(8 arccosh(1.06897)) = 9.62
    assert abs(np.cosh(8 * np.arccosh(B(0.0))) - 9.62) < 0.01


def test_chebyshev_on_eigenbasis():
    """T_n(B) v equals X T_n(B(lam)) X^dag v with T_n(cos th) = cos(n th) and
    T_n(cosh a) = cosh(n a): checks the three-term recurrence against the closed form."""
    ns = 4
    U = synth.gauge_field(ns, 1, 0.4, 8)
    M = oracle.laplacian_slice_matrix(U, 0)  # -Lap
    w, X = np.linalg.eigh(M)
    lamL, lamC = 15.0, 2.5
    v = synth.random_colour_field(ns, 1, 3)
    for order in (0, 1, 2, 5, 8):
        y = oracle.chebyshev(U, v, lamL, lamC, order)
        b = 1 + 2 * (lamC - w) / (lamL - lamC)
        tb = np.where(np.abs(b) <= 1, np.cos(order * np.arccos(np.clip(b, -1, 1))),
                      np.cosh(order * np.arccosh(np.maximum(np.abs(b), 1))) * np.sign(b) ** order)
        ref = X @ (tb * (X.conj().T @ v.reshape(-1)))
        assert np.abs(y.reshape(-1) - ref).max() < 1e-11 * max(1, np.abs(ref).max())
        # the unwanted part of the spectrum stays inside [-1, 1]
        assert np.all(np.abs(tb[w >= lamC]) <= 1 + 1e-12)


# ------------------------------------------------------------------ eigenpairs

def test_eigpairs_free_field_and_phase():
    ns, nt, nv = 4, 2, 8
    U = synth.unit_gauge_field(ns, nt)
    ev, V = oracle.laph_eigpairs(U, nv, extra=2)
    assert np.abs(ev[:, :3]).max() < 1e-12
    assert np.abs(ev[:, 3:10] - 4 * np.sin(np.pi / 4) ** 2).max() < 1e-12


def test_eigpairs_orthonormal_residual_phase():
    cfg = synth.CONFIGS["ns4_nt8"]
    U = synth.gauge_field(cfg.ns, cfg.nt, cfg.eps, cfg.seed)
    S = oracle.stout_spatial(U, cfg.stout_rho, cfg.stout_steps)
    ev, V = oracle.laph_eigpairs(S, cfg.nv, slices=[0, 5])
    for si, t in enumerate([0, 5]):
        Vt = V[si].reshape(cfg.nv, -1)
        assert np.abs(Vt.conj() @ Vt.T - np.eye(cfg.nv)).max() < 1e-13
        for n in range(cfg.nv):
            v = V[si, n]
            r = -oracle.laplacian_slice(S, t, v) - ev[si, n] * v
            assert np.linalg.norm(r) < 1e-12
            flat = v.ravel()
            a = np.abs(flat)
            i = int(np.argmax(a >= 0.1 * a.max()))
            assert flat[i].imag == 0.0 and flat[i].real > 0
        assert np.all(np.diff(ev[si]) >= 0) and ev[si, 0] >= 0


def test_eigpairs_arpack_matches_dense():
    U = synth.gauge_field(4, 1, 0.4, 3)
    S = oracle.stout_spatial(U, 0.1, 1)
    ed, Vd = oracle.laph_eigpairs(S, 6, method="dense", extra=1)
    ea, Va = oracle.laph_eigpairs(S, 6, method="arpack", extra=1)
    assert np.abs(ed - ea).max() < 1e-11


def test_eigenvalues_gauge_invariant():
    U = synth.gauge_field(4, 1, 0.5, 3)
    G = synth.gauge_transform_field(4, 1, 4)
    e1, _ = oracle.laph_eigpairs(U, 8)
    e2, _ = oracle.laph_eigpairs(_transform_links(U, G), 8)
    assert np.abs(e1 - e2).max() < 1e-12

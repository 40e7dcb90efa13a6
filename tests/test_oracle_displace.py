"""Pins of the oracle's covariant displacements and momentum overlaps (Sec. II: the
displacement types D^(j) of the quark lines D^(j) S Omega^-1 S D^(k)dag; Sec. III.B: the
momentum projection of the meson function)."""
import numpy as np
import pytest

import oracle
import synth

NS, NT = 4, 4


def _field(seed, ns=NS, nt=NT):
    r = np.random.default_rng(seed)
    return r.normal(size=(nt, ns, ns, ns, 3)) + 1j * r.normal(size=(nt, ns, ns, ns, 3))


@pytest.mark.parametrize("d,s,L", [(0, 1, 3), (1, -1, 3), (2, 1, 1), (2, -1, 2)])
def test_unit_field_is_a_shift(d, s, L):
    U = synth.unit_gauge_field(NS, NT)
    v = _field(1)
    out = oracle.displace(U, v, d, s, L)
    axis = {0: 3, 1: 2, 2: 1}[d]  # array axes are [t, z, y, x]
    assert np.array_equal(out, np.roll(v, -s * L, axis=axis))


@pytest.mark.parametrize("d,s", [(0, 1), (1, -1), (2, 1)])
def test_gauge_covariance(d, s):
    """D[U^G](G v) = G D[U] v with U_mu(x) -> G(x) U_mu(x) G(x+mu)^dag."""
    U = synth.gauge_field(NS, NT, 0.7, 3)
    G = synth.gauge_transform_field(NS, NT, 4)
    UG = np.empty_like(U)
    for mu in range(4):
        axis = {0: 3, 1: 2, 2: 1, 3: 0}[mu]
        Gn = np.roll(G, -1, axis=axis)
        UG[..., mu, :, :] = np.einsum("tzyxab,tzyxbc,tzyxdc->tzyxad", G, U[..., mu, :, :], Gn.conj())
    v = _field(5)
    lhs = oracle.displace(UG, np.einsum("tzyxab,tzyxb->tzyxa", G, v), d, s)
    rhs = np.einsum("tzyxab,tzyxb->tzyxa", G, oracle.displace(U, v, d, s))
    assert np.abs(lhs - rhs).max() < 1e-13


@pytest.mark.parametrize("d", [0, 1, 2])
def test_backward_is_adjoint_and_composition(d):
    """<a, D+ b> = <D- a, b> (the backward displacement is the adjoint of the forward one),
    and a 3-link displacement is three 1-link ones."""
    U = synth.gauge_field(NS, NT, 0.6, 6)
    a, b = _field(7), _field(8)
    lhs = np.vdot(a, oracle.displace(U, b, d, 1))
    rhs = np.vdot(oracle.displace(U, a, d, -1), b)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    w = b
    for _ in range(3):
        w = oracle.displace(U, w, d, 1, 1)
    assert np.abs(w - oracle.displace(U, b, d, 1, 3)).max() < 1e-13


def test_mom_overlap_plane_waves_and_symmetry():
    """Free plane waves e^{2 pi i q.x / Ns} e_c: O(k) = Ns^3 delta_{k, q_m - q_n} delta_{c_n c_m};
    conj O_ab(k) = O_ba(-k)^T for general fields."""
    t, z, y, x = np.meshgrid(*(np.arange(n) for n in (NT, NS, NS, NS)), indexing="ij")
    qs = [(0, 0, 0), (1, 0, 0), (0, 2, 1), (3, 3, 3)]
    cols = [0, 1, 0, 2]
    vecs = np.zeros((NT, len(qs), NS, NS, NS, 3), dtype=np.complex128)
    for j, (q, c) in enumerate(zip(qs, cols)):
        vecs[:, j, ..., c] = np.exp(2j * np.pi * (q[0] * x + q[1] * y + q[2] * z) / NS)
    for k in ((0, 0, 0), (1, 0, 0), (3, 1, 2)):
        O = oracle.mom_overlap(vecs, vecs, k)
        ref = np.zeros((len(qs), len(qs)), dtype=np.complex128)
        for n in range(len(qs)):
            for m in range(len(qs)):
                dq = tuple((qs[m][i] - qs[n][i] - k[i]) % NS for i in range(3))
                if dq == (0, 0, 0) and cols[n] == cols[m]:
                    ref[n, m] = NS ** 3
        assert np.abs(O - ref[None]).max() < 1e-12
    r = np.random.default_rng(9)
    a = r.normal(size=(NT, 3, NS, NS, NS, 3)) + 1j * r.normal(size=(NT, 3, NS, NS, NS, 3))
    b = r.normal(size=(NT, 2, NS, NS, NS, 3)) + 1j * r.normal(size=(NT, 2, NS, NS, NS, 3))
    Oab = oracle.mom_overlap(a, b, (1, 2, 0))
    Oba = oracle.mom_overlap(b, a, (-1, -2, 0))
    assert np.abs(Oab.conj() - Oba.transpose(0, 2, 1)).max() < 1e-12 * np.abs(Oab).max()


def test_displaced_meson_function_from_overlaps():
    """The displaced, momentum-projected meson function of two LapH-smeared fields
    V_s a and V_s b (Eq. mesonfunc) factorises through the overlaps of displaced
    eigenvectors: sum_{ab} c_ab sum_{nm} conj(a_an) O_nm b_bm times exp(-i p.(d1+d2)/2),
    the reduction the GPU path uses; checked against the full-field definition."""
    ns, nt, nv = 4, 4, 5
    U = synth.gauge_field(ns, nt, 0.5, 10)
    r = np.random.default_rng(11)
    V = np.empty((nt, nv, ns, ns, ns, 3), dtype=np.complex128)
    for tt in range(nt):
        q, _ = np.linalg.qr(r.normal(size=(ns ** 3 * 3, nv)) + 1j * r.normal(size=(ns ** 3 * 3, nv)))
        V[tt] = q.T.reshape(nv, ns, ns, ns, 3)
    a = r.normal(size=(nt, 4, nv)) + 1j * r.normal(size=(nt, 4, nv))
    b = r.normal(size=(nt, 4, nv)) + 1j * r.normal(size=(nt, 4, nv))
    c = r.normal(size=(4, 4)) + 1j * r.normal(size=(4, 4))
    k, (d1, s1), (d2, s2) = (1, 0, 3), (0, 1), (2, -1)
    f1 = oracle.displace_spinor(U, oracle.smeared_field(V, a), d1, s1)
    f2 = oracle.displace_spinor(U, oracle.smeared_field(V, b), d2, s2)
    dv1, dv2 = [0, 0, 0], [0, 0, 0]
    dv1[d1], dv2[d2] = 3 * s1, 3 * s2
    ref = oracle.meson_function(f1, f2, c, k=k, d1=dv1, d2=dv2)
    O = oracle.mom_overlap(oracle.displace_evecs(U, V, d1, s1), oracle.displace_evecs(U, V, d2, s2), k)
    ph = np.exp(-1j * 2 * np.pi / ns * sum(kk * (p + q) / 2 for kk, p, q in zip(k, dv1, dv2)))
    got = ph * np.einsum("ab,tan,tnm,tbm->t", c, a.conj(), O, b)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()

"""Pins of the oracle's parallel-transport network (learned preconditioner), CPU only.

The network is not in the paper; what fixes it is (i) that one layer with spin weights
built from the Wilson projectors is exactly the hopping part of the Dirac operator K of
Sec. II (so the transports inherit the pinned operator's direction, link and boundary
conventions), (ii) a site-by-site loop written independently of the array code,
(iii) gauge equivariance, and (iv) central finite differences of the backward pass.
"""
import numpy as np

import oracle
import synth
from oracle import ptnet


def _transform_links(U, G):
    out = np.empty_like(U)
    for mu in range(4):
        Gp = np.roll(G, -1, axis=3 - mu)
        out[..., mu, :, :] = G @ U[..., mu, :, :] @ np.conj(np.swapaxes(Gp, -1, -2))
    return out


def test_one_layer_is_the_wilson_operator():
    ns, nt, m0, xi = 4, 4, 0.2, 3.5
    U = synth.gauge_field(ns, nt, 0.4, 7)
    psi = synth.random_spinor(ns, nt, 8)
    W = np.zeros((1, 1, 9, 4, 4), dtype=np.complex128)
    W[0, 0, 0] = (m0 + 1 + 3 / xi) * np.eye(4)
    for mu in range(4):
        w = 1.0 if mu == 3 else 1.0 / xi
        g = oracle.gamma(mu)
        W[0, 0, 1 + mu] = -0.5 * w * (np.eye(4) - g)
        W[0, 0, 5 + mu] = -0.5 * w * (np.eye(4) + g)
    out, _ = ptnet.forward(U, [W], psi, bc_t=-1.0)
    ref = oracle.Dirac(U, m0, xi, 0.0, -1.0).K(psi)
    assert np.abs(out - ref).max() < 1e-12 * np.abs(ref).max()


def test_transport_site_loop():
    ns, nt, bc = 3, 4, -1.0
    U = synth.gauge_field(ns, nt, 0.5, 3)
    phi = synth.random_spinor(ns, nt, 4)
    for d in range(9):
        got = ptnet.transport(U, phi, d, bc)
        ref = np.empty_like(phi)
        for t in range(nt):
            for z in range(ns):
                for y in range(ns):
                    for x in range(ns):
                        if d == 0:
                            ref[t, z, y, x] = phi[t, z, y, x]
                            continue
                        mu, fwd = (d - 1) % 4, d <= 4
                        c = [x, y, z, t]
                        n = list(c)
                        L = nt if mu == 3 else ns
                        n[mu] = c[mu] + (1 if fwd else -1)
                        f = 1.0
                        if n[mu] in (-1, L):
                            n[mu] %= L
                            f = bc if mu == 3 else 1.0
                        src = phi[n[3], n[2], n[1], n[0]]
                        if fwd:
                            link = U[t, z, y, x, mu]
                        else:
                            link = U[n[3], n[2], n[1], n[0], mu].conj().T
                        ref[t, z, y, x] = f * (src @ link.T)
        assert np.abs(got - ref).max() < 1e-14, d


def test_gauge_equivariance():
    ns, nt = 3, 4
    U = synth.gauge_field(ns, nt, 0.5, 11)
    G = synth.gauge_transform_field(ns, nt, 12)
    psi = synth.random_spinor(ns, nt, 13)
    ws = ptnet.init_weights([1, 2, 4, 1], seed=5, scale=0.3)
    out, _ = ptnet.forward(U, ws, psi)
    Ug = _transform_links(U, G)
    psig = np.einsum("...ab,...sb->...sa", G, psi)
    outg, _ = ptnet.forward(Ug, ws, psig)
    ref = np.einsum("...ab,...sb->...sa", G, out)
    assert np.abs(outg - ref).max() < 1e-12 * np.abs(ref).max()


def test_backward_matches_finite_differences():
    ns, nt = 3, 4
    U = synth.gauge_field(ns, nt, 0.5, 21)
    psi = synth.random_spinor(ns, nt, 22)
    tgt = synth.random_spinor(ns, nt, 23)
    ws = ptnet.init_weights([1, 2, 2, 1], seed=9, scale=0.2)

    def loss(ws_, psi_):
        out, _ = ptnet.forward(U, ws_, psi_)
        return np.sum(np.abs(out - tgt) ** 2)

    out, acts = ptnet.forward(U, ws, psi)
    gpsi, gW = ptnet.backward(U, ws, acts, out - tgt)
    rng = np.random.default_rng(0)
    h = 1e-6
    # weights: dL/dRe = 2 Re(dL/dW*), dL/dIm = 2 Im(dL/dW*)
    for _ in range(12):
        l = int(rng.integers(len(ws)))
        idx = tuple(int(rng.integers(s)) for s in ws[l].shape)
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[l][idx] += unit * h
            wm[l][idx] -= unit * h
            fd = (loss(wp, psi) - loss(wm, psi)) / (2 * h)
            an = 2 * part(gW[l][idx])
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (l, idx, fd, an)
    for _ in range(6):
        idx = tuple(int(rng.integers(s)) for s in psi.shape)
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            pp, pm = psi.copy(), psi.copy()
            pp[idx] += unit * h
            pm[idx] -= unit * h
            fd = (loss(ws, pp) - loss(ws, pm)) / (2 * h)
            an = 2 * part(gpsi[idx])
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (idx, fd, an)

"""Plain FP64 oracle of the gauge-equivariant parallel-transport network (PT-net) used as
a learned preconditioner.  TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper has no network: this component serves the learned-preconditioner extension of
the solve (Omega x = eta, Sec. IV), whose answer is still judged by the FP64 true
residual.  A layer maps C_in spinor fields to C_out spinor fields:

    out_c(x) = sum_{c', d} W[c, c', d] (T_d phi_c')(x),
    T_0 phi = phi,  T_{+mu} phi(x) = U_mu(x) phi(x+mu),  T_{-mu} phi(x) = U_mu(x-mu)^dag phi(x-mu),

with d = 0 (self), 1..4 (+mu, mu = x,y,z,t), 5..8 (-mu), W[c, c', d] a complex 4x4 matrix
acting on spin, and hops across the time boundary multiplied by bc_t (the fermion
boundary condition).  Spin-only weights and colour-only transports make every layer
gauge equivariant.  Fields: [C][Nt,Ns,Ns,Ns,4,3] complex.
"""
from __future__ import annotations

import numpy as np


def _axis(mu):
    return {0: 3, 1: 2, 2: 1, 3: 0}[mu]  # array axes are [t, z, y, x]


def transport(U, phi, d, bc_t=-1.0):
    """T_d phi for one spinor field phi [Nt,Ns,Ns,Ns,4,3]."""
    if d == 0:
        return phi.copy()
    nt = U.shape[0]
    if d <= 4:
        mu = d - 1
        sh = np.roll(phi, -1, axis=_axis(mu))
        if mu == 3:
            sh = sh.copy()
            sh[nt - 1] *= bc_t  # hop from t = nt-1 to t = 0
        return np.einsum("...ab,...sb->...sa", U[..., mu, :, :], sh)
    mu = d - 5
    Um = np.roll(U[..., mu, :, :], 1, axis=_axis(mu))  # U_mu(x - mu)
    sh = np.roll(phi, 1, axis=_axis(mu))
    if mu == 3:
        sh = sh.copy()
        sh[0] *= bc_t  # hop from t = 0 to t = nt-1
    return np.einsum("...ba,...sb->...sa", Um.conj(), sh)


def layer(U, W, phi, bc_t=-1.0):
    """W: [C_out, C_in, 9, 4, 4] complex; phi: [C_in, ...] -> [C_out, ...]."""
    cout, cin = W.shape[0], W.shape[1]
    out = np.zeros((cout,) + phi.shape[1:], dtype=np.complex128)
    for ci in range(cin):
        for d in range(9):
            t = transport(U, phi[ci], d, bc_t)
            for co in range(cout):
                out[co] += np.einsum("st,...tc->...sc", W[co, ci, d], t)
    return out


def forward(U, weights, psi, bc_t=-1.0):
    """weights: list of layer weight arrays; psi: one spinor field.  Returns the output
    field and the list of layer inputs (for the backward pass)."""
    acts = [psi[None]]
    for W in weights:
        acts.append(layer(U, W, acts[-1], bc_t))
    return acts[-1][0], acts[:-1]


def backward(U, weights, acts, gout, bc_t=-1.0):
    """Gradients of a real loss L with g = dL/d(out)^* given: returns (dL/dpsi^*,
    [dL/dW^*]).  Uses the adjoint T_d^dag = T_{rev(d)} and the fact that spin weights and
    colour transports commute."""
    rev = [0, 5, 6, 7, 8, 1, 2, 3, 4]
    g = gout[None]
    gW = [None] * len(weights)
    for l in range(len(weights) - 1, -1, -1):
        W, phi = weights[l], acts[l]
        cout, cin = W.shape[0], W.shape[1]
        gw = np.zeros_like(W)
        for ci in range(cin):
            for d in range(9):
                t = transport(U, phi[ci], d, bc_t)
                for co in range(cout):
                    gw[co, ci, d] = np.einsum("nsc,ntc->st", g[co].reshape(-1, 4, 3), t.conj().reshape(-1, 4, 3))
        gW[l] = gw
        gin = np.zeros_like(phi)
        for co in range(cout):
            for d in range(9):
                t = transport(U, g[co], rev[d], bc_t)
                for ci in range(cin):
                    gin[ci] += np.einsum("ts,...tc->...sc", W[co, ci, d].conj(), t)
        g = gin
    return g[0], gW


def init_weights(channels, seed, scale=0.05):
    """Seeded small random weights plus an identity-like self term on the first path."""
    rng = np.random.default_rng(seed)
    ws = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        W = scale * (rng.standard_normal((cout, cin, 9, 4, 4)) + 1j * rng.standard_normal((cout, cin, 9, 4, 4)))
        W[:, :, 0] += np.eye(4)[None, None] * (1.0 / cin if cin else 1.0)
        ws.append(W)
    return ws

"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds none of the method's arithmetic: it only draws gauge fields, gauge
transformations and random vectors, and names the workload parameters.  The paper's
2+1-flavour anisotropic clover ensembles are not available; near-unit SU(3) fields
U = exp(i eps H), H = sum_a h_a lambda_a / 2 with h_a ~ N(0,1), stand in for them.
The exponential uses the Cayley-Hamilton closed form, evaluated elementwise.  Gaussian draws
go through libm, so a field is generated once and handed to both sides as data.
"""
from __future__ import annotations

import os

import numpy as np

from .configs import CONFIGS, Config  # noqa: F401


def _gell_mann():
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1] = -1j
    l[1][1, 0] = 1j
    l[2][0, 0] = 1
    l[2][1, 1] = -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2] = -1j
    l[4][2, 0] = 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2] = -1j
    l[6][2, 1] = 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l


_LAMBDA = _gell_mann()


def _su3_from_algebra(h, eps):
    """exp(i eps H), H = sum_a h_a lambda_a / 2, for a stack of coefficient rows h[n, 8].

    Elementwise over the stack: H is written out entry by entry and the exponential uses
    the Cayley-Hamilton form exp(iQ) = f0 + f1 Q + f2 Q^2 of Morningstar & Peardon
    (Phys. Rev. D 69, 054501), with Q = eps H."""
    r3 = np.sqrt(3.0)
    q = [[None] * 3 for _ in range(3)]
    q[0][0] = 0.5 * eps * (h[:, 2] + h[:, 7] / r3) + 0j
    q[1][1] = 0.5 * eps * (-h[:, 2] + h[:, 7] / r3) + 0j
    q[2][2] = 0.5 * eps * (-2.0 * h[:, 7] / r3) + 0j
    q[0][1] = 0.5 * eps * (h[:, 0] - 1j * h[:, 1])
    q[0][2] = 0.5 * eps * (h[:, 3] - 1j * h[:, 4])
    q[1][2] = 0.5 * eps * (h[:, 5] - 1j * h[:, 6])
    q[1][0], q[2][0], q[2][1] = np.conj(q[0][1]), np.conj(q[0][2]), np.conj(q[1][2])
    q2 = [[sum(q[i][k] * q[k][j] for k in range(3)) for j in range(3)] for i in range(3)]
    c1 = 0.5 * (q2[0][0] + q2[1][1] + q2[2][2]).real
    c0 = (q[0][0] * (q[1][1] * q[2][2] - q[1][2] * q[2][1])
          - q[0][1] * (q[1][0] * q[2][2] - q[1][2] * q[2][0])
          + q[0][2] * (q[1][0] * q[2][1] - q[1][1] * q[2][0])).real
    neg = c0 < 0
    c0a = np.abs(c0)
    c1s = np.maximum(c1, 1e-300)
    c0max = 2.0 * (c1s / 3.0) ** 1.5
    theta = np.arccos(np.minimum(1.0, c0a / c0max))
    u = np.sqrt(c1s / 3.0) * np.cos(theta / 3.0)
    w = np.sqrt(c1s) * np.sin(theta / 3.0)
    u2, w2 = u * u, w * w
    small = np.abs(w) < 0.05
    xi0 = np.where(small, 1.0 - w2 / 6.0 * (1.0 - w2 / 20.0 * (1.0 - w2 / 42.0)),
                   np.sin(w) / np.where(small, 1.0, w))
    cw = np.cos(w)
    e2iu = np.exp(2j * u)
    emiu = np.exp(-1j * u)
    h0 = (u2 - w2) * e2iu + emiu * (8 * u2 * cw + 2j * u * (3 * u2 + w2) * xi0)
    h1 = 2 * u * e2iu - emiu * (2 * u * cw - 1j * (3 * u2 - w2) * xi0)
    h2 = e2iu - emiu * (cw + 3j * u * xi0)
    den = 9 * u2 - w2
    f0, f1, f2 = h0 / den, h1 / den, h2 / den
    f0 = np.where(neg, np.conj(f0), f0)
    f1 = np.where(neg, -np.conj(f1), f1)
    f2 = np.where(neg, np.conj(f2), f2)
    out = np.empty((h.shape[0], 3, 3), dtype=np.complex128)
    for i in range(3):
        for j in range(3):
            out[:, i, j] = f1 * q[i][j] + f2 * q2[i][j] + (f0 if i == j else 0.0)
    return out


def gauge_field(ns: int, nt: int, eps: float, seed: int) -> np.ndarray:
    """Near-unit SU(3) links U[t,z,y,x,mu,a,b] = exp(i eps H), seeded."""
    from concurrent.futures import ThreadPoolExecutor

    rng = np.random.default_rng(seed)
    V = ns ** 3 * nt
    out = np.empty((V * 4, 3, 3), dtype=np.complex128)
    chunk = 1 << 17
    starts = list(range(0, V * 4, chunk))
    draws = [rng.standard_normal((min(chunk, V * 4 - s), 8)) for s in starts]  # fixed order

    def work(k):
        out[starts[k]:starts[k] + draws[k].shape[0]] = _su3_from_algebra(draws[k], eps)

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(work, range(len(starts))))
    return out.reshape(nt, ns, ns, ns, 4, 3, 3)


def unit_gauge_field(ns: int, nt: int) -> np.ndarray:
    U = np.zeros((nt, ns, ns, ns, 4, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def u1_gauge_field(ns: int, nt: int, phases) -> np.ndarray:
    """Links diag(e^{i phi_mu(x)}) times unit colour, for abelian background tests.
    phases: array [Nt,Ns,Ns,Ns,4] of angles."""
    U = unit_gauge_field(ns, nt)
    ph = np.exp(1j * np.asarray(phases))
    for a in range(3):
        U[..., a, a] = ph
    return U


def random_su3(n: int, seed: int) -> np.ndarray:
    """n Haar-random SU(3) matrices (QR of complex Gaussians, phases fixed, det = 1)."""
    rng = np.random.default_rng(seed)
    Z = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) / np.sqrt(2)
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=1, axis2=2)
    Q = Q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(Q)
    Q = Q / (det ** (1.0 / 3.0))[:, None, None]
    return Q


def gauge_transform_field(ns: int, nt: int, seed: int) -> np.ndarray:
    """Random SU(3) gauge transformation G[t,z,y,x,a,b]."""
    return random_su3(ns ** 3 * nt, seed).reshape(nt, ns, ns, ns, 3, 3)


def random_spinor(ns: int, nt: int, seed: int, nrhs: int | None = None) -> np.ndarray:
    rng = np.random.default_rng(seed)
    shape = (nt, ns, ns, ns, 4, 3) if nrhs is None else (nrhs, nt, ns, ns, ns, 4, 3)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def random_colour_field(ns: int, nt: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    shape = (nt, ns, ns, ns, 3)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)

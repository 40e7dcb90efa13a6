"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds none of the method's arithmetic: it only draws gauge fields, gauge
transformations and random vectors, and names the workload parameters.  The paper's
2+1-flavour anisotropic clover ensembles are not available; near-unit SU(3) fields
U = exp(i eps H), H = sum_a h_a lambda_a / 2 with h_a ~ N(0,1), stand in for them.
The exponential is taken through numpy's Hermitian eigendecomposition.  Gaussian draws
go through libm, so a field is generated once and handed to both sides as data.
"""
from __future__ import annotations

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


def _expi_hermitian(H, eps, chunk=1 << 20):
    """exp(i eps H) for a stack of Hermitian 3x3 matrices."""
    out = np.empty_like(H)
    flat_in = H.reshape(-1, 3, 3)
    flat_out = out.reshape(-1, 3, 3)
    for s in range(0, flat_in.shape[0], chunk):
        w, X = np.linalg.eigh(flat_in[s:s + chunk])
        ph = np.exp(1j * eps * w)
        flat_out[s:s + chunk] = np.einsum("nij,nj,nkj->nik", X, ph, X.conj())
    return out


def gauge_field(ns: int, nt: int, eps: float, seed: int) -> np.ndarray:
    """Near-unit SU(3) links U[t,z,y,x,mu,a,b] = exp(i eps H), seeded."""
    rng = np.random.default_rng(seed)
    V = ns ** 3 * nt
    out = np.empty((V * 4, 3, 3), dtype=np.complex128)
    chunk = 1 << 19
    for s in range(0, V * 4, chunk):
        n = min(chunk, V * 4 - s)
        h = rng.standard_normal((n, 8))
        H = np.einsum("na,aij->nij", h, _LAMBDA) * 0.5
        out[s:s + n] = _expi_hermitian(H, eps)
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

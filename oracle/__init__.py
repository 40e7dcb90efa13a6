"""Plain FP64 CPU oracle for the stochastic-LapH hot path (arXiv:1104.3870).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the CPU-baseline leg
of the benchmark may import this package.  It shares no code with the GPU library:
the C part (``laph_oracle.c``) is compiled here with gcc, and the dense pieces use
numpy/scipy library primitives (matrix build by unit vectors, LU, eigh, ARPACK).

Layouts are the canonical ones of the C-ABI (see ``laph_oracle.c``).  All arrays are
numpy complex128, C-contiguous.

Parity status: every function here is pinned by a CPU test against closed forms,
invariants or a library routine (tests/test_oracle_*.py), except where a docstring
says "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "laph_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O2 -fopenmp; -fcx-limited-range selects the
    textbook complex product and quotient instead of the libgcc calls with inf/nan
    recovery).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fcx-limited-range", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_L = ctypes.c_long
_U = ctypes.c_uint


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(build())
            sig = {
                "or_stout_spatial": (None, [_P, _P, _I, _I, _D, _I]),
                "or_plaquette_spatial": (_D, [_P, _I, _I]),
                "or_laplacian": (None, [_P, _P, _P, _I, _I]),
                "or_laplacian_slice": (None, [_P, _P, _P, _I, _I, _I]),
                "or_chebyshev": (None, [_P, _P, _P, _I, _I, _D, _D, _I]),
                "or_philox4x32_10": (None, [_P, _P, _P]),
                "or_z4_noise": (None, [_U, _U, _I, _I, _P]),
                "or_dilution_count": (_I, [_I, _I, _I]),
                "or_dilution_member": (_I, [_I, _I, _I, _I, _I]),
                "or_source": (_I, [_P, _P, _I, _I, _I, _P, _L, _P]),
                "or_sink_project": (None, [_P, _P, _I, _I, _I, _P]),
                "or_gamma": (None, [_I, _P]),
                "or_clover": (None, [_P, _I, _I, _D, _D, _D, _P]),
                "or_dirac": (None, [_P, _P, _I, _I, _D, _D, _I, _P, _P]),
                "or_omega": (None, [_P, _P, _I, _I, _D, _D, _I, _P, _P]),
                "or_dense_operator": (None, [_P, _P, _I, _I, _D, _D, _I, _P]),
                "or_cgnr": (_I, [_P, _P, _I, _I, _D, _D, _P, _P, _D, _I, _P]),
                "or_meson_function": (None, [_P, _P, _I, _I, _P, _P, _P, _P, _P]),
                "or_displace": (None, [_P, _I, _I, _I, _I, _I, _P, _P]),
                "or_baryon_function": (None, [_P, _P, _P, _I, _I, _P, _P, _P]),
                "or_mom_overlap": (None, [_P, _P, _I, _I, _I, _I, _P, _P]),
            }
            for name, (res, args) in sig.items():
                f = getattr(lib, name)
                f.restype = res
                f.argtypes = args
            _lib = lib
    return _lib


def _c(a, dtype=np.complex128):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def dims_from_links(U):
    """(Ns, Nt) from a link array of shape [Nt, Ns, Ns, Ns, 4, 3, 3]."""
    return U.shape[1], U.shape[0]


# ----------------------------------------------------------------- gauge field

def stout_spatial(U, rho, nsteps):
    """Spatial stout smearing, Sec. II (stout links, spatial staples only)."""
    lib = _load()
    U = _c(U)
    ns, nt = dims_from_links(U)
    out = np.empty_like(U)
    lib.or_stout_spatial(_ptr(U), _ptr(out), ns, nt, float(rho), int(nsteps))
    return out


def plaquette_spatial(U):
    lib = _load()
    U = _c(U)
    ns, nt = dims_from_links(U)
    return lib.or_plaquette_spatial(_ptr(U), ns, nt)


# ------------------------------------------------------------------- Laplacian

def laplacian(U, v):
    """(Lap v) per time slice, Sec. II Laplacian definition.  v: [Nt,Ns,Ns,Ns,3]."""
    lib = _load()
    U = _c(U)
    v = _c(v)
    ns, nt = dims_from_links(U)
    out = np.empty_like(v)
    lib.or_laplacian(_ptr(U), _ptr(v), _ptr(out), ns, nt)
    return out


def laplacian_slice(U, t, v3):
    lib = _load()
    U = _c(U)
    v3 = _c(v3)
    ns, nt = dims_from_links(U)
    out = np.empty_like(v3)
    lib.or_laplacian_slice(_ptr(U), _ptr(v3), _ptr(out), ns, nt, int(t))
    return out


def chebyshev(U, v, lam_l, lam_c, order):
    """T_order(B) v with B = 1 + 2/(lam_l-lam_c)(Lap + lam_c), Sec. IV."""
    lib = _load()
    U = _c(U)
    v = _c(v)
    ns, nt = dims_from_links(U)
    out = np.empty_like(v)
    lib.or_chebyshev(_ptr(U), _ptr(v), _ptr(out), ns, nt, float(lam_l), float(lam_c), int(order))
    return out


def phase_fix(vec):
    """Frozen eigenvector phase convention (Sec. IV asks for one but does not state it):
    the first component, in storage order, whose modulus is at least 0.1 of the largest
    modulus is made real and positive."""
    v = np.asarray(vec, dtype=np.complex128).ravel()
    a = np.abs(v)
    i = int(np.argmax(a >= 0.1 * a.max()))
    return (v * (np.conj(v[i]) / a[i])).reshape(np.shape(vec))


def laplacian_slice_matrix(U, t):
    """Dense matrix of -Lap on slice t, built by applying the oracle to unit vectors."""
    ns, nt = dims_from_links(U)
    n = ns ** 3 * 3
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((ns, ns, ns, 3), dtype=np.complex128)
    for j in range(n):
        e.reshape(-1)[j] = 1.0
        M[:, j] = -laplacian_slice(U, t, e).reshape(-1)
        e.reshape(-1)[j] = 0.0
    return M


def laph_eigpairs(U_smeared, nv, slices=None, method="auto", extra=0):
    """The LapH subspace (Sec. II, Eq. smearA and the V_s definition): on every time
    slice the nv lowest eigenvalues of -Lap (ascending) with unit eigenvectors in the
    frozen phase convention.  The plain definition is used: dense Hermitian eigh
    (LAPACK) when the slice dimension is <= 4000, otherwise ARPACK on the oracle
    Laplacian (tol 1e-13).  extra > 0 returns that many further eigenvalues (for gap
    reporting).  Returns (evals [len(slices), nv+extra], evecs [len(slices), nv, Ns,Ns,Ns,3]).
    """
    ns, nt = dims_from_links(U_smeared)
    slices = list(range(nt)) if slices is None else list(slices)
    n = ns ** 3 * 3
    k = nv + extra
    evals = np.empty((len(slices), k))
    evecs = np.empty((len(slices), nv, ns, ns, ns, 3), dtype=np.complex128)
    use_dense = (method == "dense") or (method == "auto" and n <= 4000)
    for si, t in enumerate(slices):
        if use_dense:
            M = laplacian_slice_matrix(U_smeared, t)
            w, X = np.linalg.eigh(M)
            w, X = w[:k], X[:, :k]
        else:
            import scipy.sparse.linalg as sla

            def mv(x, t=t):
                return -laplacian_slice(U_smeared, t, x.reshape(ns, ns, ns, 3)).reshape(-1)

            op = sla.LinearOperator((n, n), matvec=mv, dtype=np.complex128)
            w, X = sla.eigsh(op, k=k, which="SA", tol=1e-13, ncv=max(2 * k + 20, 60))
            order = np.argsort(w)
            w, X = w[order], X[:, order]
        evals[si] = w
        for j in range(nv):
            evecs[si, j] = phase_fix(X[:, j]).reshape(ns, ns, ns, 3)
    return evals, evecs


# ----------------------------------------------------------- noise and dilution

def philox4x32_10(ctr, key):
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, dtype=np.uint32)
    lib.or_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def z4_noise(s, k, nt, nv):
    """rho[t, alpha, n] in {1, i, -1, -i}; Sec. II (LapH-subspace noise) and Sec. IV
    (Z4 noise named by a 16-bit noise id s and a 16-bit configuration id k)."""
    lib = _load()
    rho = np.empty((nt, 4, nv), dtype=np.complex128)
    lib.or_z4_noise(int(s), int(k), int(nt), int(nv), _ptr(rho))
    return rho


DIL_TYPES = {"1": 0, "F": 1, "B": 2, "I": 3}


def parse_dilution(text, nt, nv):
    """Parse the paper's triplet notation, e.g. "TI16,SF,LI8" or "(TF, SF, LB4)"
    (Sec. II, dilution schemes).  Returns the 6-int scheme {typeT,JT,typeS,JS,typeL,JL}.
    Raises ValueError when N/J is not an integer."""
    parts = [p.strip() for p in text.strip().strip("()").split(",")]
    if len(parts) != 3:
        raise ValueError("need three dilution specifiers")
    out = []
    for want, p, N in zip("TSL", parts, (nt, 4, nv)):
        if not p or p[0].upper() != want:
            raise ValueError("bad specifier %r" % p)
        body = p[1:].upper()
        if body in ("1", "F"):
            out += [DIL_TYPES[body], 0]
            continue
        if body[:1] not in ("B", "I") or not body[1:].isdigit():
            raise ValueError("bad specifier %r" % p)
        J = int(body[1:])
        if J <= 0 or N % J != 0:
            raise ValueError("N/J is not an integer for %r" % p)
        out += [DIL_TYPES[body[0]], J]
    return out


def dilution_count(scheme, nt, nv):
    lib = _load()
    return (lib.or_dilution_count(scheme[0], scheme[1], nt)
            * lib.or_dilution_count(scheme[2], scheme[3], 4)
            * lib.or_dilution_count(scheme[4], scheme[5], nv))


def dilution_projector(scheme, nt, nv, b):
    """Diagonal of P^(b) over (t, alpha, n) as a 0/1 array [Nt,4,Nv] (Sec. II)."""
    lib = _load()
    nT = lib.or_dilution_count(scheme[0], scheme[1], nt)
    nS = lib.or_dilution_count(scheme[2], scheme[3], 4)
    nL = lib.or_dilution_count(scheme[4], scheme[5], nv)
    bL, bS, bT = b % nL, (b // nL) % nS, b // (nL * nS)
    P = np.zeros((nt, 4, nv))
    for t in range(nt):
        for a in range(4):
            for n in range(nv):
                P[t, a, n] = (lib.or_dilution_member(scheme[0], scheme[1], nt, t, bT)
                              and lib.or_dilution_member(scheme[2], scheme[3], 4, a, bS)
                              and lib.or_dilution_member(scheme[4], scheme[5], nv, n, bL))
    return P


def source(evecs, rho, scheme, b):
    """eta = V_s P^(b) rho  (Sec. IV), canonical spinor layout [Nt,Ns,Ns,Ns,4,3]."""
    lib = _load()
    evecs = _c(evecs)
    rho = _c(rho)
    nt, nv, ns = evecs.shape[0], evecs.shape[1], evecs.shape[2]
    sch = np.ascontiguousarray(scheme, dtype=np.int32)
    eta = np.empty((nt, ns, ns, ns, 4, 3), dtype=np.complex128)
    rc = lib.or_source(_ptr(evecs), _ptr(rho), ns, nt, nv, _ptr(sch), int(b), _ptr(eta))
    if rc != 0:
        raise ValueError("dilution index out of range")
    return eta


def sink_project(evecs, X):
    """coef[t, alpha, n] = sum_{x,c} conj(V_{t,n}(x,c)) X(x,t,c,alpha)  (Sec. IV)."""
    lib = _load()
    evecs = _c(evecs)
    X = _c(X)
    nt, nv, ns = evecs.shape[0], evecs.shape[1], evecs.shape[2]
    coef = np.empty((nt, 4, nv), dtype=np.complex128)
    lib.or_sink_project(_ptr(evecs), _ptr(X), ns, nt, nv, _ptr(coef))
    return coef


# --------------------------------------------------------------- Dirac operator

def gamma(mu):
    """gamma_{mu+1} for mu = 0..3, gamma_5 for mu = 4 (frozen chiral basis)."""
    lib = _load()
    g = np.empty((4, 4), dtype=np.complex128)
    lib.or_gamma(int(mu), _ptr(g))
    return g


def clover(U, m0, xi, csw):
    """Per-site 12x12 clover matrix A(x) (frozen anisotropic clover reading)."""
    lib = _load()
    U = _c(U)
    ns, nt = dims_from_links(U)
    A = np.empty((nt, ns, ns, ns, 12, 12), dtype=np.complex128)
    lib.or_clover(_ptr(U), ns, nt, float(m0), float(xi), float(csw), _ptr(A))
    return A


class Dirac:
    """K = A + H and Omega = gamma_4 K on a given gauge field (Sec. II: Omega = gamma_4 K)."""

    def __init__(self, U, m0, xi=3.5, csw=1.0, bc_t=-1.0):
        self.U = _c(U)
        self.ns, self.nt = dims_from_links(self.U)
        self.m0, self.xi, self.csw, self.bc_t = float(m0), float(xi), float(csw), float(bc_t)
        self.A = clover(self.U, m0, xi, csw)

    @property
    def shape(self):
        return (self.nt, self.ns, self.ns, self.ns, 4, 3)

    def K(self, psi, dagger=False):
        lib = _load()
        psi = _c(psi).reshape(self.shape)
        out = np.empty_like(psi)
        lib.or_dirac(_ptr(self.U), _ptr(self.A), self.ns, self.nt, self.xi, self.bc_t,
                     int(dagger), _ptr(psi), _ptr(out))
        return out

    def omega(self, psi, dagger=False):
        lib = _load()
        psi = _c(psi).reshape(self.shape)
        out = np.empty_like(psi)
        lib.or_omega(_ptr(self.U), _ptr(self.A), self.ns, self.nt, self.xi, self.bc_t,
                     int(dagger), _ptr(psi), _ptr(out))
        return out

    def dense(self, omega=True):
        lib = _load()
        N = 12 * self.ns ** 3 * self.nt
        Mt = np.empty((N, N), dtype=np.complex128)
        lib.or_dense_operator(_ptr(self.U), _ptr(self.A), self.ns, self.nt, self.xi,
                              self.bc_t, int(omega), _ptr(Mt))
        return Mt.T

    def solve(self, eta, tol=1e-13, maxiter=100000):
        """x = Omega^-1 eta by CG on the normal equations (the paper's fallback solver,
        Sec. IV).  Returns (x, iterations, true relative residual)."""
        lib = _load()
        eta = _c(eta).reshape(self.shape)
        x = np.empty_like(eta)
        tr = ctypes.c_double(0.0)
        it = lib.or_cgnr(_ptr(self.U), _ptr(self.A), self.ns, self.nt, self.xi, self.bc_t,
                         _ptr(eta), _ptr(x), float(tol), int(maxiter), ctypes.byref(tr))
        return x, it, tr.value

    def true_residual(self, eta, x):
        r = _c(eta).reshape(self.shape) - self.omega(x)
        return np.linalg.norm(r) / np.linalg.norm(eta)


def dense_solve(dirac: Dirac, B):
    """Omega^-1 B for the columns of B [12 V, k] by dense LU (tiny lattices only)."""
    import scipy.linalg as sla

    M = dirac.dense(omega=True)
    return sla.lu_solve(sla.lu_factor(M, check_finite=False), B, check_finite=False)


def laph_basis(evecs):
    """V_s as a dense [12 V, Nt 4 Nv] matrix: column (t, alpha, n) is eigenvector n of slice t
    placed in spin alpha (canonical spinor layout)."""
    nt, nv, ns = evecs.shape[0], evecs.shape[1], evecs.shape[2]
    V3 = ns ** 3
    Vfull = np.zeros((nt, V3, 4, 3, nt, 4, nv), dtype=np.complex128)
    for t in range(nt):
        for a in range(4):
            Vfull[t, :, a, :, t, a, :] = evecs[t].reshape(nv, V3, 3).transpose(1, 2, 0)
    return Vfull.reshape(nt * V3 * 12, nt * 4 * nv)


def perambulator(dirac: Dirac, evecs):
    """Exact tau = V_s^dag Omega^-1 V_s over (t,alpha,n) x (t',alpha',n') by dense LU
    (Sec. II, exact treatment of a quark line).  Only for tiny lattices."""
    nt, nv, ns = evecs.shape[0], evecs.shape[1], evecs.shape[2]
    M = dirac.dense(omega=True)
    V3 = ns ** 3
    N = 12 * V3 * nt
    D = nt * 4 * nv
    Vfull = np.zeros((N, D), dtype=np.complex128)
    # column (t, a, n) = eigvec n of slice t placed in spin a
    for t in range(nt):
        for a in range(4):
            for n in range(nv):
                col = np.zeros((nt, V3, 4, 3), dtype=np.complex128)
                col[t, :, a, :] = evecs[t, n].reshape(V3, 3)
                Vfull[:, (t * 4 + a) * nv + n] = col.reshape(-1)
    import scipy.linalg as sla

    X = sla.lu_solve(sla.lu_factor(M, check_finite=False), Vfull, check_finite=False)
    return Vfull.conj().T @ X


# ------------------------------------------------------------ hadron functions

def spin_apply(S, f):
    """S (4x4) applied to the spin index of a spinor field [..., 4, 3] or of LapH
    coefficients [..., 4, Nv] (axis -2 is the spin axis in both)."""
    return np.einsum("ab,...bc->...ac", np.asarray(S, dtype=np.complex128), f)


def smeared_field(evecs, coef):
    """The spinor field V_s coef of LapH coefficients coef[t, alpha, n]:
    f(x, t, c, alpha) = sum_n V_{t,n}(x, c) coef[t, alpha, n]."""
    nt, nv, ns = evecs.shape[0], evecs.shape[1], evecs.shape[2]
    V = evecs.reshape(nt, nv, ns ** 3, 3)
    f = np.einsum("tnxc,tan->txac", V, coef)
    return np.ascontiguousarray(f.reshape(nt, ns, ns, ns, 4, 3))


def quark_source(evecs, rho, scheme, b, bar=False):
    """The displaced-smeared-diluted quark source of Sec. II (Eq. varrhodef) with the
    trivial displacement, varrho^[b] = V_s P^(b) rho, as a full spinor field; with bar the
    source of the gamma_5-Hermitian estimate, -gamma_5 gamma_4 varrho^[b] (Eq. laphpropg5)."""
    f = source(evecs, rho, scheme, b)
    return -spin_apply(gamma(4) @ gamma(3), f) if bar else f


def quark_sink(evecs, X, bar=False):
    """The quark sink of Sec. II (Eq. varphidef) with the trivial displacement,
    varphi = S Omega^-1 V_s P^(b) rho with the LapH smearing S = V_s V_s^dag, for the
    solution X = Omega^-1 V_s P^(b) rho; with bar gamma_5 gamma_4 varphi (Eq. laphpropg5)."""
    f = smeared_field(evecs, sink_project(evecs, X))
    return spin_apply(gamma(4) @ gamma(3), f) if bar else f


def meson_function(f1, f2, c, k=(0, 0, 0), d1=(0, 0, 0), d2=(0, 0, 0)):
    """M(t) of Sec. III.B (Eq. mesonfunc) for full spinor fields f1, f2 [Nt,Ns,Ns,Ns,4,3]
    (f1 enters complex conjugated), spin matrix c (4x4), momentum 2 pi k / Ns and field
    displacements d1, d2."""
    lib = _load()
    f1 = _c(f1)
    f2 = _c(f2)
    nt, ns = f1.shape[0], f1.shape[1]
    c16 = _c(np.asarray(c, dtype=np.complex128).reshape(16))
    ka = np.ascontiguousarray(k, dtype=np.int32)
    a1 = np.ascontiguousarray(d1, dtype=np.int32)
    a2 = np.ascontiguousarray(d2, dtype=np.int32)
    out = np.empty(nt, dtype=np.complex128)
    lib.or_meson_function(_ptr(f1), _ptr(f2), ns, nt, _ptr(c16), _ptr(ka), _ptr(a1), _ptr(a2), _ptr(out))
    return out


def displace(U, v, direction, sign, length=3):
    """Covariant displacement of a colour field v [Nt,Ns,Ns,Ns,3] by `length` links along
    spatial direction 0..2 with sign +-1 (Sec. II, displacement types D^(j))."""
    lib = _load()
    U = _c(U)
    v = _c(v)
    ns, nt = dims_from_links(U)
    out = np.empty_like(v)
    lib.or_displace(_ptr(U), ns, nt, int(direction), int(sign), int(length), _ptr(v), _ptr(out))
    return out


def displace_spinor(U, f, direction, sign, length=3):
    """The displacement applied to every spin component of a spinor field [...,4,3]."""
    out = np.empty_like(f)
    for a in range(4):
        out[..., a, :] = displace(U, np.ascontiguousarray(f[..., a, :]), direction, sign, length)
    return out


def displace_evecs(U, evecs, direction, sign, length=3):
    """The displacement of every vector of an eigenvector-layout array [Nt,n,Ns,Ns,Ns,3]
    (vectors of one slice stay on that slice)."""
    nt, n = evecs.shape[0], evecs.shape[1]
    out = np.empty_like(evecs)
    for j in range(n):
        full = np.ascontiguousarray(evecs[:, j])  # [Nt, Ns, Ns, Ns, 3]: a field on the whole lattice
        out[:, j] = displace(U, full, direction, sign, length)
    return out


def mom_overlap(a, b, k=(0, 0, 0)):
    """O[t][n][m] = sum_x exp(-i 2 pi k.x / Ns) sum_c conj(a_n) b_m on every slice, for
    eigenvector-layout arrays a [Nt,na,Ns,Ns,Ns,3] and b [Nt,nb,...]."""
    lib = _load()
    a = _c(a)
    b = _c(b)
    nt, na, ns = a.shape[0], a.shape[1], a.shape[2]
    nb = b.shape[1]
    ka = np.ascontiguousarray(k, dtype=np.int32)
    out = np.empty((nt, na, nb), dtype=np.complex128)
    lib.or_mom_overlap(_ptr(a), _ptr(b), ns, nt, na, nb, _ptr(ka), _ptr(out))
    return out


def baryon_function(f1, f2, f3, c, k=(0, 0, 0)):
    """B(t) of Sec. III.A (Eq. baryonfunc) for three full spinor fields [Nt,Ns,Ns,Ns,4,3],
    spin tensor c (4x4x4) and momentum 2 pi k / Ns."""
    lib = _load()
    f1, f2, f3 = _c(f1), _c(f2), _c(f3)
    nt, ns = f1.shape[0], f1.shape[1]
    c64 = _c(np.asarray(c, dtype=np.complex128).reshape(64))
    ka = np.ascontiguousarray(k, dtype=np.int32)
    out = np.empty(nt, dtype=np.complex128)
    lib.or_baryon_function(_ptr(f1), _ptr(f2), _ptr(f3), ns, nt, _ptr(c64), _ptr(ka), _ptr(out))
    return out


# the six orderings of Eq. baryoncorr's source functions: (order of the noises 1, 2, 3 in
# the function, sign of the Wick contraction)
BARYON_PERMUTATIONS = [((0, 1, 2), +1), ((0, 2, 1), -1), ((1, 0, 2), -1), ((2, 1, 0), -1), ((1, 2, 0), +1),
                       ((2, 0, 1), +1)]


def baryon_correlator(snk, src, t0):
    """Eq. baryoncorr for three quark lines of one flavour: snk[t][b1][b2][b3] =
    B^[b1 b2 b3](varphi_1, varphi_2, varphi_3; t), src[s] (s over BARYON_PERMUTATIONS) =
    B(varrho_s1, varrho_s2, varrho_s3; t) indexed by the dilution indices in that order;
    C[tF] = sum_{b1 b2 b3} snk[tF][b1][b2][b3] conj(sum_s sign_s src[s][t0][b_s1][b_s2][b_s3])."""
    nt = snk.shape[0]
    out = np.zeros(nt, dtype=np.complex128)
    for (order, sign), S in zip(BARYON_PERMUTATIONS, src):
        # src[s][t0][b_order0][b_order1][b_order2] as a function of (b1, b2, b3)
        inv = np.argsort(order)
        St = np.transpose(S[t0], inv)
        out += sign * np.einsum("tijk,ijk->t", snk, St.conj())
    return out


# ------------------------------------------------------- Krylov reference solvers

def bicgstab(apply, b, tol=1e-10, maxiter=10000, trace=None):
    """BiCGStab (van der Vorst, SIAM J. Sci. Stat. Comput. 13 (1992) 631), the solver the
    paper names for Omega x = eta (Sec. IV), here unpreconditioned, from x = 0 with the
    shadow residual equal to the first residual.  apply(v) -> A v on flat vectors.
    Stops when the iterated residual |r_k| <= tol |b|, on a breakdown (rho, <r0, v> or
    omega exactly zero) or at maxiter.  Returns (x, k, history): k > 0 converged after k
    iterations, k < 0 stopped after |k| without converging; history[k] = |r_k| / |b|.
    trace: a list that receives (s, t, r) of every iteration (the half-step residual, its
    image and the new residual), for the tests of the stabilising step."""
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    r = b.copy()
    r0 = r.copy()
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    rho = alpha = omega = 1.0 + 0j
    hist = [1.0]
    for k in range(1, maxiter + 1):
        rho_new = np.vdot(r0, r)
        if rho_new == 0:
            return x, -k, hist
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = apply(p)
        den = np.vdot(r0, v)
        if den == 0:
            return x, -k, hist
        alpha = rho_new / den
        s = r - alpha * v
        t = apply(s)
        tt = np.vdot(t, t).real
        omega = np.vdot(t, s) / tt if tt > 0 else 0.0
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho = rho_new
        if trace is not None:
            trace.append((s.copy(), t.copy(), r.copy()))
        hist.append(float(np.linalg.norm(r) / nb))
        if hist[-1] <= tol:
            return x, k, hist
        if omega == 0:
            return x, -k, hist
    return x, -maxiter, hist


class EvenOdd:
    """The Schur complement of K = A + H on odd sites ((x + y + z + t) odd), the system the
    paper's even-odd preconditioned solver iterates (Sec. IV), written as the library's
    form Mhat = 1 - A_oo^-1 H_oe A_ee^-1 H_eo.  For Omega x = eta (K x = y with
    y = gamma_4 eta, Sec. II) the odd part of x solves Mhat x_o = bhat with
    bhat = A_oo^-1 (y_o - H_oe A_ee^-1 y_e), and x_e = A_ee^-1 (y_e - H_eo x_o).
    Fields are full-lattice arrays [Nt,Ns,Ns,Ns,4,3] (zero off their parity); H is K - A
    applied through the oracle's K, A^-1 is the site-wise inverse of the clover matrix."""

    def __init__(self, dirac: Dirac):
        self.D = dirac
        ns, nt = dirac.ns, dirac.nt
        t, z, y, x = np.meshgrid(*(np.arange(n) for n in (nt, ns, ns, ns)), indexing="ij")
        self.odd = (((x + y + z + t) % 2) == 1)[..., None, None].astype(np.float64)
        self.even = 1.0 - self.odd
        self.Ainv = np.linalg.inv(dirac.A)
        self.g4 = gamma(3)

    def _site(self, M, psi):
        sh = psi.shape
        return np.einsum("...ij,...j->...i", M, psi.reshape(sh[:-2] + (12,))).reshape(sh)

    def hop(self, psi):
        return self.D.K(psi) - self._site(self.D.A, psi)

    def mhat(self, xo):
        xo = xo.reshape(self.D.shape) * self.odd
        w = self._site(self.Ainv, self.hop(xo) * self.even)
        return xo - self._site(self.Ainv, self.hop(w) * self.odd)

    def y(self, eta):
        return np.einsum("ab,...bc->...ac", self.g4, eta.reshape(self.D.shape))

    def bhat(self, eta):
        y = self.y(eta)
        w = self._site(self.Ainv, y * self.even)
        return self._site(self.Ainv, (y - self.hop(w)) * self.odd)

    def full(self, xo, eta):
        xo = xo.reshape(self.D.shape) * self.odd
        y = self.y(eta)
        return xo + self._site(self.Ainv, (y - self.hop(xo)) * self.even)


def bicgstab_solve(dirac: Dirac, eta, tol=1e-10, maxiter=10000, even_odd=True):
    """Omega^-1 eta by BiCGStab, on the even-odd system (the paper's form, Sec. IV) or on
    the full K x = gamma_4 eta (the same x; Omega = gamma_4 K itself is indefinite, and
    BiCGStab stalls on it even far from the critical mass).  The iteration stops at tol
    on its own residual (of Mhat x_o = bhat, or of K x = y).  Returns (x, k, history,
    true relative residual of Omega x = eta)."""
    if even_odd:
        eo = EvenOdd(dirac)
        b = eo.bhat(eta)
        xo, k, hist = bicgstab(lambda v: eo.mhat(v).reshape(-1), b, tol, maxiter)
        x = eo.full(xo, eta)
    else:
        y = np.einsum("ab,...bc->...ac", gamma(3), np.asarray(eta).reshape(dirac.shape))
        x, k, hist = bicgstab(lambda v: dirac.K(v).reshape(-1), y, tol, maxiter)
        x = x.reshape(dirac.shape)
    return x, k, hist, dirac.true_residual(eta, x)

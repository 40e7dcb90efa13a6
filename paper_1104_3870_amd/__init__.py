"""MI355X stochastic-LapH hot path (arXiv:1104.3870) -- Python binding of liblaph.so.

Argument marshalling only: every step runs in the HIP kernels of ``liblaph.so``.  Device
memory is owned by torch tensors (complex128 fields, or float64 with a trailing
(re, im) axis), the library's workspace included: before each call the binding asks the
library how much workspace the call needs (laph_workspace_bytes) and, when the context's
workspace tensor is smaller, allocates a larger one and hands it over
(laph_set_workspace).  The library works on the stream passed at context creation
(default: torch's current stream).  The binding raises if the library has not been
built, and it never falls back to any CPU computation.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblaph.so")

LAPH_OK, LAPH_EINVAL, LAPH_EDIVIDE, LAPH_ENOCONV, LAPH_EEIG, LAPH_EHIP, LAPH_ENOMEM = range(7)
LAPH_DIL_NONE, LAPH_DIL_FULL, LAPH_DIL_BLOCK, LAPH_DIL_INTERLACE = range(4)
LAPH_OP_K, LAPH_OP_OMEGA, LAPH_OP_KDAG = range(3)
LAPH_PREC_F64, LAPH_PREC_F32, LAPH_PREC_F16, LAPH_PREC_BF16 = range(4)
LAPH_SOLVER_BICGSTAB, LAPH_SOLVER_CGNR, LAPH_SOLVER_FGMRES = range(3)
LAPH_HOP_PLAIN, LAPH_HOP_INV, LAPH_HOP_INV_DAG, LAPH_HOP_PLAIN_CG, LAPH_HOP_INV_DOT = range(5)
LAPH_DTYPE_C128, LAPH_DTYPE_C64 = range(2)
LAPH_SINK_NOALLOC_BYTES = 64 << 20  # fixed scratch of sink_project_noalloc (include/laph.h)
PRECISIONS = {"f64": LAPH_PREC_F64, "f32": LAPH_PREC_F32, "f16": LAPH_PREC_F16, "bf16": LAPH_PREC_BF16}


class LaphError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(msg)
        self.code = code


class laph_geom(ctypes.Structure):
    _fields_ = [("ns", ctypes.c_int), ("nt", ctypes.c_int)]


class laph_stout(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_double), ("nsteps", ctypes.c_int)]


class laph_lanczos(ctypes.Structure):
    _fields_ = [("krylov_dim", ctypes.c_int), ("cheb_order", ctypes.c_int), ("lambda_L", ctypes.c_double),
                ("lambda_C", ctypes.c_double), ("tol", ctypes.c_double), ("max_restarts", ctypes.c_int),
                ("seed", ctypes.c_uint32)]


class laph_eig_stats(ctypes.Structure):
    _fields_ = [("restarts", ctypes.c_int), ("matvecs", ctypes.c_int), ("max_residual", ctypes.c_double),
                ("max_orth", ctypes.c_double), ("min_gap", ctypes.c_double)]


class laph_dilution(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int * 3), ("J", ctypes.c_int * 3)]


class laph_dirac(ctypes.Structure):
    _fields_ = [("m0", ctypes.c_double), ("xi", ctypes.c_double), ("c_sw", ctypes.c_double),
                ("bc_t", ctypes.c_double)]


class laph_hop(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("mode", ctypes.c_int), ("parity", ctypes.c_int),
                ("gamma5", ctypes.c_int), ("temporal_gauge", ctypes.c_int), ("walk", ctypes.c_int),
                ("sites_per_block", ctypes.c_int), ("a", ctypes.c_double), ("c", ctypes.c_double)]


class laph_ws_params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("nv", ctypes.c_int), ("krylov_dim", ctypes.c_int), ("precision", ctypes.c_int),
                ("solver", ctypes.c_void_p), ("hop", ctypes.c_void_p), ("net", ctypes.c_void_p),
                ("n2", ctypes.c_int), ("n3", ctypes.c_int)]


class laph_solver(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int), ("solver", ctypes.c_int),
                ("precision", ctypes.c_int), ("reliable_every", ctypes.c_int), ("block_rhs", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("net", ctypes.c_void_p), ("restart", ctypes.c_int),
                ("reliable_delta", ctypes.c_double), ("dir_buffers", ctypes.c_int)]


class laph_tune_entry(ctypes.Structure):
    _fields_ = [("block_rhs", ctypes.c_int), ("sites_per_block", ctypes.c_int), ("ms_per_rhs", ctypes.c_double)]


class laph_tune_report(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("e", laph_tune_entry * 24), ("best_block_rhs", ctypes.c_int),
                ("best_sites_per_block", ctypes.c_int)]


class laph_adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double), ("loss_parity", ctypes.c_int)]


class laph_solve_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int), ("fallback_used", ctypes.c_int),
                ("true_resid", ctypes.c_double)]


class laph_kernel_timing(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_char * 48), ("ms", ctypes.c_double), ("launches", ctypes.c_long),
                ("bytes", ctypes.c_double)]


class laph_timing(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("k", laph_kernel_timing * 8)]


_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double

EXPORTS = {
    "laph_create": (_I, [ctypes.POINTER(_P), ctypes.POINTER(laph_geom), _P]),
    "laph_destroy": (_I, [_P]),
    "laph_strerror": (ctypes.c_char_p, [_I]),
    "laph_last_error": (ctypes.c_char_p, [_P]),
    "laph_forget_gauge": (_I, [_P]),
    "laph_device_bytes": (ctypes.c_size_t, [_P]),
    "laph_stout_smear": (_I, [_P, _P, ctypes.POINTER(laph_stout), _P]),
    "laph_laplacian_apply": (_I, [_P, _P, _P, _P]),
    "laph_chebyshev_apply": (_I, [_P, _P, _D, _D, _I, _P, _P]),
    "laph_eigvecs": (_I, [_P, _P, ctypes.POINTER(laph_stout), ctypes.POINTER(laph_lanczos), _I, _P, _P,
                          ctypes.POINTER(laph_eig_stats)]),
    "laph_parse_dilution": (_I, [ctypes.c_char_p, _I, _I, ctypes.POINTER(laph_dilution)]),
    "laph_dilution_count": (ctypes.c_long, [ctypes.POINTER(laph_dilution), _I, _I]),
    "laph_z4_noise": (_I, [_P, ctypes.c_uint16, ctypes.c_uint16, _I, _P]),
    "make_diluted_source": (_I, [_P, _P, _I, ctypes.c_uint16, ctypes.c_uint16, ctypes.POINTER(laph_dilution),
                                 ctypes.c_int64, _I, _P, _I]),
    "laph_dirac_apply": (_I, [_P, _P, ctypes.POINTER(laph_dirac), _I, _P, _P, _I]),
    "laph_hop_apply": (_I, [_P, _P, ctypes.POINTER(laph_dirac), ctypes.POINTER(laph_hop), _P, _P, _P, _P, _P, _P,
                            _I]),
    "dirac_solve": (_I, [_P, _P, ctypes.POINTER(laph_dirac), _P, _P, _I, ctypes.POINTER(laph_solver),
                         ctypes.POINTER(laph_solve_stats)]),
    "sink_project": (_I, [_P, _P, _I, _P, _I, _P]),
    "sink_project_noalloc": (_I, [_P, _P, _I, _P, _I, _P]),
    "laph_quark_source": (_I, [_P, _I, ctypes.c_uint16, ctypes.c_uint16, ctypes.POINTER(laph_dilution), ctypes.c_int64,
                               _I, _I, _P]),
    "laph_spin_apply": (_I, [_P, _P, _P, _I, _I, _P]),
    "laph_displace": (_I, [_P, _P, _I, _I, _I, _P, _I, _P]),
    "laph_baryon_tensor": (_I, [_P, _P, _I, _P, _P]),
    "laph_baryon_function": (_I, [_P, _P, _I, _P, _P, _I, _P, _I, _P, _I, _P]),
    "laph_baryon_correlator": (_I, [_P, _P, _P, _I, _I, _P]),
    "laph_mom_overlap": (_I, [_P, _P, _I, _P, _I, _P, _P]),
    "laph_overlap_apply": (_I, [_P, _P, _I, _I, _P, _I, _P]),
    "laph_meson_function": (_I, [_P, _P, _P, _I, _P, _I, _I, _I, _P]),
    "laph_meson_correlator": (_I, [_P, _P, _P, _I, _I, _I, _I, _P]),
    "laph_ptnet_create": (_I, [_P, _I, ctypes.POINTER(_I), ctypes.c_uint64, ctypes.POINTER(_P)]),
    "laph_ptnet_destroy": (_I, [_P]),
    "laph_ptnet_num_weights": (_I, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "laph_ptnet_get_weights": (_I, [_P, _P]),
    "laph_ptnet_set_weights": (_I, [_P, _P]),
    "laph_ptnet_forward": (_I, [_P, _P, _P, _D, _P, _P, _I]),
    "laph_ptnet_backward": (_I, [_P, _P, _P, _D, _P, _P, _P, _P, _I]),
    "laph_ptnet_train_step": (_I, [_P, _P, _P, _D, _P, _P, _I, ctypes.POINTER(laph_adam), ctypes.POINTER(_D)]),
    "laph_autotune": (_I, [_P, _P, ctypes.POINTER(laph_dirac), _I, ctypes.POINTER(laph_tune_report)]),
    "laph_workspace_bytes": (ctypes.c_size_t, [_P, _I, _P]),
    "laph_set_workspace": (_I, [_P, _P, ctypes.c_size_t]),
    "laph_set_timing": (_I, [_P, _I]),
    "laph_get_timing": (_I, [_P, ctypes.POINTER(laph_timing), _I]),
}


def lib():
    """Load liblaph.so (raises when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("liblaph.so not built: run __graft_entry__.build() "
                              "(python -m paper_1104_3870_amd.build)")
        # torch ships its own HIP runtime under the same soname; load it first so that
        # liblaph.so binds to that copy and torch's streams and allocations are valid
        # in the library (one runtime per process).
        import torch  # noqa: F401

        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc, ctx=None):
    if rc != LAPH_OK:
        L = lib()
        detail = L.laph_last_error(ctx).decode() if ctx else ""
        raise LaphError(rc, "%s%s" % (L.laph_strerror(rc).decode(), (": " + detail) if detail else ""))


def _dptr(t, dtype=None):
    """Device pointer of a contiguous CUDA tensor."""
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError("expected %s, got %s" % (dtype, t.dtype))
    return ctypes.c_void_p(t.data_ptr())


def _hptr(a):
    """Host pointer of a contiguous float64 (or complex128) numpy array."""
    import numpy as np

    if not isinstance(a, np.ndarray) or not a.flags.c_contiguous or a.dtype not in (np.float64, np.complex128):
        raise TypeError("expected a contiguous float64/complex128 numpy array")
    return ctypes.c_void_p(a.ctypes.data)


# ------------------------------------------------------------------ workspace
(LAPH_WS_STOUT, LAPH_WS_LAPLACIAN, LAPH_WS_CHEBYSHEV, LAPH_WS_EIGVECS, LAPH_WS_NOISE, LAPH_WS_SOURCE,
 LAPH_WS_DIRAC_APPLY, LAPH_WS_HOP_APPLY, LAPH_WS_SOLVE, LAPH_WS_AUTOTUNE, LAPH_WS_SINK, LAPH_WS_PTNET_FORWARD,
 LAPH_WS_PTNET_BACKWARD, LAPH_WS_PTNET_TRAIN, LAPH_WS_MOM_OVERLAP, LAPH_WS_BARYON_TENSOR,
 LAPH_WS_BARYON_FUNCTION) = range(17)

_WS = {}  # context handle value -> workspace tensor


def _key(ctx):
    return ctx.value if isinstance(ctx, ctypes.c_void_p) else int(ctx)


def laph_workspace_bytes(ctx, op, n=0, nv=0, krylov_dim=0, precision=0, solver=None, hop=None, net=None, n2=0,
                         n3=0):
    p = laph_ws_params(n, nv, krylov_dim, precision,
                       ctypes.cast(ctypes.pointer(solver), ctypes.c_void_p) if solver is not None else None,
                       ctypes.cast(ctypes.pointer(hop), ctypes.c_void_p) if hop is not None else None,
                       net.handle if isinstance(net, PTNet) else net, n2, n3)
    need = lib().laph_workspace_bytes(ctx, op, ctypes.byref(p))
    if need == 0:
        raise LaphError(LAPH_EINVAL, "laph_workspace_bytes: invalid op or parameters")
    return need


def laph_set_workspace(ctx, tensor):
    """Hand the context a workspace tensor (device, any dtype; None releases it)."""
    if tensor is None:
        _check(lib().laph_set_workspace(ctx, None, 0), ctx)
        _WS.pop(_key(ctx), None)
        return
    ptr = _dptr(tensor)
    _check(lib().laph_set_workspace(ctx, ptr, tensor.numel() * tensor.element_size()), ctx)
    _WS[_key(ctx)] = tensor


def workspace(ctx):
    """The context's workspace tensor (None before the first call)."""
    return _WS.get(_key(ctx))


def ensure_workspace(ctx, op, **params):
    """Give the context a workspace of at least what `op` needs (grown, never shrunk)."""
    import torch

    need = laph_workspace_bytes(ctx, op, **params)
    cur = _WS.get(_key(ctx))
    have = cur.numel() if cur is not None else 0
    if have >= need:
        return cur
    size = max(need, have + have // 4)
    size = (size + (2 << 20) - 1) // (2 << 20) * (2 << 20)
    # release the old one to the library first (it waits for the stream), then to torch
    _check(lib().laph_set_workspace(ctx, None, 0), ctx)
    _WS.pop(_key(ctx), None)
    del cur
    t = torch.empty(size, dtype=torch.uint8, device="cuda")
    laph_set_workspace(ctx, t)
    return t


# ------------------------------------------------------------------ ABI names

def laph_create(ns, nt, stream=None):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    h = ctypes.c_void_p()
    _check(lib().laph_create(ctypes.byref(h), ctypes.byref(laph_geom(ns, nt)), ctypes.c_void_p(stream)))
    return h


def laph_destroy(ctx):
    _check(lib().laph_destroy(ctx))
    _WS.pop(_key(ctx), None)


def laph_forget_gauge(ctx):
    _check(lib().laph_forget_gauge(ctx), ctx)


def laph_parse_dilution(text, nt, nv):
    d = laph_dilution()
    _check(lib().laph_parse_dilution(text.encode(), nt, nv, ctypes.byref(d)))
    return d


def laph_dilution_count(dil, nt, nv):
    return lib().laph_dilution_count(ctypes.byref(dil), nt, nv)


def laph_stout_smear(ctx, U, rho, nsteps, out):
    ensure_workspace(ctx, LAPH_WS_STOUT)
    _check(lib().laph_stout_smear(ctx, _dptr(U), ctypes.byref(laph_stout(rho, nsteps)), _dptr(out)), ctx)


def laph_laplacian_apply(ctx, U, v, out):
    ensure_workspace(ctx, LAPH_WS_LAPLACIAN)
    _check(lib().laph_laplacian_apply(ctx, _dptr(U), _dptr(v), _dptr(out)), ctx)


def laph_chebyshev_apply(ctx, U, lam_l, lam_c, order, v, out):
    ensure_workspace(ctx, LAPH_WS_CHEBYSHEV)
    _check(lib().laph_chebyshev_apply(ctx, _dptr(U), lam_l, lam_c, order, _dptr(v), _dptr(out)), ctx)


def laph_eigvecs(ctx, U, rho, nsteps, nv, evals_host, evecs, krylov=160, cheb_order=8, lam_l=15.0, lam_c=0.5,
                 tol=1e-9, max_restarts=50, seed=12345):
    """evals_host: numpy float64 [Nt, Nv] (filled); evecs: device complex128 [Nt, Nv, Ns, Ns, Ns, 3]."""
    import numpy as np

    assert evals_host.dtype == np.float64 and evals_host.flags["C_CONTIGUOUS"]
    ensure_workspace(ctx, LAPH_WS_EIGVECS, nv=nv, krylov_dim=krylov)
    st = laph_eig_stats()
    lz = laph_lanczos(krylov, cheb_order, lam_l, lam_c, tol, max_restarts, seed)
    rc = lib().laph_eigvecs(ctx, _dptr(U), ctypes.byref(laph_stout(rho, nsteps)), ctypes.byref(lz), nv,
                            evals_host.ctypes.data_as(ctypes.c_void_p), _dptr(evecs), ctypes.byref(st))
    _check(rc, ctx)
    return st


def laph_z4_noise(ctx, s, k, nv, rho):
    ensure_workspace(ctx, LAPH_WS_NOISE)
    _check(lib().laph_z4_noise(ctx, s, k, nv, _dptr(rho)), ctx)


def make_diluted_source(ctx, evecs, nv, noise_s, config_k, dil, b_first, n_src, eta):
    """eta: device complex128 or complex64 tensor [n_src, Nt, Ns, Ns, Ns, 4, 3]; its dtype
    selects the element type the library writes."""
    import torch

    dt = {torch.complex128: LAPH_DTYPE_C128, torch.complex64: LAPH_DTYPE_C64}.get(eta.dtype)
    if dt is None:
        raise TypeError("eta must be complex128 or complex64")
    ensure_workspace(ctx, LAPH_WS_SOURCE, nv=nv)
    _check(lib().make_diluted_source(ctx, _dptr(evecs), nv, noise_s, config_k, ctypes.byref(dil), b_first, n_src,
                                     _dptr(eta), dt), ctx)


def laph_dirac_apply(ctx, U, dirac, op, x, out, n_fields=1):
    ensure_workspace(ctx, LAPH_WS_DIRAC_APPLY, n=n_fields)
    _check(lib().laph_dirac_apply(ctx, _dptr(U), ctypes.byref(dirac), op, _dptr(x), _dptr(out), n_fields), ctx)


def laph_hop_apply(ctx, U, dirac, precision, mode, parity, inp, out, x=None, out2=None, alpha=None, gamma5=0,
                   temporal_gauge=0, walk=0, sites_per_block=0, a=0.0, c=1.0):
    """One even-odd hopping launch (see laph.h); returns the host norm2 array (n values; for
    LAPH_HOP_INV_DOT 3 n: Re <y, out>, Im <y, out>, |out|^2 per field, y passed as out2)."""
    import numpy as np

    n = inp.shape[0]
    h = laph_hop(PRECISIONS[precision] if isinstance(precision, str) else precision, mode, parity, gamma5,
                 temporal_gauge, walk, sites_per_block, a, c)
    al = None
    if alpha is not None:
        al = np.ascontiguousarray(np.asarray(alpha, dtype=np.float64))
        if al.size != n:
            raise ValueError("alpha needs one value per field")
    nrm = np.zeros(3 * n if mode == LAPH_HOP_INV_DOT else n)
    if n <= 32:
        ensure_workspace(ctx, LAPH_WS_HOP_APPLY, n=n, hop=h)
    _check(lib().laph_hop_apply(ctx, _dptr(U), ctypes.byref(dirac), ctypes.byref(h), _dptr(inp),
                                _dptr(x) if x is not None else None, _dptr(out),
                                _dptr(out2) if out2 is not None else None,
                                al.ctypes.data_as(ctypes.c_void_p) if al is not None else None,
                                nrm.ctypes.data_as(ctypes.c_void_p), n), ctx)
    return nrm


def dirac_solve(ctx, U, dirac, eta, x, n_rhs, solver, raise_on_noconv=True):
    ensure_workspace(ctx, LAPH_WS_SOLVE, n=n_rhs, solver=solver)
    stats = (laph_solve_stats * n_rhs)()
    rc = lib().dirac_solve(ctx, _dptr(U), ctypes.byref(dirac), _dptr(eta), _dptr(x), n_rhs, ctypes.byref(solver),
                           stats)
    if rc == LAPH_ENOCONV and not raise_on_noconv:
        return list(stats)
    _check(rc, ctx)
    return list(stats)


def sink_project(ctx, evecs, nv, X, n_rhs, coef):
    ensure_workspace(ctx, LAPH_WS_SINK, nv=nv, n=n_rhs)
    _check(lib().sink_project(ctx, _dptr(evecs), nv, _dptr(X), n_rhs, _dptr(coef)), ctx)


def sink_project_noalloc(ctx, evecs, nv, X, n_rhs, coef):
    """sink_project with its partial sums in the library's fixed device array (no workspace)."""
    _check(lib().sink_project_noalloc(ctx, _dptr(evecs), nv, _dptr(X), n_rhs, _dptr(coef)), ctx)


def _spin16(S):
    import numpy as np

    a = np.ascontiguousarray(np.asarray(S, dtype=np.complex128).reshape(16))
    return a, a.ctypes.data_as(ctypes.c_void_p)


def laph_quark_source(ctx, nv, noise_s, config_k, dil, b_first, n_src, out, bar=False):
    """LapH coefficients of the quark sources varrho^[b] (or varrho-bar); out [n, Nt, 4, Nv]."""
    ensure_workspace(ctx, LAPH_WS_SOURCE, nv=nv)
    _check(lib().laph_quark_source(ctx, nv, noise_s, config_k, ctypes.byref(dil), b_first, n_src, int(bar),
                                   _dptr(out)), ctx)


def laph_spin_apply(ctx, S, inp, n, nv, out):
    keep, p = _spin16(S)
    _check(lib().laph_spin_apply(ctx, p, _dptr(inp), n, nv, _dptr(out)), ctx)


def laph_meson_function(ctx, c, a, n1, b, n2, nv, out, diag=False):
    keep, p = _spin16(c)
    _check(lib().laph_meson_function(ctx, p, _dptr(a), n1, _dptr(b), n2, nv, int(diag), _dptr(out)), ctx)


def laph_meson_correlator(ctx, snk, src, n1, n2, t0, out, diag=False):
    _check(lib().laph_meson_correlator(ctx, _dptr(snk), _dptr(src), n1, n2, int(diag), t0, _dptr(out)), ctx)


def laph_displace(ctx, U, direction, sign, length, v, n, out):
    """Covariant displacement of n colour fields per slice (eigenvector layout)."""
    _check(lib().laph_displace(ctx, _dptr(U), direction, sign, length, _dptr(v), n, _dptr(out)), ctx)


def laph_mom_overlap(ctx, a, na, b, nb, k, out):
    ensure_workspace(ctx, LAPH_WS_MOM_OVERLAP)
    import numpy as np

    ka = np.ascontiguousarray(k, dtype=np.int32)
    _check(lib().laph_mom_overlap(ctx, _dptr(a), na, _dptr(b), nb, ka.ctypes.data_as(ctypes.c_void_p), _dptr(out)),
           ctx)


def laph_overlap_apply(ctx, O, na, nb, b, n, out):
    _check(lib().laph_overlap_apply(ctx, _dptr(O), na, nb, _dptr(b), n, _dptr(out)), ctx)


def laph_baryon_tensor(ctx, evecs, nv, k, T):
    """T[t][n1][n2][n3] = sum_x e^{-ip.x} eps V_n1 V_n2 V_n3 (device [Nt, nv, nv, nv])."""
    import numpy as np

    ensure_workspace(ctx, LAPH_WS_BARYON_TENSOR)
    ka = np.ascontiguousarray(k, dtype=np.int32)
    _check(lib().laph_baryon_tensor(ctx, _dptr(evecs), nv, ka.ctypes.data_as(ctypes.c_void_p), _dptr(T)), ctx)


def laph_baryon_function(ctx, T, nv, c, f1, n1, f2, n2, f3, n3, out):
    import numpy as np

    ensure_workspace(ctx, LAPH_WS_BARYON_FUNCTION, nv=nv, n=n1, n2=n2, n3=n3)
    c64 = np.ascontiguousarray(np.asarray(c, dtype=np.complex128).reshape(64))
    _check(lib().laph_baryon_function(ctx, _dptr(T), nv, c64.ctypes.data_as(ctypes.c_void_p), _dptr(f1), n1,
                                      _dptr(f2), n2, _dptr(f3), n3, _dptr(out)), ctx)


def laph_baryon_correlator(ctx, snk, src, n, t0, out):
    _check(lib().laph_baryon_correlator(ctx, _dptr(snk), _dptr(src), n, t0, _dptr(out)), ctx)


def laph_autotune(ctx, U, dirac, precision="f16"):
    """Tune the block size and LDS tile of the hopping kernel; returns the report as a dict."""
    rep = laph_tune_report()
    prec = PRECISIONS[precision] if isinstance(precision, str) else precision
    ensure_workspace(ctx, LAPH_WS_AUTOTUNE, precision=prec)
    _check(lib().laph_autotune(ctx, _dptr(U), ctypes.byref(dirac), prec, ctypes.byref(rep)), ctx)
    return {"entries": [(rep.e[i].block_rhs, rep.e[i].sites_per_block, rep.e[i].ms_per_rhs) for i in range(rep.n)],
            "best_block_rhs": rep.best_block_rhs, "best_sites_per_block": rep.best_sites_per_block}


def laph_set_timing(ctx, enable):
    _check(lib().laph_set_timing(ctx, int(enable)), ctx)


def laph_get_timing(ctx, reset=False):
    """Per kernel variant: list of dicts {kernel, ms, launches, bytes}, by decreasing ms."""
    t = laph_timing()
    _check(lib().laph_get_timing(ctx, ctypes.byref(t), int(reset)), ctx)
    return [{"kernel": t.k[i].kernel.decode(), "ms": t.k[i].ms, "launches": t.k[i].launches,
             "bytes": t.k[i].bytes} for i in range(t.n)]


def solver_params(tol=1e-10, maxiter=20000, precision="f64", solver=LAPH_SOLVER_BICGSTAB, reliable_every=50,
                  block_rhs=1, use_graph=0, net=None, restart=0, reliable_delta=0.0, dir_buffers=0):
    """laph_solver; `net` is a PTNet (or raw handle) used by LAPH_SOLVER_FGMRES."""
    h = net.handle if isinstance(net, PTNet) else net
    return laph_solver(tol, maxiter, solver, PRECISIONS[precision] if isinstance(precision, str) else precision,
                       reliable_every, block_rhs, use_graph, h, restart, reliable_delta, dir_buffers)


def laph_ptnet_create(ctx, channels, seed=0):
    ch = (_I * len(channels))(*channels)
    h = _P()
    _check(lib().laph_ptnet_create(ctx, len(channels) - 1, ch, seed, ctypes.byref(h)), ctx)
    return h


def laph_ptnet_destroy(net):
    _check(lib().laph_ptnet_destroy(net))


def laph_ptnet_num_weights(net):
    n = ctypes.c_size_t()
    _check(lib().laph_ptnet_num_weights(net, ctypes.byref(n)))
    return n.value


def laph_ptnet_get_weights(net, w):
    """w: host float64 numpy array of 2n (or n complex128)."""
    _check(lib().laph_ptnet_get_weights(net, _hptr(w)))


def laph_ptnet_set_weights(net, w):
    _check(lib().laph_ptnet_set_weights(net, _hptr(w)))


def laph_ptnet_forward(ctx, net, U, bc_t, x, out, n_fields=1):
    ensure_workspace(ctx, LAPH_WS_PTNET_FORWARD, n=n_fields, net=net)
    _check(lib().laph_ptnet_forward(ctx, net, _dptr(U), bc_t, _dptr(x), _dptr(out), n_fields), ctx)


def laph_ptnet_backward(ctx, net, U, bc_t, x, gout, gin, gw, n_fields=1):
    ensure_workspace(ctx, LAPH_WS_PTNET_BACKWARD, n=n_fields, net=net)
    _check(lib().laph_ptnet_backward(ctx, net, _dptr(U), bc_t, _dptr(x), _dptr(gout),
                                     _dptr(gin) if gin is not None else None, _hptr(gw), n_fields), ctx)


def laph_ptnet_train_step(ctx, net, U, bc_t, b, x, n_pairs, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                          loss_parity=-1):
    loss = _D()
    opt = laph_adam(lr, beta1, beta2, eps, loss_parity)
    ensure_workspace(ctx, LAPH_WS_PTNET_TRAIN, n=n_pairs, net=net)
    _check(lib().laph_ptnet_train_step(ctx, net, _dptr(U), bc_t, _dptr(b), _dptr(x), n_pairs, ctypes.byref(opt),
                                       ctypes.byref(loss)), ctx)
    return loss.value


class PTNet:
    """Owner of one learned-preconditioner network."""

    def __init__(self, ctx, channels, seed=0):
        self.channels = list(channels)
        self.handle = laph_ptnet_create(ctx, self.channels, seed)

    @property
    def n_weights(self):
        return laph_ptnet_num_weights(self.handle)

    def get_weights(self):
        import numpy as np

        w = np.zeros(2 * self.n_weights)
        laph_ptnet_get_weights(self.handle, w)
        return w.view(np.complex128)

    def set_weights(self, w):
        import numpy as np

        w = np.ascontiguousarray(np.asarray(w, dtype=np.complex128).reshape(-1))
        if w.size != self.n_weights:
            raise ValueError("expected %d complex weights, got %d" % (self.n_weights, w.size))
        laph_ptnet_set_weights(self.handle, w.view(np.float64))

    def close(self):
        if self.handle:
            laph_ptnet_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Lattice:
    """Convenience owner of one context (geometry + stream)."""

    def __init__(self, ns, nt, stream=None):
        self.ns, self.nt = ns, nt
        self.ctx = laph_create(ns, nt, stream)

    def close(self):
        if self.ctx:
            laph_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""GPU parity of the individual hot-path kernels against the oracle (through the C-ABI).

Bars: bit-exact for the Z4 noise (Sec. IV); FP64 stencils (stout step of Sec. II,
Laplacian of Sec. II, Chebyshev map of Sec. IV, Wilson-clover K and Omega = gamma_4 K of
Sec. II) within 1e-13 relative; source and sink projection (Sec. IV) within 1e-14."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1104_3870_amd as P

    P.lib()
    return P


def _ctx(P, ns, nt):
    return P.Lattice(ns, nt)


@pytest.mark.parametrize("nt,nv,s,k", [(8, 8, 0, 1), (128, 112, 3, 77), (32, 48, 65535, 65535)])
def test_z4_noise_bitexact(P, nt, nv, s, k):
    import torch

    say("z4", nt, nv, s, k)
    L = _ctx(P, 4, nt)
    rho = torch.empty((nt, 4, nv), dtype=torch.complex128, device="cuda")
    P.laph_z4_noise(L.ctx, s, k, nv, rho)
    ref = oracle.z4_noise(s, k, nt, nv)
    assert np.array_equal(host(rho), ref)


@pytest.mark.parametrize("ns,nt,eps,rho,n", [(4, 8, 0.3, 0.1, 2), (6, 4, 0.9, 0.12, 3), (8, 2, 0.02, 0.1, 1)])
def test_stout_parity(P, ns, nt, eps, rho, n):
    import torch

    say("stout", ns, nt, eps, rho, n)
    U = synth.gauge_field(ns, nt, eps, 5)
    L = _ctx(P, ns, nt)
    out = torch.empty(U.shape, dtype=torch.complex128, device="cuda")
    P.laph_stout_smear(L.ctx, dev(U), rho, n, out)
    ref = oracle.stout_spatial(U, rho, n)
    assert np.abs(host(out) - ref).max() < 1e-13
    assert np.array_equal(host(out)[..., 3, :, :], U[..., 3, :, :])


@pytest.mark.parametrize("ns,nt,eps", [(4, 8, 0.3), (6, 4, 0.9), (16, 2, 0.4)])
def test_laplacian_and_chebyshev_parity(P, ns, nt, eps):
    import torch

    say("lap", ns, nt, eps)
    U = synth.gauge_field(ns, nt, eps, 6)
    v = synth.random_colour_field(ns, nt, 2)
    L = _ctx(P, ns, nt)
    out = torch.empty(v.shape, dtype=torch.complex128, device="cuda")
    P.laph_laplacian_apply(L.ctx, dev(U), dev(v), out)
    assert rel_err(host(out), oracle.laplacian(U, v)) < 1e-14
    for order in (1, 2, 3, 8):
        P.laph_chebyshev_apply(L.ctx, dev(U), 15.0, 0.5, order, dev(v), out)
        ref = oracle.chebyshev(U, v, 15.0, 0.5, order)
        assert rel_err(host(out), ref) < 1e-13, order


@pytest.mark.parametrize("ns,nt,eps,m0", [(4, 8, 0.3, -0.04), (6, 4, 0.9, 0.1), (8, 4, 0.5, -0.2), (16, 32, 0.4, -0.04)])
def test_dirac_apply_parity(P, ns, nt, eps, m0):
    import torch

    say("dirac", ns, nt, eps, m0)
    U = synth.gauge_field(ns, nt, eps, 7)
    D = oracle.Dirac(U, m0, 3.5, 1.0, -1.0)
    psi = synth.random_spinor(ns, nt, 3)
    L = _ctx(P, ns, nt)
    prm = P.laph_dirac(m0, 3.5, 1.0, -1.0)
    out = torch.empty(psi.shape, dtype=torch.complex128, device="cuda")
    Ud, pd = dev(U), dev(psi)
    for op, ref in ((P.LAPH_OP_K, D.K(psi)), (P.LAPH_OP_OMEGA, D.omega(psi)), (P.LAPH_OP_KDAG, D.K(psi, dagger=True))):
        P.laph_dirac_apply(L.ctx, Ud, prm, op, pd, out)
        got = host(out)
        assert rel_err(got, ref) < 1e-13, op
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max(), op


def test_dirac_apply_multi_field(P):
    import torch

    ns, nt = 4, 4
    U = synth.gauge_field(ns, nt, 0.5, 8)
    D = oracle.Dirac(U, 0.05, 3.5, 1.0, -1.0)
    psi = synth.random_spinor(ns, nt, 4, nrhs=3)
    L = _ctx(P, ns, nt)
    out = torch.empty(psi.shape, dtype=torch.complex128, device="cuda")
    P.laph_dirac_apply(L.ctx, dev(U), P.laph_dirac(0.05, 3.5, 1.0, -1.0), P.LAPH_OP_OMEGA, dev(psi), out, 3)
    for r in range(3):
        assert rel_err(host(out)[r], D.omega(psi[r])) < 1e-13


@pytest.mark.parametrize("ns,nt,n", [(6, 2, 8), (4, 8, 32), (6, 4, 5)])
def test_dirac_apply_many_fields(P, ns, nt, n):
    """FP64 hops on n >= 4 fields at once take the LDS-staged multi-RHS kernel (block of
    S sites x n lanes; 6^3 x 2 leaves a ragged last block)."""
    import torch

    U = synth.gauge_field(ns, nt, 0.6, 9)
    D = oracle.Dirac(U, -0.1, 3.5, 1.0, -1.0)
    psi = synth.random_spinor(ns, nt, 5, nrhs=n)
    L = _ctx(P, ns, nt)
    prm = P.laph_dirac(-0.1, 3.5, 1.0, -1.0)
    out = torch.empty(psi.shape, dtype=torch.complex128, device="cuda")
    for op in (P.LAPH_OP_K, P.LAPH_OP_OMEGA, P.LAPH_OP_KDAG):
        P.laph_dirac_apply(L.ctx, dev(U), prm, op, dev(psi), out, n)
        got = host(out)
        for r in (0, n // 2, n - 1):
            if op == P.LAPH_OP_K:
                ref = D.K(psi[r])
            elif op == P.LAPH_OP_OMEGA:
                ref = D.omega(psi[r])
            else:
                ref = D.K(psi[r], dagger=True)
            assert rel_err(got[r], ref) < 1e-13, (op, r)


@pytest.fixture(scope="module")
def ns4_nt8_evecs():
    cfg = synth.CONFIGS["ns4_nt8"]
    U = synth.gauge_field(cfg.ns, cfg.nt, cfg.eps, cfg.seed)
    S = oracle.stout_spatial(U, cfg.stout_rho, cfg.stout_steps)
    ev, V = oracle.laph_eigpairs(S, cfg.nv)
    return cfg, U, V


@pytest.mark.parametrize("spec,b0,nsrc", [("TF,SF,LF", 0, 1), ("TF,SF,LF", 200, 7), ("TI4,SB2,LI4", 3, 20),
                                          ("T1,S1,LB2", 0, 2)])
def test_source_parity(P, ns4_nt8_evecs, spec, b0, nsrc):
    import torch

    cfg, U, V = ns4_nt8_evecs
    say("source", spec, b0, nsrc)
    L = _ctx(P, cfg.ns, cfg.nt)
    dil = P.laph_parse_dilution(spec, cfg.nt, cfg.nv)
    eta = torch.empty((nsrc, cfg.nt, cfg.ns, cfg.ns, cfg.ns, 4, 3), dtype=torch.complex128, device="cuda")
    P.make_diluted_source(L.ctx, dev(V), cfg.nv, 0, 1, dil, b0, nsrc, eta)
    rho = oracle.z4_noise(0, 1, cfg.nt, cfg.nv)
    sch = oracle.parse_dilution(spec, cfg.nt, cfg.nv)
    for j in range(nsrc):
        ref = oracle.source(V, rho, sch, b0 + j)
        assert np.abs(host(eta)[j] - ref).max() < 1e-15


def test_source_complex64(P, ns4_nt8_evecs):
    """The complex64 form is the oracle's FP64 source rounded once to FP32."""
    import torch

    cfg, U, V = ns4_nt8_evecs
    L = _ctx(P, cfg.ns, cfg.nt)
    spec, b0, nsrc = "TI4,SB2,LI4", 5, 6
    dil = P.laph_parse_dilution(spec, cfg.nt, cfg.nv)
    eta = torch.empty((nsrc, cfg.nt, cfg.ns, cfg.ns, cfg.ns, 4, 3), dtype=torch.complex64, device="cuda")
    P.make_diluted_source(L.ctx, dev(V), cfg.nv, 0, 1, dil, b0, nsrc, eta)
    rho = oracle.z4_noise(0, 1, cfg.nt, cfg.nv)
    sch = oracle.parse_dilution(spec, cfg.nt, cfg.nv)
    got = host(eta)
    for j in range(nsrc):
        ref = oracle.source(V, rho, sch, b0 + j).astype(np.complex64)
        assert np.abs(got[j] - ref).max() <= 2.0 ** -23 * np.abs(ref).max()


def test_source_rejects_bad_index(P, ns4_nt8_evecs):
    import torch

    cfg, U, V = ns4_nt8_evecs
    L = _ctx(P, cfg.ns, cfg.nt)
    dil = P.laph_parse_dilution("TF,SF,LF", cfg.nt, cfg.nv)
    eta = torch.empty((1, cfg.nt, cfg.ns, cfg.ns, cfg.ns, 4, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(P.LaphError):
        P.make_diluted_source(L.ctx, dev(V), cfg.nv, 0, 1, dil, 256, 1, eta)


@pytest.mark.parametrize("nrhs", [1, 3])
def test_sink_parity(P, ns4_nt8_evecs, nrhs):
    import torch

    cfg, U, V = ns4_nt8_evecs
    L = _ctx(P, cfg.ns, cfg.nt)
    X = synth.random_spinor(cfg.ns, cfg.nt, 9, nrhs=nrhs)
    coef = torch.empty((nrhs, cfg.nt, 4, cfg.nv), dtype=torch.complex128, device="cuda")
    P.sink_project(L.ctx, dev(V), cfg.nv, dev(X), nrhs, coef)
    for r in range(nrhs):
        ref = oracle.sink_project(V, X[r])
        assert np.abs(host(coef)[r] - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("ns,nt,nv,nrhs", [(6, 4, 130, 20), (4, 2, 7, 17), (2, 2, 3, 1)])
def test_sink_tiles(P, ns, nt, nv, nrhs):
    """Ragged row tiles (nrhs x 4 spins over 64-row tiles), column tiles (N_v over 112) and
    site ranges (V3 not a multiple of the per-block range) of the tiled projection."""
    import torch

    rng = np.random.default_rng(11)
    V = rng.standard_normal((nt, nv, ns, ns, ns, 3)) + 1j * rng.standard_normal((nt, nv, ns, ns, ns, 3))
    X = synth.random_spinor(ns, nt, 4, nrhs=nrhs)
    L = _ctx(P, ns, nt)
    coef = torch.empty((nrhs, nt, 4, nv), dtype=torch.complex128, device="cuda")
    P.sink_project(L.ctx, dev(V), nv, dev(X), nrhs, coef)
    got = host(coef)
    for r in range(nrhs):
        ref = oracle.sink_project(V, X[r])
        assert np.abs(got[r] - ref).max() < 1e-13 * np.abs(ref).max(), r


def test_sink_parity_large_nv(P):
    """24^3 slices (the production slice size) with N_v = 112 on two time slices."""
    import torch

    ns, nt, nv = 24, 2, 112
    rng = np.random.default_rng(3)
    V = rng.standard_normal((nt, nv, ns, ns, ns, 3)) + 1j * rng.standard_normal((nt, nv, ns, ns, ns, 3))
    X = synth.random_spinor(ns, nt, 2, nrhs=1)
    L = _ctx(P, ns, nt)
    coef = torch.empty((1, nt, 4, nv), dtype=torch.complex128, device="cuda")
    P.sink_project(L.ctx, dev(V), nv, dev(X), 1, coef)
    ref = oracle.sink_project(V, X[0])
    assert np.abs(host(coef)[0] - ref).max() < 1e-12 * np.abs(ref).max()

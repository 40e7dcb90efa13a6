"""GPU parity of the covariant displacements and momentum overlaps (Sec. II: displacement
types D^(j); Sec. III.B: momentum projection of the meson function) against the oracle,
through the C-ABI; FP64 throughout.

Bars: displaced fields 1e-13 of the field scale (three SU(3) products per site); overlaps
and the displaced momentum-projected meson function 1e-12 relative (sums over 3 Ns^3
terms per entry)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1104_3870_amd as P

    P.lib()
    return P


def _vecs(ns, nt, n, seed):
    r = np.random.default_rng(seed)
    return r.normal(size=(nt, n, ns, ns, ns, 3)) + 1j * r.normal(size=(nt, n, ns, ns, ns, 3))


@pytest.mark.parametrize("ns,nt,n", [(4, 8, 3), (6, 4, 5)])
def test_displace_parity(P, ns, nt, n):
    import torch

    U = synth.gauge_field(ns, nt, 0.6, 20 + ns)
    v = _vecs(ns, nt, n, 1)
    L = P.Lattice(ns, nt)
    out = torch.empty(v.shape, dtype=torch.complex128, device="cuda")
    for d, s, ln in ((0, 1, 3), (0, -1, 3), (1, 1, 2), (1, -1, 1), (2, 1, 3), (2, -1, 3), (1, 1, 0), (2, 1, 7)):
        say("displace", ns, nt, n, d, s, ln)
        P.laph_displace(L.ctx, dev(U), d, s, ln, dev(v), n, out)
        ref = oracle.displace_evecs(U, v, d, s, ln)
        assert np.abs(host(out) - ref).max() <= 1e-13 * np.abs(ref).max(), (d, s, ln)
    L.close()


@pytest.mark.parametrize("ns,nt,na,nb,k", [(4, 4, 21, 18, (1, 0, 3)), (6, 2, 5, 33, (0, 0, 0)), (4, 2, 1, 1, (3, 2, 1))])
def test_mom_overlap_parity(P, ns, nt, na, nb, k):
    import torch

    a = _vecs(ns, nt, na, 2)
    b = _vecs(ns, nt, nb, 3)
    L = P.Lattice(ns, nt)
    out = torch.empty((nt, na, nb), dtype=torch.complex128, device="cuda")
    P.laph_mom_overlap(L.ctx, dev(a), na, dev(b), nb, k, out)
    ref = oracle.mom_overlap(a, b, k)
    assert np.abs(host(out) - ref).max() <= 1e-12 * np.abs(ref).max()
    L.close()


def test_overlap_apply(P):
    import torch

    nt, na, nb, n = 4, 7, 5, 3
    r = np.random.default_rng(4)
    O = r.normal(size=(nt, na, nb)) + 1j * r.normal(size=(nt, na, nb))
    b = r.normal(size=(n, nt, 4, nb)) + 1j * r.normal(size=(n, nt, 4, nb))
    L = P.Lattice(4, nt)
    out = torch.empty((n, nt, 4, na), dtype=torch.complex128, device="cuda")
    P.laph_overlap_apply(L.ctx, dev(O), na, nb, dev(b), n, out)
    ref = np.einsum("tpm,jtbm->jtbp", O, b)
    assert np.abs(host(out) - ref).max() <= 1e-13 * np.abs(ref).max()
    L.close()


@pytest.mark.parametrize("k,j1,j2", [((1, 0, 3), (0, 1), (2, -1)), ((0, 0, 0), (1, -1), (1, 1)), ((2, 2, 0), (2, 1), (0, 1))])
def test_displaced_meson_function_end_to_end(P, k, j1, j2):
    """GPU: displace the eigenvectors, overlaps, apply to the sink coefficients, meson
    function with the displacement phase; oracle: Eq. mesonfunc on the displaced full
    fields D^(j1) V_s a and D^(j2) V_s b with the momentum and displacement phases."""
    import torch

    ns, nt, nv, n1, n2 = 4, 4, 6, 3, 2
    U = synth.gauge_field(ns, nt, 0.5, 31)
    S = oracle.stout_spatial(U, 0.1, 2)
    r = np.random.default_rng(5)
    V = np.empty((nt, nv, ns, ns, ns, 3), dtype=np.complex128)
    for tt in range(nt):
        q, _ = np.linalg.qr(r.normal(size=(ns ** 3 * 3, nv)) + 1j * r.normal(size=(ns ** 3 * 3, nv)))
        V[tt] = q.T.reshape(nv, ns, ns, ns, 3)
    a = r.normal(size=(n1, nt, 4, nv)) + 1j * r.normal(size=(n1, nt, 4, nv))
    b = r.normal(size=(n2, nt, 4, nv)) + 1j * r.normal(size=(n2, nt, 4, nv))
    c = r.normal(size=(4, 4)) + 1j * r.normal(size=(4, 4))
    dv1, dv2 = [0, 0, 0], [0, 0, 0]
    dv1[j1[0]], dv2[j2[0]] = 3 * j1[1], 3 * j2[1]
    ph = np.exp(-1j * 2 * np.pi / ns * sum(kk * (p + q) / 2 for kk, p, q in zip(k, dv1, dv2)))
    L = P.Lattice(ns, nt)
    Sd, Vd = dev(S), dev(V)
    Va = torch.empty_like(Vd)
    Vb = torch.empty_like(Vd)
    P.laph_displace(L.ctx, Sd, j1[0], j1[1], 3, Vd, nv, Va)
    P.laph_displace(L.ctx, Sd, j2[0], j2[1], 3, Vd, nv, Vb)
    O = torch.empty((nt, nv, nv), dtype=torch.complex128, device="cuda")
    P.laph_mom_overlap(L.ctx, Va, nv, Vb, nv, k, O)
    bo = torch.empty((n2, nt, 4, nv), dtype=torch.complex128, device="cuda")
    P.laph_overlap_apply(L.ctx, O, nv, nv, dev(b), n2, bo)
    M = torch.empty((nt, n1, n2), dtype=torch.complex128, device="cuda")
    P.laph_meson_function(L.ctx, c * ph, dev(a), n1, bo, n2, nv, M)
    got = host(M)
    L.close()
    for i in range(n1):
        f1 = oracle.displace_spinor(S, oracle.smeared_field(V, a[i]), j1[0], j1[1])
        for j in range(n2):
            f2 = oracle.displace_spinor(S, oracle.smeared_field(V, b[j]), j2[0], j2[1])
            ref = oracle.meson_function(f1, f2, c, k=k, d1=dv1, d2=dv2)
            assert np.abs(got[:, i, j] - ref).max() <= 1e-12 * np.abs(ref).max(), (i, j)

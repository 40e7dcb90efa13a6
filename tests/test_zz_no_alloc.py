"""sink_project_noalloc (the sink projection with its partial sums in the library's fixed
device array, for callers that cannot allocate) against sink_project and the oracle
(Sec. IV: coefficients V_s^dag X), on two calls in a row, the second with a smaller
input, in a context that has no workspace at all."""
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


def _evecs(ns, nt, nv, seed):
    """Orthonormal colour vectors per slice (QR of Gaussian columns): the projection does
    not need Laplacian eigenvectors."""
    rng = np.random.default_rng(seed)
    n = ns ** 3 * 3
    V = np.empty((nt, nv, ns, ns, ns, 3), dtype=np.complex128)
    for t in range(nt):
        q, _ = np.linalg.qr(rng.normal(size=(n, nv)) + 1j * rng.normal(size=(n, nv)))
        V[t] = q.T.reshape(nv, ns, ns, ns, 3)
    return V


def test_noalloc_matches_sink_project(P):
    import torch

    ns, nt = 8, 16
    L = P.Lattice(ns, nt)
    P.laph_set_workspace(L.ctx, None)  # this entry point needs none
    for nv, nrhs, seed in ((16, 8, 1), (12, 3, 2)):  # second call: smaller input
        say("noalloc", ns, nt, nv, nrhs)
        V = _evecs(ns, nt, nv, seed)
        X = synth.random_spinor(ns, nt, 10 + seed, nrhs=nrhs)
        Vd, Xd = dev(V), dev(X)
        c0 = torch.full((nrhs, nt, 4, nv), np.nan, dtype=torch.complex128, device="cuda")
        P.sink_project_noalloc(L.ctx, Vd, nv, Xd, nrhs, c0)
        got = host(c0)
        # the workspace form on a second context
        L2 = P.Lattice(ns, nt)
        c1 = torch.empty_like(c0)
        P.sink_project(L2.ctx, Vd, nv, Xd, nrhs, c1)
        ref_ws = host(c1)
        L2.close()
        scale = np.abs(ref_ws).max()
        assert np.isfinite(got).all()
        assert np.abs(got - ref_ws).max() <= 1e-14 * scale
        for r in (0, nrhs - 1):
            ref = oracle.sink_project(V, X[r])
            assert np.abs(got[r] - ref).max() <= 1e-13 * np.abs(ref).max()
    L.close()


def test_noalloc_rejects_oversize(P):
    import torch

    ns, nt, nv = 4, 8, 8
    L = P.Lattice(ns, nt)
    X = torch.zeros((1, nt, ns, ns, ns, 4, 3), dtype=torch.complex128, device="cuda")
    V = torch.zeros((nt, nv, ns, ns, ns, 3), dtype=torch.complex128, device="cuda")
    coef = torch.zeros((1, nt, 4, nv), dtype=torch.complex128, device="cuda")
    # n_rhs * nt * 4 * nv * 16 > the fixed array: rejected on the host before any launch
    n_big = P.LAPH_SINK_NOALLOC_BYTES // (nt * 4 * nv * 16) + 1
    with pytest.raises(P.LaphError) as e:
        P.sink_project_noalloc(L.ctx, V, nv, X, n_big, coef)
    assert e.value.code == P.LAPH_EINVAL
    L.close()

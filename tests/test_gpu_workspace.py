"""The caller-owned workspace of the C-ABI: every entry point runs in exactly the bytes
laph_workspace_bytes reports (whatever ran before on the context), fails with
LAPH_ENOMEM in too little, and gives the same answer as in a large workspace; the cached
operator follows the gauge field's contents, not its address."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host, rel_err, say

pytestmark = pytest.mark.gpu

NS, NT, M0 = 4, 8, 0.1


@pytest.fixture(scope="module")
def P():
    import paper_1104_3870_amd as P

    P.lib()
    return P


def _exact(P, ctx, op, **kw):
    """Workspace of exactly the reported size (a fresh tensor; the binding's own is dropped)."""
    import torch

    need = P.laph_workspace_bytes(ctx, op, **kw)
    t = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    off = (-t.data_ptr()) % 256
    P.laph_set_workspace(ctx, t[off:off + need])
    return need


def _starve(P, ctx):
    import torch

    P.laph_set_workspace(ctx, torch.empty(256, dtype=torch.uint8, device="cuda"))


class Calls:
    """One representative call per entry point on 4^3 x 8, each with its workspace op."""

    def __init__(self, P):
        import torch

        self.P = P
        self.U = dev(synth.gauge_field(NS, NT, 0.3, 1))
        self.prm = P.laph_dirac(M0, 3.5, 1.0, -1.0)
        self.nv = 8
        self.evecs = torch.empty((NT, self.nv, NS, NS, NS, 3), dtype=torch.complex128, device="cuda")
        V = oracle.laph_eigpairs(oracle.stout_spatial(host(self.U), 0.1, 2), self.nv)[1]
        self.evecs.copy_(torch.from_numpy(np.ascontiguousarray(V)))
        self.psi = dev(synth.random_spinor(NS, NT, 3, nrhs=4))
        self.out = torch.empty_like(self.psi)
        self.col = dev(synth.random_colour_field(NS, NT, 2))
        self.colo = torch.empty_like(self.col)
        self.Uo = torch.empty_like(self.U)
        self.coef = torch.empty((4, NT, 4, self.nv), dtype=torch.complex128, device="cuda")
        self.rho = torch.empty((NT, 4, self.nv), dtype=torch.complex128, device="cuda")
        self.dil = P.laph_parse_dilution("TF,SF,LF", NT, self.nv)
        self.sv = P.solver_params(precision="f16", block_rhs=4, solver=P.LAPH_SOLVER_CGNR)
        self.sv64 = P.solver_params(precision="f64", block_rhs=2, solver=P.LAPH_SOLVER_BICGSTAB)
        self.hop = P.laph_hop(P.LAPH_PREC_F16, P.LAPH_HOP_INV, 1, 0, 1, 0, 0, 1.0, -1.0)

    def ops(self):
        P, L = self.P, self.P.lib()
        c = ctypes.byref
        evals = np.zeros((NT, self.nv))
        lz = P.laph_lanczos(48, 8, 15.0, 2.5, 1e-10, 200, 7)
        st = (P.laph_solve_stats * 4)()
        nrm = np.zeros(4)
        d = P._dptr
        return [
            ("stout", P.LAPH_WS_STOUT, {}, lambda ctx: L.laph_stout_smear(ctx, d(self.U), c(P.laph_stout(0.1, 2)),
                                                                          d(self.Uo))),
            ("laplacian", P.LAPH_WS_LAPLACIAN, {}, lambda ctx: L.laph_laplacian_apply(ctx, d(self.U), d(self.col),
                                                                                      d(self.colo))),
            ("chebyshev", P.LAPH_WS_CHEBYSHEV, {},
             lambda ctx: L.laph_chebyshev_apply(ctx, d(self.U), 15.0, 0.5, 8, d(self.col), d(self.colo))),
            ("eigvecs", P.LAPH_WS_EIGVECS, dict(nv=self.nv, krylov_dim=48),
             lambda ctx: L.laph_eigvecs(ctx, d(self.U), c(P.laph_stout(0.1, 2)), c(lz), self.nv,
                                        evals.ctypes.data_as(ctypes.c_void_p), d(self.evecs),
                                        c(P.laph_eig_stats()))),
            ("source", P.LAPH_WS_SOURCE, dict(nv=self.nv),
             lambda ctx: L.make_diluted_source(ctx, d(self.evecs), self.nv, 0, 1, c(self.dil), 3, 4, d(self.out),
                                               P.LAPH_DTYPE_C128)),
            ("apply", P.LAPH_WS_DIRAC_APPLY, dict(n=4),
             lambda ctx: L.laph_dirac_apply(ctx, d(self.U), c(self.prm), P.LAPH_OP_OMEGA, d(self.psi), d(self.out),
                                            4)),
            ("hop", P.LAPH_WS_HOP_APPLY, dict(n=4, hop=self.hop),
             lambda ctx: L.laph_hop_apply(ctx, d(self.U), c(self.prm), c(self.hop), d(self.psi), None, d(self.out),
                                          None, None, nrm.ctypes.data_as(ctypes.c_void_p), 4)),
            ("solve_f16", P.LAPH_WS_SOLVE, dict(n=3, solver=self.sv),
             lambda ctx: L.dirac_solve(ctx, d(self.U), c(self.prm), d(self.psi), d(self.out), 3, c(self.sv), st)),
            ("solve_f64", P.LAPH_WS_SOLVE, dict(n=4, solver=self.sv64),
             lambda ctx: L.dirac_solve(ctx, d(self.U), c(self.prm), d(self.psi), d(self.out), 4, c(self.sv64), st)),
            ("sink", P.LAPH_WS_SINK, dict(nv=self.nv, n=4),
             lambda ctx: L.sink_project(ctx, d(self.evecs), self.nv, d(self.psi), 4, d(self.coef))),
            ("autotune", P.LAPH_WS_AUTOTUNE, dict(precision=P.LAPH_PREC_BF16),
             lambda ctx: L.laph_autotune(ctx, d(self.U), c(self.prm), P.LAPH_PREC_BF16, c(P.laph_tune_report()))),
        ]


def test_every_entry_point_runs_in_the_reported_bytes(P):
    import torch

    calls = Calls(P)
    L = P.Lattice(NS, NT)
    ops = calls.ops()
    # each op alone, then each op after every other (a cached operator of another kind,
    # scratch of another size): exactly the reported bytes always suffice
    for name, op, kw, fn in ops:
        say("ws", name)
        _exact(P, L.ctx, op, **kw)
        assert fn(L.ctx) == P.LAPH_OK, (name, P.lib().laph_last_error(L.ctx))
        torch.cuda.synchronize()
    for name0, op0, kw0, fn0 in ops:
        for name, op, kw, fn in ops:
            if name == name0:
                continue
            # op0 first (when it fits) leaves its cached operator and scratch history in
            # the workspace sized exactly for op
            need = _exact(P, L.ctx, op, **kw)
            if P.laph_workspace_bytes(L.ctx, op0, **kw0) <= need:
                assert fn0(L.ctx) == P.LAPH_OK, (name0, name)
            assert fn(L.ctx) == P.LAPH_OK, (name0, name, P.lib().laph_last_error(L.ctx))
    torch.cuda.synchronize()
    L.close()


def test_too_small_workspace_is_enomem(P):
    calls = Calls(P)
    L = P.Lattice(NS, NT)
    for name, op, kw, fn in calls.ops():
        _starve(P, L.ctx)
        assert fn(L.ctx) == P.LAPH_ENOMEM, name
    P.laph_set_workspace(L.ctx, None)
    name, op, kw, fn = calls.ops()[5]
    assert fn(L.ctx) == P.LAPH_ENOMEM  # no workspace at all
    L.close()


def test_exact_workspace_same_answer(P):
    """A solve in exactly its bytes returns the same x, bit for bit, as in a large one."""
    import torch

    calls = Calls(P)
    eta = calls.psi[:3].contiguous()
    xs = []
    for exact in (False, True):
        L = P.Lattice(NS, NT)
        x = torch.empty_like(eta)
        if exact:
            _exact(P, L.ctx, P.LAPH_WS_SOLVE, n=3, solver=calls.sv)
            st = (P.laph_solve_stats * 3)()
            rc = P.lib().dirac_solve(L.ctx, P._dptr(calls.U), ctypes.byref(calls.prm), P._dptr(eta), P._dptr(x), 3,
                                     ctypes.byref(calls.sv), st)
            assert rc == P.LAPH_OK
        else:
            P.laph_set_workspace(L.ctx, torch.empty(256 << 20, dtype=torch.uint8, device="cuda"))
            P.dirac_solve(L.ctx, calls.U, calls.prm, eta, x, 3, calls.sv)
        xs.append(host(x))
        L.close()
    assert np.array_equal(xs[0], xs[1])


@pytest.mark.parametrize("prec", ["f64", "f16"])
def test_cache_follows_field_contents(P, prec):
    """A different field written into the same tensor (same address) is noticed: the
    solve and the operator are those of the new field (the oracle judges both)."""
    import torch

    U1 = synth.gauge_field(NS, NT, 0.3, 21)
    U2 = synth.gauge_field(NS, NT, 0.5, 22)
    eta = synth.random_spinor(NS, NT, 4, nrhs=2)
    L = P.Lattice(NS, NT)
    Ud = dev(U1)
    ptr = Ud.data_ptr()
    prm = P.laph_dirac(M0, 3.5, 1.0, -1.0)
    x = torch.empty(eta.shape, dtype=torch.complex128, device="cuda")
    out = torch.empty_like(x)
    sv = P.solver_params(precision=prec, block_rhs=2, solver=P.LAPH_SOLVER_CGNR)
    for U in (U1, U2, U1):
        Ud.copy_(torch.from_numpy(U))
        assert Ud.data_ptr() == ptr
        D = oracle.Dirac(U, M0, 3.5, 1.0, -1.0)
        P.laph_dirac_apply(L.ctx, Ud, prm, P.LAPH_OP_OMEGA, dev(eta), out, 2)
        assert rel_err(host(out)[1], D.omega(eta[1])) < 1e-13
        st = P.dirac_solve(L.ctx, Ud, prm, dev(eta), x, 2, sv)
        for r in range(2):
            assert D.true_residual(eta[r], host(x)[r]) <= 1e-10, (prec, r)
            assert st[r].status == 0
    L.close()

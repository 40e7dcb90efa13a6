"""GPU dirac_solve against the oracle (Sec. IV: Omega x = eta by even-odd BiCGStab,
mixed precision, CG on the normal equations as fallback).

Every answer is judged by the oracle's own Omega: the true relative residual
|eta - Omega x| / |eta| must be <= 1e-10 (the bar of the workload); and x must agree
with the oracle's solution (solved to 1e-12) within cond(Omega) * 1e-10 <= 1e-8."""
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


@pytest.fixture(scope="module")
def setup():
    cfg = synth.CONFIGS["ns4_nt8"]
    U = synth.gauge_field(cfg.ns, cfg.nt, cfg.eps, cfg.seed)
    D = oracle.Dirac(U, cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    etas = synth.random_spinor(cfg.ns, cfg.nt, 21, nrhs=5)
    xs = [D.solve(e, tol=1e-12)[0] for e in etas]
    return cfg, U, D, etas, xs


def _solve(P, cfg, U, etas, **kw):
    import torch

    L = P.Lattice(cfg.ns, cfg.nt)
    prm = P.laph_dirac(cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    x = torch.empty(etas.shape, dtype=torch.complex128, device="cuda")
    sv = P.solver_params(**kw)
    st = P.dirac_solve(L.ctx, dev(U), prm, dev(etas), x, etas.shape[0], sv)
    return host(x), st


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_single_rhs(P, setup, prec):
    cfg, U, D, etas, xs = setup
    say("solve single", prec)
    x, st = _solve(P, cfg, U, etas[:2], precision=prec, block_rhs=1)
    for r in range(2):
        tr = D.true_residual(etas[r], x[r])
        say("  rhs", r, "iters", st[r].iters, "lib resid", st[r].true_resid, "oracle resid", tr)
        assert st[r].status == 0
        assert tr <= 1e-10
        assert abs(tr - st[r].true_resid) <= 1e-12
        assert rel_err(x[r], xs[r]) <= 1e-8


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_cgnr_mixed_multi_rhs(P, setup, prec):
    """Mixed-precision CG on the normal equations with FP64 reliable updates, 5 RHS in a
    padded block of 8."""
    cfg, U, D, etas, xs = setup
    x, st = _solve(P, cfg, U, etas, precision=prec, block_rhs=8, solver=P.LAPH_SOLVER_CGNR)
    for r in range(5):
        assert D.true_residual(etas[r], x[r]) <= 1e-10
        assert rel_err(x[r], xs[r]) <= 1e-8


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_cgnr_direction_buffers(P, setup, prec):
    """The fused CG loop keeps up to dir_buffers directions until their steps are added to
    the solution increment.  Every ring size must give the same iterate up to rounding: a
    step lost or taken twice would be repaired only by the next reliable update, at the
    cost of extra iterations, so the iteration counts of all ring sizes must agree within
    a few and every answer must meet the bar."""
    cfg, U, D, etas, xs = setup
    its = {}
    for k in (1, 2, 3, 5, 8):
        x, st = _solve(P, cfg, U, etas, precision=prec, block_rhs=8, solver=P.LAPH_SOLVER_CGNR, dir_buffers=k)
        its[k] = [q.iters for q in st]
        say("  dir_buffers", k, "iters", its[k])
        for r in range(5):
            assert st[r].status == 0 and st[r].fallback_used == 0
            assert D.true_residual(etas[r], x[r]) <= 1e-10
            assert rel_err(x[r], xs[r]) <= 1e-8
    for r in range(5):
        col = [its[k][r] for k in its]
        assert max(col) - min(col) <= max(2, min(col) // 50), its
    with pytest.raises(P.LaphError):
        _solve(P, cfg, U, etas[:1], precision=prec, solver=P.LAPH_SOLVER_CGNR, dir_buffers=9)


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_bicgstab_step_ring(P, setup, prec):
    """The fused low-precision BiCGStab owes its steps alpha p + omega s to the solution
    increment in a ring of dir_buffers (p, s) pairs and takes them together.  Every ring
    size must give the same iterate up to rounding (a step lost or taken twice would be
    repaired only by the next reliable update, at the cost of extra iterations): the
    iteration counts must agree within a few and every answer must meet the bar.  FP16
    records make the update decisions, and with them the count, vary with the rounding
    order of the increment by a few more iterations than FP32."""
    cfg, U, D, etas, xs = setup
    its = {}
    for k in (1, 2, 3, 5, 8):
        x, st = _solve(P, cfg, U, etas, precision=prec, block_rhs=8, dir_buffers=k)
        its[k] = [q.iters for q in st]
        say("  bicgstab dir_buffers", k, "iters", its[k])
        for r in range(5):
            assert st[r].status == 0 and st[r].fallback_used == 0
            assert D.true_residual(etas[r], x[r]) <= 1e-10
            assert rel_err(x[r], xs[r]) <= 1e-8
    slack = 3 if prec == "f32" else 5
    for r in range(5):
        col = [its[k][r] for k in its]
        assert max(col) - min(col) <= max(slack, min(col) // 20), its


def test_bicgstab_graph_replay_matches_eager(P, setup):
    """The fused BiCGStab iteration replayed from HIP graphs (one per ring position) gives
    bit-identical solutions and iteration counts to eager launches."""
    cfg, U, D, etas, xs = setup
    kw = dict(precision="f16", block_rhs=4, solver=P.LAPH_SOLVER_BICGSTAB)
    x0, s0 = _solve(P, cfg, U, etas[:4], use_graph=0, **kw)
    for rep in range(2):
        x1, s1 = _solve(P, cfg, U, etas[:4], use_graph=1, **kw)
        say("  bicgstab iters eager", [q.iters for q in s0], "graph", [q.iters for q in s1])
        assert [q.iters for q in s0] == [q.iters for q in s1]
        assert np.array_equal(x0, x1)
    for r in range(4):
        assert s1[r].fallback_used == 0 and D.true_residual(etas[r], x1[r]) <= 1e-10


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_multi_rhs_masked(P, setup, prec):
    """5 right-hand sides in blocks of 8 (padded, uneven convergence): each equals the
    oracle solution within the residual bound."""
    cfg, U, D, etas, xs = setup
    say("solve block", prec)
    x, st = _solve(P, cfg, U, etas, precision=prec, block_rhs=8)
    for r in range(5):
        tr = D.true_residual(etas[r], x[r])
        assert tr <= 1e-10
        assert rel_err(x[r], xs[r]) <= 1e-8


def test_cgnr(P, setup):
    cfg, U, D, etas, xs = setup
    x, st = _solve(P, cfg, U, etas[:1], solver=P.LAPH_SOLVER_CGNR)
    assert st[0].fallback_used == 0
    assert D.true_residual(etas[0], x[0]) <= 1e-10
    assert rel_err(x[0], xs[0]) <= 1e-8


@pytest.mark.parametrize("prec,block", [("f64", 1), ("f16", 4)])
def test_forced_fallback(P, setup, prec, block):
    """BiCGStab capped at 4 iterations per attempt cannot converge; the CGNR fallback of
    Sec. IV must still reach the bar (forced from the host), after the plain FP64 form and
    after the fused low-precision form (whose owed steps and increment must reach x before
    the hand-off)."""
    cfg, U, D, etas, xs = setup
    x, st = _solve(P, cfg, U, etas[:block], maxiter=4, precision=prec, block_rhs=block)
    for r in range(block):
        assert st[r].fallback_used == 1
        assert D.true_residual(etas[r], x[r]) <= 1e-10


def test_zero_source(P, setup):
    cfg, U, D, etas, xs = setup
    z = np.zeros_like(etas[:2])
    z[1] = etas[1]
    x, st = _solve(P, cfg, U, z, block_rhs=2)
    assert np.abs(x[0]).max() == 0
    assert D.true_residual(etas[1], x[1]) <= 1e-10


@pytest.mark.parametrize("prec,solver", [("f16", "cgnr"), ("f16", "bicgstab"), ("bf16", "cgnr"),
                                         ("bf16", "bicgstab"), ("f32", "cgnr")])
def test_tiny_tails_low_precision(P, prec, solver):
    """Regression: a source on one time slice of a long lattice at a heavy mass has a
    solution that falls below the FP32 normal range far from the source; the FP16 site
    scales must stay finite there (they once became denormal and 1/scale infinite)."""
    import torch

    ns, nt, m0 = 4, 128, 1.5
    U = synth.gauge_field(ns, nt, 0.3, 2)
    D = oracle.Dirac(U, m0, 3.5, 1.0, -1.0)
    eta = np.zeros((1, nt, ns, ns, ns, 4, 3), dtype=np.complex128)
    eta[0, 0] = synth.random_spinor(ns, 1, 5)[0]
    L = P.Lattice(ns, nt)
    x = torch.empty(eta.shape, dtype=torch.complex128, device="cuda")
    kind = P.LAPH_SOLVER_CGNR if solver == "cgnr" else P.LAPH_SOLVER_BICGSTAB
    st = P.dirac_solve(L.ctx, dev(U), P.laph_dirac(m0, 3.5, 1.0, -1.0), dev(eta), x, 1,
                       P.solver_params(precision=prec, solver=kind))
    xs = host(x)
    assert np.isfinite(xs).all()
    assert st[0].fallback_used == 0
    assert D.true_residual(eta[0], xs[0]) <= 1e-10
    # the exact solution falls below the FP32 normal range far from the source
    x64 = D.solve(eta[0], tol=1e-13)[0]
    assert np.abs(x64[nt // 2]).max() < 1e-30


@pytest.mark.parametrize("prec", ["f16", "f64"])
def test_autotune_report(P, setup, prec):
    cfg, U, D, etas, xs = setup
    say("autotune", prec)
    L = P.Lattice(cfg.ns, cfg.nt)
    prm = P.laph_dirac(cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    rep = P.laph_autotune(L.ctx, dev(U), prm, prec)
    say("  best R", rep["best_block_rhs"], "S", rep["best_sites_per_block"], "entries", len(rep["entries"]))
    Rs = sorted({e[0] for e in rep["entries"]})
    if prec == "f64":
        assert Rs == [1, 2, 4, 8, 16, 32] and all(e[1] == 0 for e in rep["entries"])
    else:
        assert Rs == [4, 8, 16, 32] and len(rep["entries"]) == 12
        assert all(e[0] * e[1] in (64, 128, 256) for e in rep["entries"])
        best = [e for e in rep["entries"] if e[0] == rep["best_block_rhs"] and e[1] == rep["best_sites_per_block"]]
        assert len(best) == 1
    assert all(e[2] > 0 for e in rep["entries"])
    assert rep["best_block_rhs"] in Rs
    # the tuned block size is what block_rhs = 0 uses; the answer is judged as always
    x, st = _solve(P, cfg, U, etas, precision=prec, block_rhs=0, solver=P.LAPH_SOLVER_CGNR)
    for r in range(etas.shape[0]):
        assert st[r].status == 0 and D.true_residual(etas[r], x[r]) <= 1e-10


@pytest.mark.parametrize("solver", ["bicgstab", "cgnr"])
def test_untuned_block_rhs_zero(P, setup, solver):
    """block_rhs = 0 on a fresh context: the solve runs the autotuner itself, inside the
    workspace sized before it (the fused epilogues' partial sums sized for the smallest tile
    the tuner may pick)."""
    cfg, U, D, etas, xs = setup
    kind = P.LAPH_SOLVER_CGNR if solver == "cgnr" else P.LAPH_SOLVER_BICGSTAB
    x, st = _solve(P, cfg, U, etas, precision="f16", block_rhs=0, solver=kind, use_graph=1)
    for r in range(etas.shape[0]):
        assert st[r].status == 0 and st[r].fallback_used == 0
        assert D.true_residual(etas[r], x[r]) <= 1e-10
        assert rel_err(x[r], xs[r]) <= 1e-8


@pytest.mark.parametrize("prec", ["f16", "f64"])
def test_graph_replay_matches_eager(P, setup, prec):
    cfg, U, D, etas, xs = setup
    say("graph replay", prec)
    kw = dict(precision=prec, block_rhs=4, solver=P.LAPH_SOLVER_CGNR)
    x0, s0 = _solve(P, cfg, U, etas[:4], use_graph=0, **kw)
    for rep in range(2):  # two solves, each replaying its captured iteration many times
        x1, s1 = _solve(P, cfg, U, etas[:4], use_graph=1, **kw)
        say("  iters eager", [q.iters for q in s0], "graph", [q.iters for q in s1])
        assert [q.iters for q in s0] == [q.iters for q in s1]
        assert np.array_equal(x0, x1)
    for r in range(4):
        assert D.true_residual(etas[r], x1[r]) <= 1e-10


@pytest.fixture(scope="module")
def mid():
    """16^3 x 32 field of the mid-size workload at its mass (a few hundred CG iterations)
    and four Gaussian sources."""
    cfg = synth.CONFIGS["ns16_nt32"]
    U = synth.gauge_field(cfg.ns, cfg.nt, cfg.eps, cfg.seed)
    D = oracle.Dirac(U, cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    etas = synth.random_spinor(cfg.ns, cfg.nt, 31, nrhs=4)
    return cfg, U, D, etas


def test_mixed_iterations_bound(P, mid):
    """Low-precision inner vectors cost at most a few percent more CG iterations than the
    FP64 solver on the same block (Sec. IV: mixed precision with reliable updates must not
    change the method).  A sign or index error in a low-precision hop would be repaired by
    the FP64 reliable updates and show only here, as extra iterations.  Bars on the mean
    over the block: FP32 and FP16 within 5% of FP64; BF16 (8-bit mantissa, so the CG
    recurrence drifts from the true residual an order of magnitude faster and every
    reliable update restarts the search direction) within 20%."""
    cfg, U, D, etas = mid
    mean = {}
    for prec in ("f64", "f32", "f16", "bf16"):
        say("iterations", prec)
        x, st = _solve(P, cfg, U, etas, precision=prec, block_rhs=4, solver=P.LAPH_SOLVER_CGNR)
        for r in range(etas.shape[0]):
            assert st[r].status == 0 and st[r].fallback_used == 0
            assert D.true_residual(etas[r], x[r]) <= 1e-10
        mean[prec] = float(np.mean([q.iters for q in st]))
        say("  iters", [q.iters for q in st], "mean", mean[prec])
    assert mean["f64"] > 100, mean
    assert mean["f32"] <= 1.05 * mean["f64"], mean
    assert mean["f16"] <= 1.05 * mean["f64"], mean
    assert mean["bf16"] <= 1.20 * mean["f64"], mean


def test_bicgstab_mixed_iterations_bound(P, mid):
    """The same for BiCGStab (Sec. IV), the paper's solver: the fused low-precision
    iteration (inner products from the hopping epilogues, owed steps, FP64 reliable
    updates) on the block of four against FP64 BiCGStab, without the fallback.  FP32
    within 5%; FP16 within 20%: BiCGStab's two-sided recurrence (the shadow residual)
    loses the rounding of 11-bit records faster than CG's, which FP16 CG absorbs at +1%."""
    cfg, U, D, etas = mid
    mean = {}
    for prec in ("f64", "f32", "f16"):
        say("bicgstab iterations", prec)
        x, st = _solve(P, cfg, U, etas, precision=prec, block_rhs=4, solver=P.LAPH_SOLVER_BICGSTAB)
        for r in range(etas.shape[0]):
            assert st[r].status == 0 and st[r].fallback_used == 0
            assert D.true_residual(etas[r], x[r]) <= 1e-10
        mean[prec] = float(np.mean([q.iters for q in st]))
        say("  iters", [q.iters for q in st], "mean", mean[prec])
    assert mean["f64"] > 50, mean
    assert mean["f32"] <= 1.05 * mean["f64"], mean
    assert mean["f16"] <= 1.20 * mean["f64"], mean

"""Pins of the oracle's BiCGStab and even-odd Schur system (Sec. IV: the paper's solver
on the even-odd preconditioned system).

* BiCGStab on a small random well-conditioned non-Hermitian matrix equals LAPACK's solve.
* Finite termination: without breakdown BiCG's residual polynomial of degree n annihilates
  the first residual of an n x n system, and BiCGStab's residual carries that factor, so n
  iterations solve it to rounding (a wrong alpha, beta or direction update does not).
* The stabilising step of every iteration is a one-dimensional minimal-residual step: the
  new residual is the least-squares residual of s over span{A s} (LAPACK's least squares;
  a conjugated omega still converges, but fails this).
* CG on the normal equations (the oracle's fallback solver and the CPU baseline's
  iteration count): its k-th iterate minimises |eta - Omega x| over the Krylov space
  K_k(Omega^dag Omega, Omega^dag eta), built here by Arnoldi with two Gram-Schmidt passes
  and solved by LAPACK's least squares; a slower but convergent CG fails it.
* The Schur identity: for the solution x of Omega x = eta (the oracle's CG on the normal
  equations to a true residual of 1e-13, itself pinned to dense LU), the odd part solves
  Mhat x_o = bhat and the even reconstruction returns x (a dropped hopping term, a wrong
  parity or gamma_4 fails it).
* BiCGStab on the full and on the even-odd system of the 4^3 x 8 field reaches that
  solution."""
import numpy as np

import oracle
import synth


def test_bicgstab_small_matrix():
    rng = np.random.default_rng(4)
    n = 60
    A = np.eye(n) * 4 + (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) / np.sqrt(n)
    b = rng.normal(size=n) + 1j * rng.normal(size=n)
    x, k, hist = oracle.bicgstab(lambda v: A @ v, b, tol=1e-13, maxiter=500)
    assert k > 0 and hist[-1] <= 1e-13
    ref = np.linalg.solve(A, b)
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)


def _random_system(n, seed):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 2 + (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) / np.sqrt(n)
    b = rng.normal(size=n) + 1j * rng.normal(size=n)
    return A, b


def test_bicgstab_finite_termination():
    for n in range(2, 9):
        for seed in range(20):
            A, b = _random_system(n, 100 * n + seed)
            x, k, hist = oracle.bicgstab(lambda v: A @ v, b, tol=0.0, maxiter=n)
            assert abs(k) <= n
            res = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
            assert res <= 1e-11, (n, seed, k, res)


def test_bicgstab_stabilising_step_minimises_residual():
    A, b = _random_system(60, 4)
    trace = []
    x, k, hist = oracle.bicgstab(lambda v: A @ v, b, tol=1e-12, maxiter=500, trace=trace)
    assert k > 0 and len(trace) == k
    for s, t, r in trace:
        np.testing.assert_allclose(t, A @ s, rtol=0, atol=1e-13 * np.linalg.norm(A @ s))
        w = np.linalg.lstsq(t[:, None], s, rcond=None)[0][0]
        assert np.linalg.norm(r - (s - w * t)) <= 1e-12 * np.linalg.norm(s)


def _setup():
    cfg = synth.CONFIGS["ns4_nt8"]
    U = synth.gauge_field(cfg.ns, cfg.nt, cfg.eps, cfg.seed)
    D = oracle.Dirac(U, cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    eta = synth.random_spinor(cfg.ns, cfg.nt, 41)
    x, it, tr = D.solve(eta, tol=1e-13)
    assert it > 0 and tr <= 1e-13
    return D, eta, x


def test_schur_identity():
    D, eta, x = _setup()
    eo = oracle.EvenOdd(D)
    xo = x * eo.odd
    b = eo.bhat(eta)
    assert np.abs(eo.mhat(xo) - b).max() <= 1e-11 * np.abs(b).max()
    assert np.abs(eo.full(xo, eta) - x).max() <= 1e-11 * np.abs(x).max()
    # every field the system produces lives on odd sites
    assert np.abs(b * eo.even).max() == 0 and np.abs(eo.mhat(xo) * eo.even).max() == 0


def test_bicgstab_full_and_even_odd():
    D, eta, x = _setup()
    for eo in (False, True):
        y, k, hist, tr = oracle.bicgstab_solve(D, eta, tol=1e-12, maxiter=2000, even_odd=eo)
        assert k > 0 and tr <= 1e-10, (eo, k, tr)
        assert np.linalg.norm(y - x) <= 1e-9 * np.linalg.norm(x)


def test_cgnr_iterates_minimise_the_residual():
    cfg = synth.CONFIGS["ns4_nt8"]
    U = synth.gauge_field(cfg.ns, cfg.nt, cfg.eps, cfg.seed)
    D = oracle.Dirac(U, cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    eta = synth.random_spinor(cfg.ns, cfg.nt, 41)
    sh, e = D.shape, eta.reshape(-1)
    w = D.omega(eta, dagger=True).reshape(-1)
    Q = [w / np.linalg.norm(w)]
    for k in range(1, 11):
        OQ = np.stack([D.omega(q.reshape(sh)).reshape(-1) for q in Q], axis=1)
        c = np.linalg.lstsq(OQ, e, rcond=None)[0]
        best = np.linalg.norm(e - OQ @ c) / np.linalg.norm(e)
        xk = np.stack(Q, axis=1) @ c
        x, it, tr = D.solve(eta, tol=0.0, maxiter=k)
        assert it == -k
        assert abs(tr - best) <= 1e-10 * best, (k, tr, best)
        assert np.linalg.norm(x.reshape(-1) - xk) <= 1e-8 * np.linalg.norm(xk), k
        z = D.omega(D.omega(Q[-1].reshape(sh)), dagger=True).reshape(-1)
        for _ in range(2):
            for q in Q:
                z = z - np.vdot(q, z) * q
        Q.append(z / np.linalg.norm(z))

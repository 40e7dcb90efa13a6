"""Pins of the oracle's baryon function and baryon correlator (Sec. III.A, Eqs. baryonfunc
and baryoncorr).

Strongest pin: with full time x spin x LapH dilution each quark line's estimate is exact
for any noise (Sec. II), so the baryon correlator assembled from baryon functions with the
six noise orderings of Eq. baryoncorr equals the six-term Wick contraction of three dense
smeared quark lines Q = S Omega^-1 S written out over sites, colours (epsilon tensors) and
spins (4^3 x 8 field; three LapH vectors per slice keep the 12^3 dilution triples of one
source time few).  A wrong epsilon, sign or noise ordering fails it."""
import itertools

import numpy as np
import pytest

import oracle
import synth
import wick
from wick import EPS


def _fields(seed, n=3, ns=4, nt=2):
    return [synth.random_spinor(ns, nt, seed + i) for i in range(n)]


def _tensor(seed, sparse=False):
    r = np.random.default_rng(seed)
    c = r.normal(size=(4, 4, 4)) + 1j * r.normal(size=(4, 4, 4))
    if sparse:
        mask = np.zeros((4, 4, 4), dtype=bool)
        for idx in r.choice(64, size=2, replace=False):
            mask.flat[idx] = True
        c = np.where(mask, c, 0)
    return c


def test_epsilon_table():
    assert EPS[0, 1, 2] == 1 and EPS[1, 0, 2] == -1 and EPS[2, 0, 1] == 1 and EPS[1, 2, 0] == 1


def test_antisymmetry_under_quark_exchange():
    """Swapping two quarks together with their spin indices flips the sign (epsilon)."""
    f1, f2, f3 = _fields(1)
    c = _tensor(2)
    k = (1, 0, 2)
    b = oracle.baryon_function(f1, f2, f3, c, k)
    assert np.abs(oracle.baryon_function(f2, f1, f3, c.transpose(1, 0, 2), k) + b).max() <= 1e-12 * np.abs(b).max()
    assert np.abs(oracle.baryon_function(f3, f2, f1, c.transpose(2, 1, 0), k) + b).max() <= 1e-12 * np.abs(b).max()
    # equal fields in an antisymmetric slot with a symmetric spin tensor vanish
    cs = c + c.transpose(1, 0, 2)
    assert np.abs(oracle.baryon_function(f1, f1, f3, cs, k)).max() <= 1e-12 * np.abs(b).max()


def test_gauge_invariance_and_momentum():
    """B is unchanged when all three fields are rotated by the same site-local SU(3)
    matrices (epsilon_abc G_aa' G_bb' G_cc' = det G epsilon_a'b'c'); a plane wave
    e^{iq.x} on one field shifts the momentum k -> k - q."""
    ns, nt = 4, 2
    f1, f2, f3 = _fields(3)
    c = _tensor(4)
    G = synth.gauge_transform_field(ns, nt, 5)
    rot = [np.einsum("tzyxab,tzyxsb->tzyxsa", G, f) for f in (f1, f2, f3)]
    b = oracle.baryon_function(f1, f2, f3, c, (0, 1, 1))
    assert np.abs(oracle.baryon_function(*rot, c, (0, 1, 1)) - b).max() <= 1e-12 * np.abs(b).max()
    t, z, y, x = np.meshgrid(*(np.arange(n) for n in (nt, ns, ns, ns)), indexing="ij")
    q = (1, 3, 2)
    wave = np.exp(2j * np.pi * (q[0] * x + q[1] * y + q[2] * z) / ns)[..., None, None]
    lhs = oracle.baryon_function(f1, f2, wave * f3, c, (2, 1, 0))
    rhs = oracle.baryon_function(f1, f2, f3, c, tuple(a - b for a, b in zip((2, 1, 0), q)))
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


@pytest.fixture(scope="module")
def exact3():
    cfg = synth.CONFIGS["ns4_nt8"]
    nv = 3
    U = synth.gauge_field(cfg.ns, cfg.nt, cfg.eps, cfg.seed)
    S = oracle.stout_spatial(U, cfg.stout_rho, cfg.stout_steps)
    ev, V = oracle.laph_eigpairs(S, nv)
    D = oracle.Dirac(U, cfg.m0, cfg.xi, cfg.csw, cfg.bc_t)
    B = oracle.laph_basis(V)
    X = oracle.dense_solve(D, B)
    Q = B @ (B.conj().T @ X) @ B.conj().T
    return cfg, nv, V, X, Q


def test_baryon_correlator_full_dilution_is_exact(exact3):
    cfg, nv, V, X, Q = exact3
    nt, ns = cfg.nt, cfg.ns
    t0, k = 3, (1, 0, 0)
    c, cp = _tensor(6, sparse=True), _tensor(7, sparse=True)
    sch = oracle.parse_dilution("TF,SF,LF", nt, nv)
    bs = [b for b in range(oracle.dilution_count(sch, nt, nv)) if b // (4 * nv) == t0]
    nb = len(bs)
    shape = (nt, ns, ns, ns, 4, 3)
    rhos = [oracle.z4_noise(s, 5, nt, nv) for s in (1, 2, 3)]
    snk_f = [[oracle.quark_sink(V, (X[:, b] * r.ravel()[b]).reshape(shape)) for b in bs] for r in rhos]
    src_f = [[oracle.quark_source(V, r, sch, b) for b in bs] for r in rhos]
    snk = np.zeros((nt, nb, nb, nb), dtype=np.complex128)
    for i, j, l in itertools.product(range(nb), repeat=3):
        snk[:, i, j, l] = oracle.baryon_function(snk_f[0][i], snk_f[1][j], snk_f[2][l], c, k)
    src = []
    for order, sign in oracle.BARYON_PERMUTATIONS:
        S = np.zeros((nt, nb, nb, nb), dtype=np.complex128)
        for i, j, l in itertools.product(range(nb), repeat=3):
            S[:, i, j, l] = oracle.baryon_function(src_f[order[0]][i], src_f[order[1]][j], src_f[order[2]][l], cp, k)
        src.append(S)
    est = oracle.baryon_correlator(snk, src, t0)
    # brute force: six Wick terms of three dense quark lines Q(x tF, x0 t0)
    ref = wick.baryon_wick(Q, ns, nt, t0, c, cp, k)
    assert np.abs(est - ref).max() <= 1e-10 * np.abs(ref).max()

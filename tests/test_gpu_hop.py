"""Element-wise parity of the solver's even-odd hopping kernels (laph_hop_apply) against
the oracle's Wilson-clover operator, in every storage precision and fused epilogue.

The reference is built here from the oracle alone: D_{p,1-p} in is the oracle's K applied
to `in` restricted to the sites of parity 1-p, read on the sites of parity p (the clover
term is site-local, so K and its hopping part agree there; Sec. II splits K = A + H), A^-1
is the inverse of the oracle's per-site clover matrix and gamma_5 is the oracle's.

Inputs are chosen exactly representable in the storage precision (FP16: multiples of
2^-10 with the largest component of every site and field equal to 1, so that the stored
scale is 1; BF16: multiples of 2^-7; FP32: FP32 numbers), so that in the caller's gauge
the only differences from the exact FP64 result are the FP32 arithmetic with FP32 links
and clover inverse, and the rounding of the stored outputs.  Bounds (stated per element
or per site and field, u the unit roundoff of the storage format):
  FP16 out:  |d| <= 2^-12 max|ref_site| + e_arith     (one FP32 scale per site and field)
  BF16 out:  |d| <= 2^-8 |ref| + e_arith              (per component)
  FP32 out:  |d| <= 2^-24 |ref| + e_arith
with e_arith = 2e-5 (|a| + |c|) for inputs of magnitude <= 1 (FP32 sums of ~100 terms
with FP32 operands).  In temporal gauge the rotated inputs are rounded too, which adds
8 u (|c| + |a|) max|input| per element.  Norms of the fused epilogues are checked against
the sum of squares of the returned (stored) outputs to 1e-6 relative and against the
reference within the propagated rounding; the inner products <y, out> of the BiCGStab
epilogue (INV_DOT) against those of the stored outputs to 4e-6 of sum |y| |out|.  FP64
hops: 1e-13 relative.
"""
import zlib

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host, say

pytestmark = pytest.mark.gpu

XI, CSW, BC = 3.5, 1.0, -1.0
U_OUT = {"f16": 2.0 ** -12, "bf16": 2.0 ** -8, "f32": 2.0 ** -24}
U_IN = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8, "f32": 2.0 ** -24}


@pytest.fixture(scope="module")
def P():
    import paper_1104_3870_amd as P

    P.lib()
    return P


class Ref:
    """Oracle pieces of the even-odd operator on one field."""

    def __init__(self, ns, nt, eps, seed, m0):
        self.ns, self.nt, self.m0 = ns, nt, m0
        self.U = synth.gauge_field(ns, nt, eps, seed)
        self.D = oracle.Dirac(self.U, m0, XI, CSW, BC)
        self.Ainv = np.linalg.inv(self.D.A)
        t, z, y, x = np.meshgrid(*(np.arange(n) for n in (nt, ns, ns, ns)), indexing="ij")
        self.par = (x + y + z + t) % 2
        self.g5 = oracle.gamma(4)
        self.ainv_norm = float(np.linalg.norm(self.Ainv, ord=2, axis=(-2, -1)).max())

    def mask(self, v, p):
        return v * (self.par == p)[..., None, None]

    def hop(self, v, p):
        """D_{p,1-p} v on parity p (zero elsewhere), v: [nt,ns,ns,ns,4,3]."""
        return self.mask(self.D.K(self.mask(v, 1 - p)), p)

    def gamma5(self, v):
        return np.einsum("ab,...bc->...ac", self.g5, v)

    def ainv(self, v):
        sh = v.shape
        return np.einsum("...ij,...j->...i", self.Ainv, v.reshape(sh[:-2] + (12,))).reshape(sh)


def exact_fields(rng, prec, shape):
    """Random spinor fields exactly representable in the storage precision."""
    if prec == "f16":
        k = rng.integers(-1023, 1024, size=shape + (2,)).astype(np.float64)
        k[..., 0, 0, 0] = 1024.0  # largest component of every site and field: scale 1
        v = k / 1024.0
    elif prec == "bf16":
        v = rng.integers(-127, 128, size=shape + (2,)).astype(np.float64) / 128.0
    elif prec == "f32":
        v = rng.uniform(-1, 1, size=shape + (2,)).astype(np.float32).astype(np.float64)
    else:
        v = rng.uniform(-1, 1, size=shape + (2,))
    return v[..., 0] + 1j * v[..., 1]


def check_out(got, ref, prec, p, par, e_site):
    """got, ref: [n, nt, ns, ns, ns, 4, 3]; e_site: extra absolute error per element."""
    assert np.all(got[:, par != p] == 0), "other parity not zero"
    d = got - ref
    if prec == "f16":
        smax = np.maximum(np.abs(ref.real), np.abs(ref.imag)).max(axis=(-2, -1), keepdims=True)
        bound = U_OUT[prec] * smax * 1.001 + e_site
        ok_re = np.abs(d.real) <= bound
        ok_im = np.abs(d.imag) <= bound
    else:
        ok_re = np.abs(d.real) <= U_OUT[prec] * np.abs(ref.real) * 1.001 + e_site
        ok_im = np.abs(d.imag) <= U_OUT[prec] * np.abs(ref.imag) * 1.001 + e_site
    bad = ~(ok_re & ok_im)
    if bad.any():
        i = np.argwhere(bad)[0]
        raise AssertionError("element %s: got %r ref %r (max |d| %.3e, e_site %.3e)"
                             % (tuple(i), got[tuple(i)], ref[tuple(i)], np.abs(d).max(), e_site))


def run_case(P, ref, prec, mode, p, R, gamma5, tg, walk, spb, a, c, seed, y_is_x=False):
    import torch

    say("hop", ref.ns, ref.nt, prec, mode, "p", p, "R", R, "g5", gamma5, "tg", tg, "walk", walk, "S", spb)
    rng = np.random.default_rng(seed)
    shape = (R, ref.nt, ref.ns, ref.ns, ref.ns, 4)
    inp = exact_fields(rng, prec, shape + (3,))
    use_x = mode in (P.LAPH_HOP_INV_DAG, P.LAPH_HOP_PLAIN_CG, P.LAPH_HOP_INV_DOT) or (seed % 2 == 0)
    x = exact_fields(rng, prec, shape + (3,)) if use_x else None
    y = exact_fields(rng, prec, shape + (3,)) if mode == P.LAPH_HOP_INV_DOT else None
    if y_is_x:
        y = x
    r0 = exact_fields(rng, prec, shape + (3,)) if mode == P.LAPH_HOP_PLAIN_CG else None
    alpha = rng.uniform(0.2, 1.5, size=R) if mode == P.LAPH_HOP_PLAIN_CG else None
    if alpha is not None and prec != "f64":
        alpha = alpha.astype(np.float32).astype(np.float64)  # the kernel takes alpha in FP32

    L = P.Lattice(ref.ns, ref.nt)
    prm = P.laph_dirac(ref.m0, XI, CSW, BC)
    out = dev(r0) if r0 is not None else torch.empty(shape + (3,), dtype=torch.complex128, device="cuda")
    out2 = torch.empty_like(out) if mode == P.LAPH_HOP_INV_DAG else None
    if y is not None:
        out2 = dev(y)  # INV_DOT: the field y, an input
    xd = dev(x) if use_x else None
    if y_is_x:
        out2 = xd  # the same device field: the kernel's y = x form
    nrm = P.laph_hop_apply(L.ctx, dev(ref.U), prm, prec, mode, p, dev(inp), out, x=xd,
                           out2=out2, alpha=alpha, gamma5=gamma5, temporal_gauge=tg, walk=walk, sites_per_block=spb,
                           a=a, c=c)
    got = host(out)
    L.close()

    # reference
    hop = np.stack([ref.hop(inp[r], p) for r in range(R)])
    if gamma5:
        hop = ref.gamma5(hop)
    inv = mode in (P.LAPH_HOP_INV, P.LAPH_HOP_INV_DAG, P.LAPH_HOP_INV_DOT)
    body = c * (ref.ainv(hop) if inv else hop)
    xs = ref.mask(x, p) if use_x else 0.0
    v = body + a * xs

    if prec == "f64":
        want = v if mode != P.LAPH_HOP_PLAIN_CG else None
        scale = np.abs(want).max()
        assert np.abs(got - want).max() <= 1e-13 * scale, np.abs(got - want).max() / scale
        return
    gain = ref.ainv_norm if inv else 1.0
    e_arith = 2e-5 * (abs(a) + abs(c) * max(gain, 1.0))
    if tg:
        e_arith += 8 * U_IN[prec] * (abs(c) * max(gain, 1.0) + abs(a)) * 2.0
    if mode == P.LAPH_HOP_PLAIN_CG:
        want = ref.mask(r0, p) - alpha[:, None, None, None, None, None, None] * v
        check_out(got, want, prec, p, ref.par, e_arith * alpha.max() + (U_IN[prec] * 2 if tg else 0.0))
    else:
        want = v
        check_out(got, want, prec, p, ref.par, e_arith)
    if mode in (P.LAPH_HOP_INV_DAG, P.LAPH_HOP_PLAIN_CG):
        # the epilogue's norms come from the stored values
        stored = np.sum(np.abs(got) ** 2, axis=(1, 2, 3, 4, 5, 6))
        np.testing.assert_allclose(nrm, stored, rtol=1e-6, atol=0)
        exact = np.sum(np.abs(want) ** 2, axis=(1, 2, 3, 4, 5, 6))
        np.testing.assert_allclose(nrm, exact, rtol=8 * U_IN[prec] + 1e-5 + (2e-3 if tg else 0.0), atol=0)
    if mode == P.LAPH_HOP_INV_DOT:
        # <y, out> and |out|^2 per field from the stored out (FP32 sums of 24 products per
        # site and field, FP64 beyond: 4e-6 of sum |y| |out|), and against the exact out
        # within sum |y| |got - want| (+ the rounding of the rotated y in temporal gauge)
        assert np.array_equal(host(out2), y), "INV_DOT changed its input y"
        ym = ref.mask(y, p)
        ax = (1, 2, 3, 4, 5, 6)
        dots = nrm.reshape(R, 3)
        got_dot = np.sum(np.conj(ym) * got, axis=ax)
        mag = np.sum(np.abs(ym) * np.abs(got), axis=ax)
        e_tg = 8 * U_IN[prec] * mag if tg else 0.0
        for e, val in ((0, got_dot.real), (1, got_dot.imag)):
            assert np.all(np.abs(dots[:, e] - val) <= 4e-6 * mag + e_tg), (e, dots[:, e], val)
        stored = np.sum(np.abs(got) ** 2, axis=ax)
        np.testing.assert_allclose(dots[:, 2], stored, rtol=1e-6 + (8 * U_IN[prec] if tg else 0.0), atol=0)
        exact = np.sum(np.conj(ym) * want, axis=ax)
        dev_ = np.sum(np.abs(ym) * np.abs(got - want), axis=ax)
        assert np.all(np.abs(dots[:, 0] + 1j * dots[:, 1] - exact) <= dev_ + 4e-6 * mag + e_tg)
    if mode == P.LAPH_HOP_INV_DAG:
        # out2 = A^-1 gamma_5 out; the reference applies them to the exact out, so the
        # rounding of the stored out enters through |A^-1|
        g2 = host(out2)
        want2 = ref.ainv(ref.gamma5(want))
        d_out = np.abs(got - want).max()
        e2 = ref.ainv_norm * d_out * np.sqrt(24) + 2e-5 * ref.ainv_norm
        check_out(g2, want2, prec, p, ref.par, e2)


_REFS = {}


def get_ref(ns, nt, m0=-0.05):
    key = (ns, nt, m0)
    if key not in _REFS:
        _REFS[key] = Ref(ns, nt, 0.4 if ns > 4 else 0.3, 11 + ns + nt, m0)
    return _REFS[key]


MODES = ["PLAIN", "INV", "INV_DAG", "PLAIN_CG", "INV_DOT"]


@pytest.mark.parametrize("prec", ["f16", "bf16", "f32"])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("ns,nt", [(4, 8), (6, 4)])
@pytest.mark.parametrize("tg,walk", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_hop_small(P, prec, mode, ns, nt, tg, walk):
    """Every mode, precision, gauge and site order on 4^3 x 8 and 6^3 x 4 (Vh = 432: the
    32-lane blocks of 8 sites leave a ragged last block), both parities, R = 4 and 32."""
    ref = get_ref(ns, nt)
    m = getattr(P, "LAPH_HOP_" + mode)
    for R, p, g5 in ((4, walk, 0), (32, 1 - walk, 1)):
        a, c = (1.0, -1.0) if mode != "PLAIN" else (0.5, -0.7)
        run_case(P, ref, prec, m, p, R, g5, tg, walk, 0, a, c, seed=zlib.crc32(repr((ns, nt, mode, prec, tg, walk, R)).encode()) % 1000)


@pytest.mark.parametrize("prec", ["f16", "bf16", "f32"])
@pytest.mark.parametrize("R,S", [(8, 0), (16, 0), (4, 3), (8, 7), (2, 5), (1, 64)])
def test_hop_blocks_and_tiles(P, prec, R, S):
    """Other block sizes and explicit tiles (S sites x R lanes, S not dividing Vh)."""
    ref = get_ref(6, 4)
    for mode in (P.LAPH_HOP_INV, P.LAPH_HOP_INV_DAG, P.LAPH_HOP_PLAIN_CG, P.LAPH_HOP_INV_DOT):
        run_case(P, ref, prec, mode, 1, R, 0, 1, 0, S, 1.0, -1.0, seed=R * 100 + S)


@pytest.mark.parametrize("R,tg,p,mode", [(1, 0, 0, "PLAIN"), (4, 1, 1, "INV"), (32, 1, 0, "INV"), (32, 0, 1, "PLAIN")])
def test_hop_fp64(P, R, tg, p, mode):
    """The FP64 hop of the reliable updates and the plain solver (1e-13 relative)."""
    ref = get_ref(6, 4)
    run_case(P, ref, "f64", getattr(P, "LAPH_HOP_" + mode), p, R, R % 2, tg, 0, 0, 0.3, -1.0, seed=R + 7 * tg)


@pytest.mark.parametrize("prec", ["f16", "bf16", "f32"])
@pytest.mark.parametrize("mode", MODES)
def test_hop_16x32(P, prec, mode):
    """The tiled site walk on 16^3 x 32 at R = 32 in temporal gauge (the solver's launch
    shape); the INV hop of FP16 also in the caller's gauge."""
    ref = get_ref(16, 32, -0.12)
    m = getattr(P, "LAPH_HOP_" + mode)
    run_case(P, ref, prec, m, 1, 32, 1 if mode == "PLAIN_CG" else 0, 1, 0, 0, 1.0, -1.0, seed=3)
    if prec == "f16" and mode == "INV":
        run_case(P, ref, prec, m, 0, 32, 0, 0, 0, 0, 1.0, -1.0, seed=4)


@pytest.mark.parametrize("prec", ["f16", "bf16", "f32"])
@pytest.mark.parametrize("tg", [0, 1])
def test_hop_dot_y_is_x(P, prec, tg):
    """INV_DOT with y the own-site operand x itself (BiCGStab's <s, M s>): the kernel
    takes y from the loaded x instead of a second load."""
    ref = get_ref(6, 4)
    for R, p in ((4, 0), (32, 1)):
        run_case(P, ref, prec, P.LAPH_HOP_INV_DOT, p, R, 0, tg, 0, 0, 1.0, -1.0, seed=40 + R + tg, y_is_x=True)


def test_hop_fp64_16x32(P):
    ref = get_ref(16, 32, -0.12)
    run_case(P, ref, "f64", P.LAPH_HOP_INV, 1, 32, 0, 1, 0, 0, 1.0, -1.0, seed=5)


def test_hop_rejects_bad_arguments(P):
    import torch

    import paper_1104_3870_amd as PP

    ref = get_ref(4, 8)
    L = P.Lattice(4, 8)
    inp = dev(exact_fields(np.random.default_rng(2), "f16", (4, 8, 4, 4, 4, 4, 3)))
    out = torch.empty_like(inp)
    prm = P.laph_dirac(ref.m0, XI, CSW, BC)
    for kw in (dict(mode=P.LAPH_HOP_INV_DAG),  # needs x and out2
               dict(mode=P.LAPH_HOP_INV, inp=inp[:3], out=out[:3]),  # 3 fields: not a power of two
               dict(mode=P.LAPH_HOP_PLAIN_CG, x=inp),  # needs alpha
               dict(mode=P.LAPH_HOP_INV, parity=2),
               dict(mode=P.LAPH_HOP_INV, sites_per_block=128),  # 128 x 4 lanes > 256
               dict(mode=P.LAPH_HOP_INV_DAG, precision="f64", x=inp, out2=out),
               dict(mode=P.LAPH_HOP_INV_DOT, x=inp),  # needs y in out2
               dict(mode=P.LAPH_HOP_INV_DOT, precision="f64", x=inp, out2=out)):
        args = dict(precision="f16", parity=0)
        args.update(kw)
        prec, mode, parity = args.pop("precision"), args.pop("mode"), args.pop("parity")
        i_, o_ = args.pop("inp", inp), args.pop("out", out)
        with pytest.raises(PP.LaphError) as e:
            P.laph_hop_apply(L.ctx, dev(ref.U), prm, prec, mode, parity, i_, o_, **args)
        assert e.value.code == P.LAPH_EINVAL, kw
    L.close()

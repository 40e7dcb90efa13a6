// Multi-right-hand-side hopping kernel for the low-precision inner solves (FP32
// arithmetic, FP16 / BF16 / FP32 records).
//
// k_dslash_lds stages a block's links (stored as their first two rows, reconstruct-12: the
// third row of an SU(3) matrix is conj(row0 x row1)) and clover blocks in LDS and gives
// every lane one (site, right-hand side); see its section below.
#include <cstdlib>
#include <string>
#include <type_traits>

#include "dslash_mr.h"
#include "spinor_io.h"

namespace {

// s[q][alpha][c] for NR right-hand sides r0 .. r0+NR-1 of site j (site-major layout:
// each right-hand side's spinor is one contiguous record)
template <class SP, int NR>
__device__ __forceinline__ void load_site(const typename SP::E *s, const float *nrm, long Vh, int R, long j, int r0,
                                          Cx<float> (&out)[NR][4][3])
{
#pragma unroll
    for (int q = 0; q < NR; q++) {
        Cx<float> v[12];
        ld_spinor12<SP, float>(s, nrm, Vh, R, j, r0 + q, v);
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int c = 0; c < 3; c++) out[q][a][c] = v[a * 3 + c];
    }
}

template <class SP, int NR>
__device__ __forceinline__ void store_site(typename SP::E *s, float *nrm, long Vh, int R, long j, int r0,
                                           const Cx<float> (&in)[NR][4][3])
{
#pragma unroll
    for (int q = 0; q < NR; q++) {
        Cx<float> v[12];
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int c = 0; c < 3; c++) v[a * 3 + c] = in[q][a][c];
        st_spinor12<SP, float>(s, nrm, Vh, R, j, r0 + q, v);
    }
}

// link U (3x3) from its two stored rows
__device__ __forceinline__ void load_link12(const float4 *lk, long k, Cx<float> (&U)[9])
{
    float4 a = lk[k * 3], b = lk[k * 3 + 1], c = lk[k * 3 + 2];
    U[0] = {a.x, a.y};
    U[1] = {a.z, a.w};
    U[2] = {b.x, b.y};
    U[3] = {b.z, b.w};
    U[4] = {c.x, c.y};
    U[5] = {c.z, c.w};
    // row 2 = conj(row0 x row1)
    Cx<float> t0 = U[1] * U[5] - U[2] * U[4];
    Cx<float> t1 = U[2] * U[3] - U[0] * U[5];
    Cx<float> t2 = U[0] * U[4] - U[1] * U[3];
    U[6] = {t0.re, -t0.im};
    U[7] = {t1.re, -t1.im};
    U[8] = {t2.re, -t2.im};
}

// packed Hermitian 6x6 block (per-site AoS, 36 floats) times NR 6-vectors
template <int NR>
__device__ __forceinline__ void clover_site(const float4 *cl, long i, const Cx<float> (&in)[NR][4][3],
                                            Cx<float> (&out)[NR][4][3])
{
    const float4 *p = cl + i * 18;
#pragma unroll
    for (int blk = 0; blk < 2; blk++) {
        float e[36];
#pragma unroll
        for (int k = 0; k < 9; k++) {
            float4 v = p[blk * 9 + k];
            e[4 * k] = v.x;
            e[4 * k + 1] = v.y;
            e[4 * k + 2] = v.z;
            e[4 * k + 3] = v.w;
        }
#pragma unroll
        for (int q = 0; q < NR; q++) {
            Cx<float> v[6], o[6];
#pragma unroll
            for (int s = 0; s < 2; s++)
#pragma unroll
                for (int c = 0; c < 3; c++) v[s * 3 + c] = in[q][blk * 2 + s][c];
#pragma unroll
            for (int k = 0; k < 6; k++) o[k] = e[k] * v[k];
            int idx = 6;
#pragma unroll
            for (int r = 1; r < 6; r++)
#pragma unroll
                for (int c = 0; c < r; c++) {
                    Cx<float> L = {e[idx], e[idx + 1]};
                    idx += 2;
                    o[r] = o[r] + L * v[c];
                    o[c] = o[c] + conjmul(L, v[r]);
                }
#pragma unroll
            for (int s = 0; s < 2; s++)
#pragma unroll
                for (int c = 0; c < 3; c++) out[q][blk * 2 + s][c] = o[s * 3 + c];
        }
    }
}

// the LDS-staged kernel runs at least 3 waves per SIMD (at most 168 VGPRs); no
// instantiation spills, and the FP16 ones of the CG iteration need 90-95 VGPRs (5 waves)
#ifndef LAPH_LDS_WAVES
#define LAPH_LDS_WAVES 3
#endif
#define LAPH_LDS_ATTR __attribute__((amdgpu_waves_per_eu(LAPH_LDS_WAVES)))

// ------------------------------------------------------------ LDS-staged variant
// One block holds S sites x R right-hand sides, one lane per (site, right-hand side).  The
// 8 S links of the block (hop weight, boundary factor and for M_PLAIN the output factor
// folded in; backward links stored as their adjoint) and its S clover blocks are staged
// in LDS once, so a lane does only the spin projection, one SU(3) product per direction
// and the clover product, with explicit FMA chains.  The kernel is bound by VALU issue:
// neighbour records come through buffer loads (one offset register each) in a software-
// pipelined direction loop, the record scale and the gamma_5 sign ride on the
// accumulating FMAs, index divisions are multiply-highs, unit links of a temporal gauge
// are skipped, the sites are walked in tiles through time (MrArgs::wby) and outputs are
// stored non-temporally.
constexpr int kLkF4 = 5;  // float4 per staged link (18 floats used)

__device__ __forceinline__ Cx<float> cmul_f(Cx<float> a, Cx<float> b)
{
    return {fmaf(-a.im, b.im, a.re * b.re), fmaf(a.im, b.re, a.re * b.im)};
}
__device__ __forceinline__ void cfma_f(Cx<float> &acc, Cx<float> a, Cx<float> b)  // acc += a b
{
    acc.re = fmaf(a.re, b.re, acc.re);
    acc.re = fmaf(-a.im, b.im, acc.re);
    acc.im = fmaf(a.re, b.im, acc.im);
    acc.im = fmaf(a.im, b.re, acc.im);
}
__device__ __forceinline__ void cfmac_f(Cx<float> &acc, Cx<float> a, Cx<float> b)  // acc += conj(a) b
{
    acc.re = fmaf(a.re, b.re, acc.re);
    acc.re = fmaf(a.im, b.im, acc.re);
    acc.im = fmaf(a.re, b.im, acc.im);
    acc.im = fmaf(-a.im, b.re, acc.im);
}

// element k (alpha*3 + c) of a raw record as FP32 (no scale)
template <class SP>
__device__ __forceinline__ float lo_f(const typename SP::E &e)
{
    if constexpr (std::is_same<SP, S16>::value)
        return __low2float(e);
    else
        return SP::ld(&e, 0, 1.0f).re;
}
template <class SP>
__device__ __forceinline__ float hi_f(const typename SP::E &e)
{
    if constexpr (std::is_same<SP, S16>::value)
        return __high2float(e);
    else
        return SP::ld(&e, 0, 1.0f).im;
}

// h = a + K b for K = KR + i KI in {+-1, +-i} (the record's scale is applied when the
// link product is accumulated); with FP16 storage every term is one mixed-precision FMA
template <class SP, int KR, int KI>
__device__ __forceinline__ Cx<float> proj(const typename SP::E &a, const typename SP::E &b, float unit)
{
    const float are = lo_f<SP>(a), aim = hi_f<SP>(a), bre = lo_f<SP>(b), bim = hi_f<SP>(b);
    if constexpr (KI == 0)
        return {fmaf(bre, (float)KR * unit, are), fmaf(bim, (float)KR * unit, aim)};
    else
        return {fmaf(bim, -(float)KI * unit, are), fmaf(bre, (float)KI * unit, aim)};
}

// acc += s K o for K = KR + i KI in {+-1, +-i}
template <int KR, int KI>
__device__ __forceinline__ void acc_k(Cx<float> &acc, float s, Cx<float> o)
{
    if constexpr (KI == 0) {
        acc.re = fmaf((float)KR * s, o.re, acc.re);
        acc.im = fmaf((float)KR * s, o.im, acc.im);
    } else {
        acc.re = fmaf(-(float)KI * s, o.im, acc.re);
        acc.im = fmaf((float)KI * s, o.re, acc.im);
    }
}

// spin projection of a neighbour record: h0, h1 are the two independent colour vectors
// of (1 -+ gamma_mu) psi (FWD: 1 - gamma_mu, backward: 1 + gamma_mu), unscaled
template <int MU, bool FWD, class SP>
__device__ __forceinline__ void proj_lds(const Spin12<SP> &sp, float unit, Cx<float> (&h0)[3], Cx<float> (&h1)[3])
{
    const auto *v = sp.v;  // v[alpha * 3 + c]
    constexpr int sg = FWD ? 1 : -1;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        if (MU == 0) {
            h0[c] = proj<SP, 0, sg>(v[c], v[9 + c], unit);
            h1[c] = proj<SP, 0, sg>(v[3 + c], v[6 + c], unit);
        } else if (MU == 1) {
            h0[c] = proj<SP, sg, 0>(v[c], v[9 + c], unit);
            h1[c] = proj<SP, -sg, 0>(v[3 + c], v[6 + c], unit);
        } else if (MU == 2) {
            h0[c] = proj<SP, 0, sg>(v[c], v[6 + c], unit);
            h1[c] = proj<SP, 0, -sg>(v[3 + c], v[9 + c], unit);
        } else {
            h0[c] = proj<SP, -sg, 0>(v[c], v[6 + c], unit);
            h1[c] = proj<SP, -sg, 0>(v[3 + c], v[9 + c], unit);
        }
    }
}

// reconstruction of all four spin components of a hop from the two colour vectors o0, o1
// of its projected half spinor, each term scaled inside the accumulating FMA: by sc (upper
// components) and sl (lower components: sc, or -sc when gamma_5 follows the hop)
template <int MU, bool FWD>
__device__ __forceinline__ void accum(const Cx<float> (&o0)[3], const Cx<float> (&o1)[3], float sc, float sl,
                                      Cx<float> (&acc)[4][3])
{
    constexpr int f = FWD ? 1 : -1;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        acc_k<1, 0>(acc[0][c], sc, o0[c]);
        acc_k<1, 0>(acc[1][c], sc, o1[c]);
        if (MU == 0) {
            acc_k<0, -f>(acc[2][c], sl, o1[c]);
            acc_k<0, -f>(acc[3][c], sl, o0[c]);
        } else if (MU == 1) {
            acc_k<-f, 0>(acc[2][c], sl, o1[c]);
            acc_k<f, 0>(acc[3][c], sl, o0[c]);
        } else if (MU == 2) {
            acc_k<0, -f>(acc[2][c], sl, o0[c]);
            acc_k<0, f>(acc[3][c], sl, o1[c]);
        } else {
            acc_k<-f, 0>(acc[2][c], sl, o0[c]);
            acc_k<-f, 0>(acc[3][c], sl, o1[c]);
        }
    }
}

// staged link (weights folded in, backward links as their adjoint) times h0, h1, then accum
template <int MU, bool FWD>
__device__ __forceinline__ void mult_lds(const float4 *lk, const Cx<float> (&h0)[3], const Cx<float> (&h1)[3], float sc,
                                         float sl, Cx<float> (&acc)[4][3])
{
    const float2 *l2 = reinterpret_cast<const float2 *>(lk);
    Cx<float> o0[3], o1[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        Cx<float> u0 = {l2[a * 3].x, l2[a * 3].y}, u1 = {l2[a * 3 + 1].x, l2[a * 3 + 1].y},
                  u2 = {l2[a * 3 + 2].x, l2[a * 3 + 2].y};
        o0[a] = cmul_f(u0, h0[0]);
        cfma_f(o0[a], u1, h0[1]);
        cfma_f(o0[a], u2, h0[2]);
        o1[a] = cmul_f(u0, h1[0]);
        cfma_f(o1[a], u1, h1[1]);
        cfma_f(o1[a], u2, h1[2]);
    }
    accum<MU, FWD>(o0, o1, sc, sl, acc);
}

// a hop whose link is the unit matrix (temporal gauge): wid is the hop weight that the
// staged links carry folded in
template <int MU, bool FWD>
__device__ __forceinline__ void mult_unit(const Cx<float> (&h0)[3], const Cx<float> (&h1)[3], float sc, float sl,
                                          float wid, Cx<float> (&acc)[4][3])
{
    accum<MU, FWD>(h0, h1, sc * wid, sl * wid, acc);
}

// ul: the link is the unit matrix with weight wid (time direction in temporal gauge)
template <int MU, bool FWD, class SP>
__device__ __forceinline__ void hop_lds(const float4 *lk, const Spin12<SP> &sp, float sc, float g5s, float unit,
                                        bool ul, float wid, Cx<float> (&acc)[4][3])
{
    Cx<float> h0[3], h1[3];
    proj_lds<MU, FWD, SP>(sp, unit, h0, h1);
    if (MU == 3 && ul)
        mult_unit<MU, FWD>(h0, h1, sc, g5s * sc, wid, acc);
    else
        mult_lds<MU, FWD>(lk, h0, h1, sc, g5s * sc, acc);
}

// buffer resource over n bytes at p (raw 32-bit loads; reads past n return zero)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *p, unsigned n)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)n, 0x00020000);
}

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// neighbour record and its scale (1 without a scale) through buffer loads: one 32-bit
// offset register per record, the chunk stride R 16 in a scalar register (the caller
// guarantees Vh R sizeof(record) < 2^32)
template <class SP>
__device__ __forceinline__ void ld_nb(__amdgpu_buffer_rsrc_t rin, __amdgpu_buffer_rsrc_t rnrm, int nb, int R, int r,
                                      Spin12<SP> &sp, float &sc)
{
    constexpr int C = sizeof(Spin12<SP>) / 16;
    const int cs = R * 16;
    const unsigned off = ((unsigned)nb * (unsigned)(C * R) + (unsigned)r) * 16u;
#pragma unroll
    for (int q = 0; q < C; q++) {
        u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rin, (int)off, q * cs, 0);
        reinterpret_cast<uint4 *>(&sp)[q] = make_uint4(v.x, v.y, v.z, v.w);
    }
    if constexpr (SP::kNorm)
        sc = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rnrm, (int)(((unsigned)nb * (unsigned)R + (unsigned)r) * 4u), 0, 0));
    else
        sc = 1.0f;
}

// neighbour record of the input field (32-bit site index)
template <int MU, bool FWD, class SP>
__device__ __forceinline__ void dir_lds(__amdgpu_buffer_rsrc_t rin, __amdgpu_buffer_rsrc_t rnrm, const float4 *slk,
                                        int nb, int R, int r, float g5s, float unit, bool ul, float wid,
                                        Cx<float> (&acc)[4][3])
{
    Spin12<SP> sp;
    float sc;
    ld_nb<SP>(rin, rnrm, nb, R, r, sp, sc);
    hop_lds<MU, FWD, SP>(slk + (FWD ? MU : 4 + MU) * kLkF4, sp, sc, g5s, unit, ul, wid, acc);
}

// neighbour records kept in flight by the software-pipelined direction loop (0: the
// compiler's own schedule), measured on gfx950 at 24^3 x 128, R = 32, FP16.  Every mode
// runs the pipeline: with the clover-inverse epilogue and an own-site addend it takes
// 109-116 VGPRs (4 waves per SIMD, no spills) and cut those hops from 1.75-2.0 ms to
// 1.6-1.7 ms against the compiler's schedule, which waits on every neighbour load
#ifndef LAPH_PIPE_D
#define LAPH_PIPE_D 2
#endif

__device__ __forceinline__ void clover_one(const float4 *p, const Cx<float> (&in)[4][3], Cx<float> (&out)[4][3])
{
#pragma unroll
    for (int blk = 0; blk < 2; blk++) {
        float e[36];
#pragma unroll
        for (int k = 0; k < 9; k++) {
            float4 v = p[blk * 9 + k];
            e[4 * k] = v.x;
            e[4 * k + 1] = v.y;
            e[4 * k + 2] = v.z;
            e[4 * k + 3] = v.w;
        }
        Cx<float> v[6], o[6];
#pragma unroll
        for (int s = 0; s < 2; s++)
#pragma unroll
            for (int c = 0; c < 3; c++) v[s * 3 + c] = in[blk * 2 + s][c];
#pragma unroll
        for (int k = 0; k < 6; k++) o[k] = e[k] * v[k];
        int idx = 6;
#pragma unroll
        for (int rr = 1; rr < 6; rr++)
#pragma unroll
            for (int c = 0; c < rr; c++) {
                Cx<float> L = {e[idx], e[idx + 1]};
                idx += 2;
                cfma_f(o[rr], L, v[c]);
                cfmac_f(o[c], L, v[rr]);
            }
#pragma unroll
        for (int s = 0; s < 2; s++)
#pragma unroll
            for (int c = 0; c < 3; c++) out[blk * 2 + s][c] = o[s * 3 + c];
    }
}

// sites per block for R right-hand sides (block = S R lanes)
inline size_t lds_bytes(int S) { return (size_t)S * (8 * kLkF4 + 18) * sizeof(float4); }

// n / d through the launcher's multiply-high reciprocal m; m = 0 stands for d = 1 (the
// launcher guarantees a valid m for every other divisor, so no division code is emitted)
__device__ __forceinline__ unsigned udiv(unsigned n, unsigned d, unsigned m)
{
    (void)d;
    return m ? __umulhi(n, m) : n;
}

// checkerboard index and coordinates of position pos of the site walk (MrArgs::wby):
// tiles of ns x by x bz sites (full rows) one after the other, each visited slice by slice
// through all nt time slices, the sites of a tile slice in (x, y, z) order.  The XCD remap
// gives every XCD one contiguous range of the walk, so the records a slice reads from the
// slices before and after it were fetched by the same XCD one slice earlier.
__device__ __forceinline__ int walk_site(const MrArgs &P, unsigned pos, int &x, int &y, int &z, int &t)
{
    const unsigned ns = P.ns, nsh = ns >> 1;
    unsigned xh;
    if (P.wby == 0) {
        const unsigned r = udiv(pos, nsh, P.m_nsh), r2 = udiv(r, ns, P.m_ns), r3 = udiv(r2, ns, P.m_ns);
        xh = pos - r * nsh;
        y = (int)(r - r2 * ns);
        z = (int)(r2 - r3 * ns);
        t = (int)r3;
    } else {
        const unsigned by = P.wby, bz = P.wbz, A = nsh * by * bz, nt = P.nt;
        const unsigned q = udiv(pos, A, P.m_A), loc = pos - q * A;  // q = tile nt + t
        const unsigned tile = udiv(q, nt, P.m_nt);
        t = (int)(q - tile * nt);
        const unsigned q1 = udiv(loc, nsh, P.m_nsh), zz = udiv(q1, by, P.m_by);
        xh = loc - q1 * nsh;
        const unsigned nty = ns / by, tz = udiv(tile, nty, P.m_nty);
        y = (int)((tile - tz * nty) * by + (q1 - zz * by));
        z = (int)(tz * bz + zz);
    }
    x = 2 * (int)xh + ((y + z + t + P.par) & 1);
    return (int)xh + (int)nsh * (y + (int)ns * (z + (int)ns * t));
}

#ifndef LAPH_LDS_NT
#define LAPH_LDS_NT 1
#endif
// output records streamed past L2 (1: every epilogue, 2: all but M_INV_AFTER_DAG)
template <int MODE>
constexpr bool nt_out()
{
    return LAPH_LDS_NT == 1 || (LAPH_LDS_NT == 2 && MODE != M_INV_AFTER_DAG);
}

// HX: the launch has an own-site addend (P.x); a compile-time switch so that the hops of
// the CG iteration without one keep the register budget of the pipelined loop
template <class SP, int MODE, bool HX>
__global__ __launch_bounds__(256) LAPH_LDS_ATTR void k_dslash_lds(const MrArgs P)
{
    extern __shared__ float4 smem[];
    const int R = P.R;
    const int S = blockDim.x / R;  // sites per block
    float4 *slk = smem;                 // [S][8][kLkF4]
    float4 *scl = smem + S * 8 * kLkF4;  // [S][18]
    const long Vh = P.Vh;
    const int ns = P.ns, nt = P.nt, par = P.par, opar = par ^ 1;
    const long pos0 = (long)xcd_block(blockIdx.x, gridDim.x) * S;  // walk position of lane-site 0
    const float4 *lk = (const float4 *)P.links;
    constexpr bool kInv = MODE == M_INV_AFTER || MODE == M_INV_AFTER_DAG || MODE == M_INV_AFTER_DOT;
    const float fout = kInv ? 1.0f : (float)P.c;  // folded into the links
    for (int k = threadIdx.x; k < S * 8; k += blockDim.x) {
        const int sl = k >> 3, d = k & 7, mu = d & 3;
        if (pos0 + sl >= Vh) continue;
        int x, y, z, t;
        const long i = walk_site(P, (unsigned)(pos0 + sl), x, y, z, t);
        if (mu == 3 && P.tgauge && (d < 4 ? t + 1 < nt : t > 0)) continue;  // unit link, not read
        float w = fout * (mu == 3 ? (float)P.wt : (float)P.ws);
        long li;
        if (d < 4) {
            if (mu == 3 && t + 1 == nt) w *= (float)P.bct;
            li = (long)(mu * 2 + par) * Vh + i;
        } else {
            int xx = x, yy = y, zz = z, tt = t;
            if (mu == 0) xx = x == 0 ? ns - 1 : x - 1;
            else if (mu == 1) yy = y == 0 ? ns - 1 : y - 1;
            else if (mu == 2) zz = z == 0 ? ns - 1 : z - 1;
            else {
                tt = t == 0 ? nt - 1 : t - 1;
                if (t == 0) w *= (float)P.bct;
            }
            li = (long)(mu * 2 + opar) * Vh + (lex_index(xx, yy, zz, tt, ns) >> 1);
        }
        Cx<float> U[9];
        load_link12(lk, li, U);
        float f[20];
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) {
                Cx<float> u = d < 4 ? U[a * 3 + b] : Cx<float>{U[b * 3 + a].re, -U[b * 3 + a].im};
                f[2 * (a * 3 + b)] = w * u.re;
                f[2 * (a * 3 + b) + 1] = w * u.im;
            }
        f[18] = f[19] = 0.0f;
        float4 *dst = slk + (size_t)k * kLkF4;
#pragma unroll
        for (int q = 0; q < kLkF4; q++) dst[q] = make_float4(f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]);
    }
    if constexpr (kInv) {
        const float4 *cl = (const float4 *)P.clov;
        const float cc = (float)P.c;
        for (int k = threadIdx.x; k < S * 18; k += blockDim.x) {
            const int sl = k / 18;
            if (pos0 + sl >= Vh) continue;
            int x, y, z, t;
            const long i = walk_site(P, (unsigned)(pos0 + sl), x, y, z, t);
            float4 v = cl[i * 18 + (k - sl * 18)];
            scl[k] = make_float4(cc * v.x, cc * v.y, cc * v.z, cc * v.w);
        }
    }
    __syncthreads();
    const int sl = threadIdx.x / R, r = threadIdx.x - sl * R;
    const bool valid = sl < S && pos0 + sl < Vh;
    // block reduction of NQ values per lane
    constexpr bool kRed = MODE == M_INV_AFTER_DAG || MODE == M_PLAIN_CG || MODE == M_INV_AFTER_DOT;
    constexpr int NQ = MODE == M_INV_AFTER_DOT ? 3 : 1;
    if constexpr (!kRed) {
        if (!valid) return;
    }
    // this lane's |out|^2 (DAG) or |r|^2 (CG), or Re, Im <y, out> and |out|^2 (DOT): 24
    // terms of one site and right-hand side in FP32, the sums over sites in FP64
    float nq = 0.0f, dre = 0.0f, dim = 0.0f;
    if (valid) {
    // 32-bit site arithmetic (the host checks Vh * R * 12 < 2^31): neighbour checkerboard
    // indices from the site's own, lex = 2 cb + (x & 1) since Ns is even
    int x, y, z, t;
    const int cb = walk_site(P, (unsigned)(pos0 + sl), x, y, z, t);
    // temporal gauge: unit time links except from the last slice forward (and into the
    // first slice backward); the branch is uniform over a block, whose sites share t
    const bool unit_f = P.tgauge && t + 1 < nt, unit_b = P.tgauge && t > 0;
    const float wid = fout * (float)P.wt;
    const int sy = ns >> 1, sz = sy * ns, st = sz * ns;
    const int xo = x & 1;
    const int nxp = (x + 1 < ns) ? cb + xo : cb + 1 - sy;
    const int nxm = (x > 0) ? cb - 1 + xo : cb + sy - 1;
    const int nyp = (y + 1 < ns) ? cb + sy : cb - (ns - 1) * sy;
    const int nym = (y > 0) ? cb - sy : cb + (ns - 1) * sy;
    const int nzp = (z + 1 < ns) ? cb + sz : cb - (ns - 1) * sz;
    const int nzm = (z > 0) ? cb - sz : cb + (ns - 1) * sz;
    const int ntp = (t + 1 < nt) ? cb + st : cb - (nt - 1) * st;
    const int ntm = (t > 0) ? cb - st : cb + (nt - 1) * st;
    const long i = cb;
    Cx<float> acc[4][3];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) acc[a][c] = {0.0f, 0.0f};
    const float4 *my = slk + (size_t)sl * 8 * kLkF4;
    const float unit = P.unit;
    const float g5s = P.g5d ? -1.0f : 1.0f;  // gamma_5 after the hop: lower components negated
    const __amdgpu_buffer_rsrc_t rin = buf_rsrc(P.in, (unsigned)(Vh * R * sizeof(Spin12<SP>)));
    const __amdgpu_buffer_rsrc_t rnrm = buf_rsrc(P.in_nrm, SP::kNorm ? (unsigned)(Vh * R * 4) : 0u);
    constexpr int D = LAPH_PIPE_D;
    if constexpr (D > 0) {
        // D neighbour records in flight: the slot a direction's spin projection frees is
        // refilled with the record D directions ahead before that direction's link product,
        // so the loads overlap the arithmetic (scheduling fences keep this order)
        const int nbs[8] = {nxp, nxm, nyp, nym, nzp, nzm, ntp, ntm};
        Spin12<SP> bs[D];
        float cs[D];
#pragma unroll
        for (int k = 0; k < D; k++) ld_nb<SP>(rin, rnrm, nbs[k], R, r, bs[k], cs[k]);
#pragma unroll
        for (int k = 0; k < 8; k++) {
            Cx<float> h0[3], h1[3];
            __builtin_amdgcn_sched_barrier(0);
            switch (k) {
            case 0: proj_lds<0, true, SP>(bs[k % D], unit, h0, h1); break;
            case 1: proj_lds<0, false, SP>(bs[k % D], unit, h0, h1); break;
            case 2: proj_lds<1, true, SP>(bs[k % D], unit, h0, h1); break;
            case 3: proj_lds<1, false, SP>(bs[k % D], unit, h0, h1); break;
            case 4: proj_lds<2, true, SP>(bs[k % D], unit, h0, h1); break;
            case 5: proj_lds<2, false, SP>(bs[k % D], unit, h0, h1); break;
            case 6: proj_lds<3, true, SP>(bs[k % D], unit, h0, h1); break;
            default: proj_lds<3, false, SP>(bs[k % D], unit, h0, h1); break;
            }
            const float sck = cs[k % D];
            __builtin_amdgcn_sched_barrier(0);
            if (k + D < 8) ld_nb<SP>(rin, rnrm, nbs[k + D], R, r, bs[k % D], cs[k % D]);
            __builtin_amdgcn_sched_barrier(0);
            const float4 *lk = my + ((k & 1) ? 4 + (k >> 1) : (k >> 1)) * kLkF4;
            switch (k) {
            case 0: mult_lds<0, true>(lk, h0, h1, sck, g5s * sck, acc); break;
            case 1: mult_lds<0, false>(lk, h0, h1, sck, g5s * sck, acc); break;
            case 2: mult_lds<1, true>(lk, h0, h1, sck, g5s * sck, acc); break;
            case 3: mult_lds<1, false>(lk, h0, h1, sck, g5s * sck, acc); break;
            case 4: mult_lds<2, true>(lk, h0, h1, sck, g5s * sck, acc); break;
            case 5: mult_lds<2, false>(lk, h0, h1, sck, g5s * sck, acc); break;
            case 6:
                if (unit_f)
                    mult_unit<3, true>(h0, h1, sck, g5s * sck, wid, acc);
                else
                    mult_lds<3, true>(lk, h0, h1, sck, g5s * sck, acc);
                break;
            default:
                if (unit_b)
                    mult_unit<3, false>(h0, h1, sck, g5s * sck, wid, acc);
                else
                    mult_lds<3, false>(lk, h0, h1, sck, g5s * sck, acc);
                break;
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    } else {
        dir_lds<0, true, SP>(rin, rnrm, my, nxp, R, r, g5s, unit, false, wid, acc);
        dir_lds<0, false, SP>(rin, rnrm, my, nxm, R, r, g5s, unit, false, wid, acc);
        dir_lds<1, true, SP>(rin, rnrm, my, nyp, R, r, g5s, unit, false, wid, acc);
        dir_lds<1, false, SP>(rin, rnrm, my, nym, R, r, g5s, unit, false, wid, acc);
        dir_lds<2, true, SP>(rin, rnrm, my, nzp, R, r, g5s, unit, false, wid, acc);
        dir_lds<2, false, SP>(rin, rnrm, my, nzm, R, r, g5s, unit, false, wid, acc);
        dir_lds<3, true, SP>(rin, rnrm, my, ntp, R, r, g5s, unit, unit_f, wid, acc);
        dir_lds<3, false, SP>(rin, rnrm, my, ntm, R, r, g5s, unit, unit_b, wid, acc);
    }
    Cx<float> res[4][3];
    if constexpr (kInv) {
        clover_one(scl + (size_t)sl * 18, acc, res);
    } else {
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int c = 0; c < 3; c++) res[a][c] = acc[a][c];
    }
    // a run-time test even when HX holds: an unconditional load of x is hoisted to the
    // start of the kernel, where its registers push the pipelined loop into spills
    // the own-site record as loaded (DOT with y = x, BiCGStab's t = M s and <s, t>, takes
    // y from it)
    Spin12<SP> xrec;
    float xn = 1.0f;
    if (HX && P.x) {
        xrec = ld_rec<SP>((const typename SP::E *)P.x, i, R, r);
        if constexpr (SP::kNorm) xn = P.x_nrm[i * R + r];
        const float sx = (float)P.a * xn;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const Cx<float> xv = SP::ld(&xrec.v[k], 0, 1.0f);
            res[k / 3][k % 3].re = fmaf(sx, xv.re, res[k / 3][k % 3].re);
            res[k / 3][k % 3].im = fmaf(sx, xv.im, res[k / 3][k % 3].im);
        }
    }
    Cx<float> v[12];
#pragma unroll
    for (int k = 0; k < 12; k++) v[k] = res[k / 3][k % 3];
    if constexpr (MODE == M_INV_AFTER_DAG) {
        // out as stored; |out|^2 and A^-1 gamma_5 out from the rounded values (what a
        // separate pass would read back); the staged clover block holds c A^-1
        st_spinor12_round<SP, nt_out<MODE>()>((typename SP::E *)P.out, P.out_nrm, Vh, R, i, r, v);
        Cx<float> g[4][3], o2[4][3];
#pragma unroll
        for (int k = 0; k < 12; k++) {
            nq = fmaf(v[k].re, v[k].re, fmaf(v[k].im, v[k].im, nq));
            g[k / 3][k % 3] = k < 6 ? v[k] : cneg(v[k]);
        }
        clover_one(scl + (size_t)sl * 18, g, o2);
        const float ic = 1.0f / (float)P.c;
#pragma unroll
        for (int k = 0; k < 12; k++) v[k] = ic * o2[k / 3][k % 3];
        st_spinor12<SP, float, nt_out<MODE>()>((typename SP::E *)P.out2, P.out2_nrm, Vh, R, i, r, v);
    } else if constexpr (MODE == M_PLAIN_CG) {
        // residual update of CG on the normal equations, r -= alpha out; |r|^2 of the
        // stored residual (the solution increment follows in the direction update)
        if (P.sc[r].active) {
            const float al = (float)P.sc[r].alpha.x;
            Cx<float> a[12];
            ld_spinor12<SP, float>((const typename SP::E *)P.cg_r, P.cg_r_nrm, Vh, R, i, r, a);
#pragma unroll
            for (int k = 0; k < 12; k++) a[k] = {fmaf(-al, v[k].re, a[k].re), fmaf(-al, v[k].im, a[k].im)};
            st_spinor12_round<SP, nt_out<MODE>()>((typename SP::E *)P.cg_r, P.cg_r_nrm, Vh, R, i, r, a);
#pragma unroll
            for (int k = 0; k < 12; k++) nq = fmaf(a[k].re, a[k].re, fmaf(a[k].im, a[k].im, nq));
        }
    } else if constexpr (MODE == M_INV_AFTER_DOT) {
        // out as stored; <y, out> and |out|^2 from the stored records: sums of products of
        // the records' values (FP16: exact in FP32, one mixed FMA each), times the scales
        Spin12<SP> orec;
        float so;
        st_spinor12_rec<SP, nt_out<MODE>()>((typename SP::E *)P.out, P.out_nrm, i, R, r, v, orec, so);
        Spin12<SP> yrec = xrec;
        float sy = xn;
        if (P.dot_y != P.x) {
            yrec = ld_rec<SP>((const typename SP::E *)P.dot_y, i, R, r);
            if constexpr (SP::kNorm) sy = P.dot_y_nrm[i * R + r];
        }
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const Cx<float> h = SP::ld(&orec.v[k], 0, 1.0f), y = SP::ld(&yrec.v[k], 0, 1.0f);
            nq = fmaf(h.re, h.re, fmaf(h.im, h.im, nq));
            dre = fmaf(y.re, h.re, fmaf(y.im, h.im, dre));
            dim = fmaf(y.re, h.im, fmaf(-y.im, h.re, dim));
        }
        nq *= so * so;
        dre *= so * sy;
        dim *= so * sy;
    } else {
        st_spinor12<SP, float, nt_out<MODE>()>((typename SP::E *)P.out, P.out_nrm, Vh, R, i, r, v);
    }
    }  // valid
    if constexpr (kRed) {
        // deterministic block sum per right-hand side over the lanes sl = 0 .. S-1 of each
        // r; each block stores its NQ x R sums contiguously ([block][value][RHS]: whole cache
        // lines, where one value per line for every block cost a fifth of the output bytes)
        __shared__ double red[NQ][256];
        if constexpr (NQ == 3) {
            red[0][threadIdx.x] = (double)dre;
            red[1][threadIdx.x] = (double)dim;
            red[2][threadIdx.x] = (double)nq;
        } else {
            red[0][threadIdx.x] = (double)nq;
        }
        __syncthreads();
        if ((int)threadIdx.x < R) {
#pragma unroll
            for (int e = 0; e < NQ; e++) {
                double s2 = 0.0;
                for (int q = 0; q < S; q++) s2 += red[e][q * R + threadIdx.x];
                P.partial[((size_t)blockIdx.x * NQ + e) * R + threadIdx.x] = s2;
            }
        }
    }
}

// out = A x with optional gamma_5 on x (local, per-site clover)
template <class SP, int NR>
__global__ __launch_bounds__(256) void k_clover_mr(const float4 *__restrict__ cl, const typename SP::E *__restrict__ x,
                                                   const float *x_nrm, typename SP::E *__restrict__ out, float *out_nrm,
                                                   long Vh, int R, int g5_in)
{
    long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int G = R / NR;
    if (tid >= Vh * G) return;
    long i = tid / G;
    int r0 = (int)(tid - i * G) * NR;
    Cx<float> v[NR][4][3], o[NR][4][3];
    load_site<SP, NR>(x, x_nrm, Vh, R, i, r0, v);
    if (g5_in) {
#pragma unroll
        for (int q = 0; q < NR; q++)
#pragma unroll
            for (int c = 0; c < 3; c++) {
                v[q][2][c] = cneg(v[q][2][c]);
                v[q][3][c] = cneg(v[q][3][c]);
            }
    }
    clover_site<NR>(cl, i, v, o);
    store_site<SP, NR>(out, out_nrm, Vh, R, i, r0, o);
}

// per-site packed clover blocks (SoA FP64) -> per-site AoS FP32 (72 floats)
__global__ void k_clover_aos(const double *__restrict__ soa, float *__restrict__ aos, long Vh)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= 2 * Vh) return;
    int par = (int)(t / Vh);
    long i = t - (long)par * Vh;
    for (int e = 0; e < 72; e++) aos[t * 72 + e] = (float)soa[((long)par * 72 + e) * Vh + i];
}

// even-odd SoA FP64 links -> reconstruct-12 AoS FP32 (rows 0 and 1)
__global__ void k_links12(const double2 *__restrict__ g64, float4 *__restrict__ lk, long Vh)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= 8 * Vh) return;
    long mp = t / Vh, i = t - mp * Vh;  // mp = mu * 2 + par
    double2 e[6];
    for (int k = 0; k < 6; k++) e[k] = g64[(mp * 9 + k) * Vh + i];
    lk[t * 3] = make_float4((float)e[0].x, (float)e[0].y, (float)e[1].x, (float)e[1].y);
    lk[t * 3 + 1] = make_float4((float)e[2].x, (float)e[2].y, (float)e[3].x, (float)e[3].y);
    lk[t * 3 + 2] = make_float4((float)e[4].x, (float)e[4].y, (float)e[5].x, (float)e[5].y);
}

}  // namespace

double dslash_mr_bytes(long Vh, int R, int sbytes, bool has_norm, int mode, bool has_x, bool y_is_x)
{
    double site = 8.0 * 48;  // reconstruct-12 FP32 links
    if (mode == M_INV_AFTER || mode == M_INV_AFTER_DAG || mode == M_INV_AFTER_DOT) site += 72.0 * 4;
    // in, out[, x][, out2 or a y other than x]; the CG form also reads r (and writes it
    // instead of out)
    int streams = 2 + (has_x ? 1 : 0) + (mode == M_INV_AFTER_DAG || (mode == M_INV_AFTER_DOT && !y_is_x) ? 1 : 0);
    if (mode == M_PLAIN_CG) streams += 1;
    double per_rhs = 12.0 * sbytes * streams + (has_norm ? 4.0 * streams : 0.0);
    return (double)Vh * (site + R * per_rhs);
}

template <class SP>
constexpr int prec_id()
{
    return std::is_same<SP, S16>::value ? LAPH_PREC_F16 : std::is_same<SP, SB16>::value ? LAPH_PREC_BF16 : LAPH_PREC_F32;
}

// sites per block of the LDS-staged kernel: the caller's override, the tuned value, else
// 256 / R lanes per block
int lds_tile_sites(laph_ctx *c, int prec, int R)
{
    if (c->tile_override > 0) return c->tile_override;
    auto it = c->lds_tile.find({prec, R});
    if (it != c->lds_tile.end()) return it->second;
    return R >= 4 ? 256 / R : 64;
}

template <class SP>
constexpr const char *prec_name()
{
    return std::is_same<SP, S16>::value ? "f16" : std::is_same<SP, SB16>::value ? "bf16" : "f32";
}

static long rec_bytes(int prec) { return prec == LAPH_PREC_F32 ? 96 : 48; }

// the kernel indexes sites in 32 bits, reads neighbour records through 32-bit byte
// offsets and divides site indices by ns and ns / 2 with multiply-high reciprocals
static bool lds_fits(long Vh, int R, long rec, int ns)
{
    return Vh * R * 12 < (1L << 31) && Vh * R * rec < (1L << 32) &&
           (unsigned long long)Vh * (unsigned long long)ns < (1ull << 32);
}

int lds_max_rhs(laph_ctx *c, int prec)
{
    for (int R = 32; R >= 1; R /= 2)
        if (lds_fits(c->g.Vh, R, rec_bytes(prec), c->g.ns)) return R;
    return 0;
}

long lds_dag_blocks(laph_ctx *c, int prec, int R)
{
    const int S = lds_tile_sites(c, prec, R);
    return (c->g.Vh + S - 1) / S;
}

#ifndef LAPH_WALK_BY
#define LAPH_WALK_BY 6
#endif
#ifndef LAPH_WALK_BZ
#define LAPH_WALK_BZ 6
#endif
// y (k = 0) and z (k = 1) extent of the tiles of the LDS kernel's site walk: the largest
// divisor of ns not above LAPH_WALK_BY / LAPH_WALK_BZ (0: checkerboard order)
static int walk_tile(int ns, int k)
{
    const int lim = k == 0 ? LAPH_WALK_BY : LAPH_WALK_BZ;
    for (int d = lim; d >= 1; d--)
        if (ns % d == 0) return d;
    return 0;
}

// m = ceil(2^32 / d): umulhi(n, m) = floor(n / d) whenever n d < 2^32 (m d - 2^32 < d);
// 0 for d = 1
static unsigned umulhi_magic(long d)
{
    if (d <= 1) return 0;
    return (unsigned)(((1ull << 32) + (unsigned long long)d - 1) / (unsigned long long)d);
}
// every index n the kernel divides by d is below nmax: the reciprocal is exact when
static bool magic_ok(long d, long nmax) { return (unsigned long long)nmax * (unsigned long long)d < (1ull << 32); }

bool lds_walk_tiled(laph_ctx *c)
{
    const int ns = c->g.ns, nt = c->g.nt;
    const long Vh = c->g.Vh;
    const int by = walk_tile(ns, 0), bz = walk_tile(ns, 1);
    const long A = (long)(ns / 2) * by * bz;
    return c->walk_mode == 0 && by > 0 && bz > 0 && magic_ok(A, Vh) && magic_ok(nt, Vh) && magic_ok(ns, Vh);
}

template <class SP>
void launch_dslash_mr(laph_ctx *c, int mode, const MrArgs &a, hipStream_t st)
{
    LAPH_CHECK(lds_fits(a.Vh, a.R, sizeof(Spin12<SP>), a.ns), LAPH_EINVAL,
               "%d right-hand sides of %ld sites exceed the 32-bit indexing of the multi-RHS hopping kernel", a.R,
               a.Vh);
    LAPH_CHECK(a.R >= 1 && a.R <= 32 && (a.R & (a.R - 1)) == 0, LAPH_EINVAL, "block of %d right-hand sides", a.R);
    const int S = lds_tile_sites(c, prec_id<SP>(), a.R);
    LAPH_CHECK(S >= 1 && S * a.R <= 256, LAPH_EINVAL, "tile of %d sites x %d right-hand sides", S, a.R);
    MrArgs b = a;
    // the tiled walk's divisors (tile slice, nt, tile extent, tiles per row) need exact
    // reciprocals for every position below Vh; otherwise checkerboard order
    if (lds_walk_tiled(c)) {
        b.wby = walk_tile(a.ns, 0);
        b.wbz = walk_tile(a.ns, 1);
    } else {
        b.wby = b.wbz = 0;
    }
    const long A = (long)(a.ns / 2) * b.wby * b.wbz;
    b.m_nsh = umulhi_magic(a.ns / 2);
    b.m_ns = umulhi_magic(a.ns);
    b.m_nt = umulhi_magic(a.nt);
    b.m_by = b.wby ? umulhi_magic(b.wby) : 0;
    b.m_nty = b.wby ? umulhi_magic(a.ns / b.wby) : 0;
    b.m_A = b.wby ? umulhi_magic(A) : 0;
    b.unit = 1.0f;
    b.tgauge = a.tgauge;
    dim3 grid(nblocks_for(a.Vh, S)), block(S * a.R);
    hipEvent_t e0, e1;
    timing_begin(c, &e0, &e1);
    const bool hx = a.x != nullptr;
    LAPH_CHECK(hx || (mode != M_INV_AFTER_DAG && mode != M_PLAIN_CG && mode != M_INV_AFTER_DOT), LAPH_EINVAL,
               "fused hopping epilogues need the own-site operand");
    LAPH_CHECK(mode != M_INV_AFTER_DOT || (a.dot_y && a.partial), LAPH_EINVAL, "the dot epilogue needs y");
    if (mode == M_INV_AFTER_DOT)
        hipLaunchKernelGGL((k_dslash_lds<SP, M_INV_AFTER_DOT, true>), grid, block, lds_bytes(S), st, b);
    else if (mode == M_INV_AFTER_DAG)
        hipLaunchKernelGGL((k_dslash_lds<SP, M_INV_AFTER_DAG, true>), grid, block, lds_bytes(S), st, b);
    else if (mode == M_PLAIN_CG)
        hipLaunchKernelGGL((k_dslash_lds<SP, M_PLAIN_CG, true>), grid, block, lds_bytes(S), st, b);
    else if (mode == M_INV_AFTER && hx)
        hipLaunchKernelGGL((k_dslash_lds<SP, M_INV_AFTER, true>), grid, block, lds_bytes(S), st, b);
    else if (mode == M_INV_AFTER)
        hipLaunchKernelGGL((k_dslash_lds<SP, M_INV_AFTER, false>), grid, block, lds_bytes(S), st, b);
    else if (hx)
        hipLaunchKernelGGL((k_dslash_lds<SP, M_PLAIN, true>), grid, block, lds_bytes(S), st, b);
    else
        hipLaunchKernelGGL((k_dslash_lds<SP, M_PLAIN, false>), grid, block, lds_bytes(S), st, b);
    LAPH_HIP(hipGetLastError());
    if (e0)
        timing_end(c, e0, e1,
                   dslash_mr_bytes(a.Vh, a.R, SP::bytes, SP::kNorm, mode, a.x != nullptr,
                                   mode == M_INV_AFTER_DOT && a.dot_y == a.x),
                   timing_label("dslash_lds", prec_name<SP>(), mode, a.R));
}

template <class SP>
void launch_clover_mr(laph_ctx *c, const void *cl, const void *x, const float *x_nrm, void *out, float *out_nrm,
                      long Vh, int R, int g5_in, hipStream_t st)
{
    (void)c;
    long n = Vh * R;
    hipLaunchKernelGGL((k_clover_mr<SP, 1>), dim3(nblocks_for(n, 256)), dim3(256), 0, st, (const float4 *)cl,
                       (const typename SP::E *)x, x_nrm, (typename SP::E *)out, out_nrm, Vh, R, g5_in);
    LAPH_HIP(hipGetLastError());
}

void build_lp_operator(laph_ctx *c, const double2 *g64, const double *clinv64, float4 *links12, float *clinv_aos)
{
    long Vh = c->g.Vh;
    hipLaunchKernelGGL(k_links12, dim3(nblocks_for(8 * Vh, 256)), dim3(256), 0, c->stream, g64, links12, Vh);
    hipLaunchKernelGGL(k_clover_aos, dim3(nblocks_for(2 * Vh, 256)), dim3(256), 0, c->stream, clinv64, clinv_aos, Vh);
    LAPH_HIP(hipGetLastError());
}

template void launch_dslash_mr<S32>(laph_ctx *, int, const MrArgs &, hipStream_t);
template void launch_dslash_mr<S16>(laph_ctx *, int, const MrArgs &, hipStream_t);
template void launch_dslash_mr<SB16>(laph_ctx *, int, const MrArgs &, hipStream_t);
template void launch_clover_mr<S32>(laph_ctx *, const void *, const void *, const float *, void *, float *, long, int,
                                    int, hipStream_t);
template void launch_clover_mr<S16>(laph_ctx *, const void *, const void *, const float *, void *, float *, long, int,
                                    int, hipStream_t);
template void launch_clover_mr<SB16>(laph_ctx *, const void *, const void *, const float *, void *, float *, long, int,
                                     int, hipStream_t);

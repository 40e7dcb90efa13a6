// Even-odd anisotropic Wilson-clover hopping kernel with fused clover epilogues.
#include "spinor_io.h"

namespace {

template <typename A>
struct Spin {
    Cx<A> v[4][3];
};

template <typename A>
__device__ __forceinline__ void mat_vec(const Cx<A> (&U)[9], const Cx<A> (&h)[3], Cx<A> (&o)[3])
{
#pragma unroll
    for (int a = 0; a < 3; a++) o[a] = U[a * 3] * h[0] + U[a * 3 + 1] * h[1] + U[a * 3 + 2] * h[2];
}
template <typename A>
__device__ __forceinline__ void mat_dag_vec(const Cx<A> (&U)[9], const Cx<A> (&h)[3], Cx<A> (&o)[3])
{
#pragma unroll
    for (int a = 0; a < 3; a++) o[a] = conjmul(U[a], h[0]) + conjmul(U[3 + a], h[1]) + conjmul(U[6 + a], h[2]);
}

// Element e of a field stored as planes of Vh (links, clover) or Vh R (spinors) entries:
// plane + e.  With O32 (the launcher checks that every plane is below 4 GiB) the plane
// start stays a uniform (scalar) address and each lane adds one 32-bit byte offset, so a
// neighbour spinor costs one address register instead of twelve 64-bit pairs.
template <bool O32, typename T>
__device__ __forceinline__ const T &elem(const T *plane, long e)
{
    if constexpr (O32)
        return *(const T *)((const char *)plane + ((unsigned)e * (unsigned)sizeof(T)));
    else
        return plane[e];
}
template <bool O32, typename T>
__device__ __forceinline__ T &elem(T *plane, long e)
{
    if constexpr (O32)
        return *(T *)((char *)plane + ((unsigned)e * (unsigned)sizeof(T)));
    else
        return plane[e];
}

template <class GP, typename A, bool O32>
__device__ __forceinline__ void load_link(const typename GP::E *g, int mu, int par, long Vh, long i, Cx<A> (&U)[9])
{
    const typename GP::E *p = g + (long)(mu * 2 + par) * 9 * Vh;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        const auto v = elem<O32>(p + (long)k * Vh, i);
        U[k] = {(A)v.x, (A)v.y};
    }
}

template <class SP, bool O32>
__device__ __forceinline__ void load_spinor(const typename SP::E *s, const float *nrm, long Vh, int R, long i, int r,
                                            Spin<typename SP::A> &out)
{
    Cx<typename SP::A> v[12];
    if constexpr (O32) {
        static_assert(std::is_same<SP, S64>::value, "32-bit offsets: FP64 plane layout only");
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const double2 e = elem<true>(s + (long)k * Vh * R, i * R + r);
            v[k] = {e.x, e.y};
        }
    } else {
        ld_spinor12<SP, typename SP::A>(s, nrm, Vh, R, i, r, v);
    }
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) out.v[a][c] = v[a * 3 + c];
}

template <class SP, bool O32>
__device__ __forceinline__ void store_spinor(typename SP::E *s, float *nrm, long Vh, int R, long i, int r,
                                             const Spin<typename SP::A> &in)
{
    Cx<typename SP::A> v[12];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) v[a * 3 + c] = in.v[a][c];
    if constexpr (O32) {
        static_assert(std::is_same<SP, S64>::value, "32-bit offsets: FP64 plane layout only");
#pragma unroll
        for (int k = 0; k < 12; k++) elem<true>(s + (long)k * Vh * R, i * R + r) = make_double2(v[k].re, v[k].im);
    } else {
        st_spinor12<SP, typename SP::A>(s, nrm, Vh, R, i, r, v);
    }
}

// packed Hermitian 6x6 block times a 6-vector
template <class CP, typename A, bool O32 = false>
__device__ __forceinline__ void herm6(const typename CP::E *cl, long Vh, long i, const Cx<A> (&v)[6], Cx<A> (&o)[6])
{
    A d[6];
#pragma unroll
    for (int k = 0; k < 6; k++) d[k] = (A)elem<O32>(cl + (long)k * Vh, i);
#pragma unroll
    for (int k = 0; k < 6; k++) o[k] = d[k] * v[k];
    int e = 6;
#pragma unroll
    for (int r = 1; r < 6; r++)
#pragma unroll
        for (int c = 0; c < r; c++) {
            Cx<A> L = {(A)elem<O32>(cl + (long)e * Vh, i), (A)elem<O32>(cl + (long)(e + 1) * Vh, i)};
            e += 2;
            o[r] = o[r] + L * v[c];
            o[c] = o[c] + conjmul(L, v[r]);
        }
}

template <class CP, typename A, bool O32 = false>
__device__ __forceinline__ void clover_mul(const typename CP::E *cl, long Vh, long i, const Spin<A> &in, Spin<A> &out)
{
#pragma unroll
    for (int blk = 0; blk < 2; blk++) {
        Cx<A> v[6], o[6];
#pragma unroll
        for (int s = 0; s < 2; s++)
#pragma unroll
            for (int c = 0; c < 3; c++) v[s * 3 + c] = in.v[blk * 2 + s][c];
        herm6<CP, A, O32>(cl + (long)blk * 36 * Vh, Vh, i, v, o);
#pragma unroll
        for (int s = 0; s < 2; s++)
#pragma unroll
            for (int c = 0; c < 3; c++) out.v[blk * 2 + s][c] = o[s * 3 + c];
    }
}

template <typename A>
__device__ __forceinline__ void acc_upper(Spin<A> &acc, const Cx<A> (&w0)[3], const Cx<A> (&w1)[3])
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        acc.v[0][c] = acc.v[0][c] + w0[c];
        acc.v[1][c] = acc.v[1][c] + w1[c];
    }
}

// Rolled FP64 hops: one loop trip per direction d = 2 mu + (backward), the spin structure
// of (1 -/+ gamma_mu) taken from per-direction unit coefficients, so that only one
// direction's neighbour and link are live at a time (150 instead of ~290 registers: three
// waves per SIMD instead of one for this latency-bound kernel).
// h0 = w s0 + a0 s_p0, h1 = w s1 + a1 s_p1 (p0, p1) = (3, 2) for mu < 2, else (2, 3);
// acc0 += o0, acc1 += o1, acc2 += b2 o_q2, acc3 += b3 o_q3 with (q2, q3) = (1, 0) for
// mu < 2, else (0, 1); forward units below (the gamma matrices of the chiral basis),
// backward hops negate them and take U_mu(x - mu)^dag.
struct HopCoef {
    double a0r, a0i, a1r, a1i, b2r, b2i, b3r, b3i;
};
__device__ __forceinline__ Cx<double> unit_mul(double ur, double ui, Cx<double> z)
{
    return {ur * z.re - ui * z.im, ur * z.im + ui * z.re};
}

template <bool O32>
__device__ __forceinline__ void hop_rolled(const DslashArgs &P, long i, int r, int x, int y, int z, int t,
                                           Spin<double> &acc)
{
    constexpr HopCoef kc[4] = {{0, 1, 0, 1, 0, -1, 0, -1},
                               {1, 0, -1, 0, -1, 0, 1, 0},
                               {0, 1, 0, -1, 0, -1, 0, 1},
                               {-1, 0, -1, 0, -1, 0, -1, 0}};
    const int R = P.R, ns = P.ns, nt = P.nt, par = P.par;
    const long Vh = P.Vh;
    const double2 *in = (const double2 *)P.in;
    const double2 *g = (const double2 *)P.gauge;
#pragma unroll 1
    for (int d = 0; d < 8; d++) {
        const int mu = d >> 1;
        const bool fwd = !(d & 1);
        const int st = fwd ? 1 : -1;
        int xx = x, yy = y, zz = z, tt = t;
        double w = mu == 3 ? P.wt : P.ws;
        if (mu == 0) xx = (x + st + ns) % ns;
        if (mu == 1) yy = (y + st + ns) % ns;
        if (mu == 2) zz = (z + st + ns) % ns;
        if (mu == 3) {
            tt = (t + st + nt) % nt;
            if (fwd ? t + 1 == nt : t == 0) w *= P.bct;
        }
        const long nb = lex_index(xx, yy, zz, tt, ns) >> 1;
        Spin<double> s;
        load_spinor<S64, O32>(in, nullptr, Vh, R, nb, r, s);
        // U_mu(x), or for the backward hop U_mu(x - mu)^dag: planes read transposed, conjugated
        const double2 *gp = g + (long)(mu * 2 + (fwd ? par : par ^ 1)) * 9 * Vh;
        const long li = fwd ? i : nb;
        const double cj = fwd ? 1.0 : -1.0;
        Cx<double> U[9];
#pragma unroll
        for (int k = 0; k < 9; k++) {
            const double2 v = elem<O32>(gp + (long)(fwd ? k : (k % 3) * 3 + k / 3) * Vh, li);
            U[k] = {v.x, cj * v.y};
        }
        const HopCoef &q = kc[mu];
        const double sa = fwd ? w : -w, sb = fwd ? 1.0 : -1.0;
        const bool sw = mu < 2;
        Cx<double> h0[3], h1[3], o0[3], o1[3];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            h0[c] = w * s.v[0][c] + unit_mul(sa * q.a0r, sa * q.a0i, sw ? s.v[3][c] : s.v[2][c]);
            h1[c] = w * s.v[1][c] + unit_mul(sa * q.a1r, sa * q.a1i, sw ? s.v[2][c] : s.v[3][c]);
        }
        mat_vec(U, h0, o0);
        mat_vec(U, h1, o1);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            acc.v[0][c] = acc.v[0][c] + o0[c];
            acc.v[1][c] = acc.v[1][c] + o1[c];
            acc.v[2][c] = acc.v[2][c] + unit_mul(sb * q.b2r, sb * q.b2i, sw ? o1[c] : o0[c]);
            acc.v[3][c] = acc.v[3][c] + unit_mul(sb * q.b3r, sb * q.b3i, sw ? o0[c] : o1[c]);
        }
    }
}

// checkerboard index and coordinates of position pos of the tiled site walk: tiles of
// Ns x by x bz sites (x halved by the parity), one after the other, each visited slice by
// slice through all Nt slices; the time neighbours of a tile slice are the tile slices just
// before and after it in the walk, so that with many right-hand sides per site they are
// still in L2 (in checkerboard order they are Ns^3 / 2 sites away)
__device__ __forceinline__ long walk_coords(unsigned pos, int ns, int nt, int par, int by, int bz, int &x, int &y,
                                            int &z, int &t)
{
    const unsigned nsh = (unsigned)ns >> 1, A = nsh * by * bz;
    const unsigned q = pos / A, loc = pos - q * A;
    const unsigned tile = q / (unsigned)nt;
    t = (int)(q - tile * nt);
    const unsigned q1 = loc / nsh, xh = loc - q1 * nsh;
    const unsigned zz = q1 / (unsigned)by, yy = q1 - zz * by;
    const unsigned nty = (unsigned)ns / by, tz = tile / nty, ty = tile - tz * nty;
    y = (int)(ty * by + yy);
    z = (int)(tz * bz + zz);
    x = 2 * (int)xh + ((y + z + t + par) & 1);
    return (long)xh + (long)nsh * (y + (long)ns * (z + (long)ns * t));
}

template <class SP, class GP, class CP, int MODE, bool O32>
__global__ __launch_bounds__(256) void k_dslash(const DslashArgs P)
{
    using A = typename SP::A;
    unsigned b = xcd_block(blockIdx.x, gridDim.x);
    long tid = (long)b * blockDim.x + threadIdx.x;
    const int R = P.R;
    const long Vh = P.Vh;
    if (tid >= Vh * R) return;
    // 32-bit lane arithmetic: the launcher guarantees Vh R < 2^28
    const unsigned pos = (unsigned)tid / (unsigned)R;
    const int r = (int)((unsigned)tid - pos * (unsigned)R);
    const int ns = P.ns, nt = P.nt, par = P.par, opar = par ^ 1;
    int x, y, z, t;
    long i;
    if (P.wby) {
        i = walk_coords(pos, ns, nt, par, P.wby, P.wbz, x, y, z, t);
    } else {
        i = pos;
        cb_coords(i, par, ns, x, y, z, t);
    }
    const auto *in = (const typename SP::E *)P.in;
    const auto *g = (const typename GP::E *)P.gauge;

    Spin<A> acc;
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) acc.v[a][c] = {(A)0, (A)0};

    hop_rolled<O32>(P, i, r, x, y, z, t, acc);

    if (P.g5d) {
#pragma unroll
        for (int c = 0; c < 3; c++) {
            acc.v[2][c] = cneg(acc.v[2][c]);
            acc.v[3][c] = cneg(acc.v[3][c]);
        }
    }

    const A ca = (A)P.a, cc = (A)P.c;
    const auto *cl = (const typename CP::E *)P.clov;
    Spin<A> res;
    if constexpr (MODE == M_PLAIN) {
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int c = 0; c < 3; c++) res.v[a][c] = cc * acc.v[a][c];
        if (P.x) {
            Spin<A> xv;
            load_spinor<SP, O32>((const typename SP::E *)P.x, P.x_nrm, Vh, R, i, r, xv);
#pragma unroll
            for (int a = 0; a < 4; a++)
#pragma unroll
                for (int c = 0; c < 3; c++) res.v[a][c] = res.v[a][c] + ca * xv.v[a][c];
        }
    } else if constexpr (MODE == M_INV_AFTER) {
        Spin<A> m;
        clover_mul<CP, A, O32>(cl, Vh, i, acc, m);
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int c = 0; c < 3; c++) res.v[a][c] = cc * m.v[a][c];
        if (P.x) {
            Spin<A> xv;
            load_spinor<SP, O32>((const typename SP::E *)P.x, P.x_nrm, Vh, R, i, r, xv);
#pragma unroll
            for (int a = 0; a < 4; a++)
#pragma unroll
                for (int c = 0; c < 3; c++) res.v[a][c] = res.v[a][c] + ca * xv.v[a][c];
        }
    } else if constexpr (MODE == M_INV_OF_SUM) {
        Spin<A> xv, sum;
        load_spinor<SP, O32>((const typename SP::E *)P.x, P.x_nrm, Vh, R, i, r, xv);
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int c = 0; c < 3; c++) sum.v[a][c] = ca * xv.v[a][c] + cc * acc.v[a][c];
        clover_mul<CP, A, O32>(cl, Vh, i, sum, res);
    } else {  // M_CLOV_ADD
        Spin<A> xv, m;
        load_spinor<SP, O32>((const typename SP::E *)P.x, P.x_nrm, Vh, R, i, r, xv);
        clover_mul<CP, A, O32>(cl, Vh, i, xv, m);
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int c = 0; c < 3; c++) res.v[a][c] = m.v[a][c] + cc * acc.v[a][c];
    }
    store_spinor<SP, O32>((typename SP::E *)P.out, P.out_nrm, Vh, R, i, r, res);
}

template <class SP, class CP>
__global__ __launch_bounds__(256) void k_clover_apply(const typename CP::E *__restrict__ cl,
                                                       const typename SP::E *__restrict__ x, const float *x_nrm,
                                                       typename SP::E *__restrict__ out, float *out_nrm, long Vh,
                                                       int R, int g5_in)
{
    using A = typename SP::A;
    long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (tid >= Vh * R) return;
    long i = tid / R;
    int r = (int)(tid - i * R);
    Spin<A> v, o;
    load_spinor<SP, false>(x, x_nrm, Vh, R, i, r, v);
    if (g5_in) {
#pragma unroll
        for (int c = 0; c < 3; c++) {
            v.v[2][c] = cneg(v.v[2][c]);
            v.v[3][c] = cneg(v.v[3][c]);
        }
    }
    clover_mul<CP, A>(cl, Vh, i, v, o);
    store_spinor<SP, false>(out, out_nrm, Vh, R, i, r, o);
}

}  // namespace

double dslash_bytes(long Vh, int R, int gbytes, int cbytes, int sbytes, bool has_norm, int mode, bool has_x)
{
    // algorithmic bytes: 8 links, the clover block set if used, one input spinor per
    // site (neighbour re-reads are cache traffic), the output and the epilogue operand
    double site = 8.0 * 9 * gbytes;
    if (mode != M_PLAIN) site += 72.0 * cbytes;
    double per_rhs = 12.0 * sbytes * (2 + (has_x ? 1 : 0)) + (has_norm ? 4.0 * (2 + (has_x ? 1 : 0)) : 0.0);
    return (double)Vh * (site + R * per_rhs);
}

template <class SP, class GP, class CP, bool O32>
void launch_modes(int mode, dim3 grid, dim3 block, hipStream_t st, const DslashArgs &a)
{
    switch (mode) {
    case M_PLAIN: hipLaunchKernelGGL((k_dslash<SP, GP, CP, M_PLAIN, O32>), grid, block, 0, st, a); break;
    case M_INV_AFTER: hipLaunchKernelGGL((k_dslash<SP, GP, CP, M_INV_AFTER, O32>), grid, block, 0, st, a); break;
    case M_INV_OF_SUM: hipLaunchKernelGGL((k_dslash<SP, GP, CP, M_INV_OF_SUM, O32>), grid, block, 0, st, a); break;
    default: hipLaunchKernelGGL((k_dslash<SP, GP, CP, M_CLOV_ADD, O32>), grid, block, 0, st, a); break;
    }
}

template <class SP, class GP, class CP>
void launch_dslash(laph_ctx *c, int mode, const DslashArgs &a, hipStream_t st)
{
    long n = a.Vh * a.R;
    dim3 grid(nblocks_for(n, 256)), block(256);
    hipEvent_t e0, e1;
    timing_begin(c, &e0, &e1);
    // 32-bit lane offsets: every spinor plane (Vh R entries) stays below 4 GiB (the link
    // and clover planes are smaller); callers split larger batches
    LAPH_CHECK((unsigned long long)n * sizeof(double2) < (1ull << 32), LAPH_EINVAL,
               "%d FP64 fields of %ld sites exceed the hopping kernel's 32-bit offsets", a.R, a.Vh);
    // many right-hand sides per site: a site's records span R x 192 B, so the time
    // neighbours of checkerboard order (Ns^3 / 2 sites away) fall out of L2; walk tiles
    // through time instead (3 x 3 where Ns allows it, else 2 x 2)
    DslashArgs b = a;
    b.wby = b.wbz = 0;
    if (a.R >= 8) b.wby = b.wbz = (a.ns % 3 == 0) ? 3 : 2;
    launch_modes<SP, GP, CP, true>(mode, grid, block, st, b);
    LAPH_HIP(hipGetLastError());
    bool has_x = a.x != nullptr && (mode != M_PLAIN || a.x);
    if (e0)
        timing_end(c, e0, e1, dslash_bytes(a.Vh, a.R, GP::bytes, CP::bytes, SP::bytes, SP::kNorm, mode, has_x),
                   timing_label("dslash", SP::bytes == 16 ? "f64" : "f32", mode, a.R));
}

template <class SP, class CP>
void launch_clover_apply(laph_ctx *c, const void *clov, const void *x, const float *x_nrm, void *out, float *out_nrm,
                         long Vh, int R, int g5_in, hipStream_t st)
{
    long n = Vh * R;
    hipLaunchKernelGGL((k_clover_apply<SP, CP>), dim3(nblocks_for(n, 256)), dim3(256), 0, st,
                       (const typename CP::E *)clov, (const typename SP::E *)x, x_nrm, (typename SP::E *)out,
                       out_nrm, Vh, R, g5_in);
    LAPH_HIP(hipGetLastError());
}

template void launch_dslash<S64, G64, C64>(laph_ctx *, int, const DslashArgs &, hipStream_t);
template void launch_clover_apply<S64, C64>(laph_ctx *, const void *, const void *, const float *, void *, float *,
                                            long, int, int, hipStream_t);

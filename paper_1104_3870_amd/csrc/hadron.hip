// Hadron building blocks in LapH space (Sec. II: quark sources and sinks, the gamma_5-
// Hermitian estimate; Sec. III.B: meson functions and the meson correlator).
//
// With the trivial displacement and zero momentum every quark source varrho = V_s c and
// every LapH-smeared quark sink varphi = V_s V_s^dag X = V_s c is a linear combination of
// the LapH eigenvectors, so the sums over sites and colours of a meson function reduce to
// the LapH index (V_s^dag V_s = 1 on every slice): the functions are batched complex
// products of coefficient arrays coef[r][t][alpha][n] (the layout of sink_project).
#include <cmath>

#include "laph_impl.h"

namespace {

constexpr int kMT = 16;   // meson-function tile: kMT x kMT (i, j) per block
// LapH indices per LDS stage (all four spins of each: 4 kMN K values); each lane stages
// one (row, n) of A and one of B, with c applied to B's four spins on the way, so that
// every coefficient is read once per tile (staging K in spin-major order read each B value
// four times: 46 us for 32 x 32 lines on 128 slices at N_v = 112, now 31 us)
constexpr int kMN = 16;
constexpr int kMQ = 2 * kMT * kMN / (kMT * kMT);  // (row, n) items per lane
static_assert(kMQ * kMT * kMT == 2 * kMT * kMN && kMQ % 2 == 0, "whole items per lane, A and B alike");

__device__ __forceinline__ double2 cmadd_conj(double2 acc, double2 a, double2 b)  // acc + conj(a) b
{
    acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(-a.y, b.x, acc.y));
    return acc;
}

struct Spin4 {
    double2 m[16];  // row-major 4x4 complex
};

// out[r][t][alpha][n] = sum_beta S[alpha][beta] in[r][t][beta][n]; one lane per (r, t, n)
__global__ void k_spin_apply(Spin4 S, const double2 *__restrict__ in, double2 *__restrict__ out, long nrt, int nv)
{
    long q = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (q >= nrt * nv) return;
    long rt = q / nv;
    int n = (int)(q - rt * nv);
    double2 v[4];
#pragma unroll
    for (int b = 0; b < 4; b++) v[b] = in[(rt * 4 + b) * nv + n];
#pragma unroll
    for (int a = 0; a < 4; a++) {
        double2 s = make_double2(0.0, 0.0);
#pragma unroll
        for (int b = 0; b < 4; b++) s = cadd(s, cmul(S.m[a * 4 + b], v[b]));
        out[(rt * 4 + a) * nv + n] = s;
    }
}

// M[t][i][j] = sum_{alpha, n} conj(a[i][t][alpha][n]) (c b_j)[t][alpha][n],
// (c b)[alpha] = sum_beta c[alpha][beta] b[beta]: per slice the product A^dag (c B) over
// K = 4 nv.  Block = one slice t and a kMT x kMT tile of (i, j); both operands staged in
// LDS kMN LapH indices (4 kMN K values) at a time, c applied while B is staged.
__global__ __launch_bounds__(kMT *kMT) void k_meson(Spin4 c, const double2 *__restrict__ a, int n1,
                                                    const double2 *__restrict__ b, int n2, int nt, int nv,
                                                    double2 *__restrict__ out)
{
    __shared__ double2 sa[4 * kMN][kMT + 1];
    __shared__ double2 sb[4 * kMN][kMT + 1];
    const int t = blockIdx.z;
    const int i0 = blockIdx.x * kMT, j0 = blockIdx.y * kMT;
    const int ti = threadIdx.x % kMT, tj = threadIdx.x / kMT;
    double2 acc = make_double2(0.0, 0.0);
    for (int n0 = 0; n0 < nv; n0 += kMN) {
        // item e of the stage (lane + 256 q): operand B (upper half) or A, row sr, LapH
        // offset dn; every load of the stage is issued before the LDS stores
        double2 v[kMQ][4];
#pragma unroll
        for (int q = 0; q < kMQ; q++) {
            const int e = threadIdx.x + q * kMT * kMT;
            const bool isb = e >= kMT * kMN;
            const int se = e - (isb ? kMT * kMN : 0), sr = se / kMN, n = n0 + se - sr * kMN;
            const bool rok = isb ? j0 + sr < n2 : i0 + sr < n1;
            const double2 *src = isb ? b + ((long)(j0 + sr) * nt + t) * 4 * nv : a + ((long)(i0 + sr) * nt + t) * 4 * nv;
#pragma unroll
            for (int c4 = 0; c4 < 4; c4++) v[q][c4] = make_double2(0.0, 0.0);
            if (rok && n < nv) {
#pragma unroll
                for (int c4 = 0; c4 < 4; c4++) v[q][c4] = src[(long)c4 * nv + n];
            }
        }
#pragma unroll
        for (int q = 0; q < kMQ; q++) {
            const int e = threadIdx.x + q * kMT * kMT;
            const bool isb = e >= kMT * kMN;
            const int se = e - (isb ? kMT * kMN : 0), sr = se / kMN, dn = se - sr * kMN;
            if (isb) {
#pragma unroll
                for (int al = 0; al < 4; al++) {
                    double2 cb = make_double2(0.0, 0.0);
#pragma unroll
                    for (int be = 0; be < 4; be++) cb = cadd(cb, cmul(c.m[al * 4 + be], v[q][be]));
                    sb[al * kMN + dn][sr] = cb;
                }
            } else {
#pragma unroll
                for (int al = 0; al < 4; al++) sa[al * kMN + dn][sr] = v[q][al];
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 4 * kMN; kk++) acc = cmadd_conj(acc, sa[kk][ti], sb[kk][tj]);
        __syncthreads();
    }
    const int i = i0 + ti, j = j0 + tj;
    if (i < n1 && j < n2) out[((long)t * n1 + i) * n2 + j] = acc;
}

// diagonal: M[t][i] = sum_{alpha, n} conj(a[i][t][alpha][n]) (c b_i)[t][alpha][n]; one
// block of 64 lanes per (i, t)
__global__ __launch_bounds__(64) void k_meson_diag(Spin4 c, const double2 *__restrict__ a,
                                                    const double2 *__restrict__ b, int nt, int nv,
                                                    double2 *__restrict__ out)
{
    const int i = blockIdx.x, t = blockIdx.y;
    const long base = ((long)i * nt + t) * 4 * nv;
    double2 acc = make_double2(0.0, 0.0);
    for (int n = threadIdx.x; n < nv; n += 64) {
        double2 bv[4];
#pragma unroll
        for (int be = 0; be < 4; be++) bv[be] = b[base + (long)be * nv + n];
#pragma unroll
        for (int al = 0; al < 4; al++) {
            double2 cb = make_double2(0.0, 0.0);
#pragma unroll
            for (int be = 0; be < 4; be++) cb = cadd(cb, cmul(c.m[al * 4 + be], bv[be]));
            acc = cmadd_conj(acc, a[base + (long)al * nv + n], cb);
        }
    }
    __shared__ double2 red[64];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 32; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(long)t * gridDim.x + i] = red[0];
}

// connected meson correlator for every sink slice tF (one block per tF):
//   C[tF] = - sum_{i,j} Msnk[tF][i][j] conj(Msrc[t0][i][j])
__global__ __launch_bounds__(256) void k_corr_conn(const double2 *__restrict__ snk, const double2 *__restrict__ src,
                                                   long nij, int t0, double2 *__restrict__ out)
{
    const int tf = blockIdx.x;
    double2 acc = make_double2(0.0, 0.0);
    for (long q = threadIdx.x; q < nij; q += 256)
        acc = cmadd_conj(acc, src[(long)t0 * nij + q], snk[(long)tf * nij + q]);
    __shared__ double2 red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[tf] = make_double2(-red[0].x, -red[0].y);
}

// disconnected (internal-line) term: C[tF] = (sum_i Dsnk[tF][i]) conj(sum_i Dsrc[t0][i])
__global__ __launch_bounds__(256) void k_corr_disc(const double2 *__restrict__ snk, const double2 *__restrict__ src,
                                                   int n, int t0, double2 *__restrict__ out)
{
    const int tf = blockIdx.x;
    double2 as = make_double2(0.0, 0.0), ad = make_double2(0.0, 0.0);
    for (int q = threadIdx.x; q < n; q += 256) {
        as = cadd(as, snk[(long)tf * n + q]);
        ad = cadd(ad, src[(long)t0 * n + q]);
    }
    __shared__ double2 r1[256], r2[256];
    r1[threadIdx.x] = as;
    r2[threadIdx.x] = ad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            r1[threadIdx.x] = cadd(r1[threadIdx.x], r1[threadIdx.x + s]);
            r2[threadIdx.x] = cadd(r2[threadIdx.x], r2[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[tf] = cconjmul(r2[0], r1[0]);
}

Spin4 spin4(const double *h)
{
    Spin4 s;
    for (int k = 0; k < 16; k++) {
        LAPH_CHECK(std::isfinite(h[2 * k]) && std::isfinite(h[2 * k + 1]), LAPH_EINVAL, "spin matrix not finite");
        s.m[k] = make_double2(h[2 * k], h[2 * k + 1]);
    }
    return s;
}

}  // namespace

extern "C" int laph_spin_apply(laph_ctx_t c, const double *S, const double *in, int n, int nv, double *out)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(S && in && out && n > 0 && nv > 0, LAPH_EINVAL, "bad arguments");
    const long nrt = (long)n * c->g.nt;
    hipLaunchKernelGGL(k_spin_apply, dim3(nblocks_for(nrt * nv, 256)), dim3(256), 0, c->stream, spin4(S),
                       (const double2 *)in, (double2 *)out, nrt, nv);
    LAPH_HIP(hipGetLastError());
    LAPH_API_END(c)
}

extern "C" int laph_meson_function(laph_ctx_t c, const double *cs, const double *a, int n1, const double *b, int n2,
                                   int nv, int diag, double *out)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(cs && a && b && out && n1 > 0 && n2 > 0 && nv > 0, LAPH_EINVAL, "bad arguments");
    LAPH_CHECK(!diag || n1 == n2, LAPH_EINVAL, "diag needs n1 == n2");
    const int nt = c->g.nt;
    const Spin4 s = spin4(cs);
    // with per-kernel timing on, HIP events on the library's stream around the launch
    // (algorithmic bytes: both coefficient arrays in, the function out)
    hipEvent_t e0, e1;
    timing_begin(c, &e0, &e1);
    if (diag) {
        LAPH_CHECK(n1 <= 65535 && nt <= 65535, LAPH_EINVAL, "too many fields for one launch");
        hipLaunchKernelGGL(k_meson_diag, dim3(n1, nt), dim3(64), 0, c->stream, s, (const double2 *)a,
                           (const double2 *)b, nt, nv, (double2 *)out);
    } else {
        const unsigned gi = (n1 + kMT - 1) / kMT, gj = (n2 + kMT - 1) / kMT;
        LAPH_CHECK(gj <= 65535 && nt <= 65535, LAPH_EINVAL, "too many fields for one launch");
        hipLaunchKernelGGL(k_meson, dim3(gi, gj, nt), dim3(kMT * kMT), 0, c->stream, s, (const double2 *)a, n1,
                           (const double2 *)b, n2, nt, nv, (double2 *)out);
    }
    LAPH_HIP(hipGetLastError());
    if (e0)
        timing_end(c, e0, e1, 16.0 * ((double)(n1 + n2) * nt * 4 * nv + (double)nt * n1 * (diag ? 1 : n2)),
                   diag ? "meson_function_diag" : "meson_function");
    LAPH_API_END(c)
}

extern "C" int laph_meson_correlator(laph_ctx_t c, const double *snk, const double *src, int n1, int n2, int diag,
                                     int t0, double *out)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(snk && src && out && n1 > 0 && n2 > 0, LAPH_EINVAL, "bad arguments");
    LAPH_CHECK(t0 >= 0 && t0 < c->g.nt, LAPH_EINVAL, "t0 out of range");
    LAPH_CHECK(!diag || n1 == n2, LAPH_EINVAL, "diag needs n1 == n2");
    if (diag)
        hipLaunchKernelGGL(k_corr_disc, dim3(c->g.nt), dim3(256), 0, c->stream, (const double2 *)snk,
                           (const double2 *)src, n1, t0, (double2 *)out);
    else
        hipLaunchKernelGGL(k_corr_conn, dim3(c->g.nt), dim3(256), 0, c->stream, (const double2 *)snk,
                           (const double2 *)src, (long)n1 * n2, t0, (double2 *)out);
    LAPH_HIP(hipGetLastError());
    LAPH_API_END(c)
}

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
constexpr int kMK = 16;   // K (spin x LapH index) staged per LDS step

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
// LDS kMK K-values at a time, c applied while B is staged.
__global__ __launch_bounds__(kMT *kMT) void k_meson(Spin4 c, const double2 *__restrict__ a, int n1,
                                                    const double2 *__restrict__ b, int n2, int nt, int nv,
                                                    double2 *__restrict__ out)
{
    __shared__ double2 sa[kMK][kMT + 1];
    __shared__ double2 sb[kMK][kMT + 1];
    const int t = blockIdx.z;
    const int i0 = blockIdx.x * kMT, j0 = blockIdx.y * kMT;
    const int ti = threadIdx.x % kMT, tj = threadIdx.x / kMT;
    const int K = 4 * nv;
    double2 acc = make_double2(0.0, 0.0);
    for (int k0 = 0; k0 < K; k0 += kMK) {
        // stage: consecutive lanes take consecutive K of one row (rows i0 + sr of A, j0 + sr of B)
        {
            const int sk = threadIdx.x % kMK, sr = threadIdx.x / kMK;
            const int k = k0 + sk;
            double2 va = make_double2(0.0, 0.0), vb = make_double2(0.0, 0.0);
            if (k < K) {
                const int al = k / nv, n = k - (k / nv) * nv;
                const int i = i0 + sr, j = j0 + sr;
                if (i < n1) va = a[(((long)i * nt + t) * 4 + al) * nv + n];
                if (j < n2) {
                    const double2 *bj = b + ((long)j * nt + t) * 4 * nv + n;
#pragma unroll
                    for (int be = 0; be < 4; be++) vb = cadd(vb, cmul(c.m[al * 4 + be], bj[(long)be * nv]));
                }
            }
            sa[sk][sr] = va;
            sb[sk][sr] = vb;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kMK; kk++) acc = cmadd_conj(acc, sa[kk][ti], sb[kk][tj]);
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

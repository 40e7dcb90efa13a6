// Z4 noise, diluted LapH sources and the sink projection V_s^dag X (Sec. II, Sec. IV).
#include "laph_impl.h"

namespace {

// Philox4x32-10 (Salmon et al., SC'11): ten rounds, Weyl key schedule.
__device__ __forceinline__ uint4 philox10(uint4 c, uint2 k)
{
#pragma unroll
    for (int r = 0; r < 10; r++) {
        uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
        k.x += 0x9E3779B9u;
        k.y += 0xBB67AE85u;
    }
    return c;
}

__global__ void k_z4(uint32_t key0, int nt, int nv, double2 *rho)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    long n = (long)nt * 4 * nv;
    if (i >= n) return;
    int e = (int)(i % nv);
    int a = (int)((i / nv) % 4);
    int t = (int)(i / (4L * nv));
    uint4 w = philox10(make_uint4((uint32_t)e, (uint32_t)a, (uint32_t)t, 0u), make_uint2(key0, 0x4C415048u));
    switch (w.x & 3u) {
    case 0: rho[i] = make_double2(1, 0); break;
    case 1: rho[i] = make_double2(0, 1); break;
    case 2: rho[i] = make_double2(-1, 0); break;
    default: rho[i] = make_double2(0, -1); break;
    }
}

struct Dil {
    int type[3], J[3], cnt[3], N[3];
};

__device__ __forceinline__ bool member(const Dil &d, int k, int i, int b)
{
    switch (d.type[k]) {
    case LAPH_DIL_NONE: return b == 0;
    case LAPH_DIL_FULL: return i == b;
    case LAPH_DIL_BLOCK: return (int)(((long)d.J[k] * i) / d.N[k]) == b;
    default: return i % d.J[k] == b;
    }
}

// eta_j(x, t, c, alpha) = sum_{n in L(b_L)} V_{t,n}(x, c) rho(t, alpha, n), j = 0..nsrc-1
__global__ void k_source(const double2 *__restrict__ evecs, const double2 *__restrict__ rho, Dil d, long b_first,
                         int nsrc, long V3, int nt, int nv, double2 *__restrict__ eta)
{
    long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
    long per = V3 * nt * 3;
    if (tid >= per * nsrc) return;
    int j = (int)(tid / per);
    long rem = tid - (long)j * per;
    int c = (int)(rem % 3);
    long s = rem / 3;
    int t = (int)(s / V3);
    long xyz = s - (long)t * V3;
    long b = b_first + j;
    int bL = (int)(b % d.cnt[2]);
    int bS = (int)((b / d.cnt[2]) % d.cnt[1]);
    int bT = (int)(b / ((long)d.cnt[2] * d.cnt[1]));
    double2 *out = eta + ((long)j * V3 * nt + s) * 12;
    double2 acc[4] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
    if (member(d, 0, t, bT)) {
        for (int n = 0; n < nv; n++) {
            if (!member(d, 2, n, bL)) continue;
            double2 v = evecs[(((long)t * nv + n) * V3 + xyz) * 3 + c];
            for (int a = 0; a < 4; a++)
                if (member(d, 1, a, bS)) acc[a] = cadd(acc[a], cmul(v, rho[((long)t * 4 + a) * nv + n]));
        }
    }
    for (int a = 0; a < 4; a++) out[a * 3 + c] = acc[a];
}

// coef[r][t][alpha][n] for a tile of NT eigenvectors: one block per (t, tile, r)
constexpr int NT = 8;
__global__ __launch_bounds__(256) void k_sink(const double2 *__restrict__ evecs, const double2 *__restrict__ X,
                                              long V3, int nt, int nv, double2 *__restrict__ coef)
{
    int t = blockIdx.x;
    int n0 = blockIdx.y * NT;
    int r = blockIdx.z;
    double acc[NT][4][2];
#pragma unroll
    for (int q = 0; q < NT; q++)
#pragma unroll
        for (int a = 0; a < 4; a++) acc[q][a][0] = acc[q][a][1] = 0.0;
    const double2 *Xs = X + ((long)r * nt + t) * V3 * 12;
    for (long xyz = threadIdx.x; xyz < V3; xyz += blockDim.x) {
        double2 xv[12];
#pragma unroll
        for (int k = 0; k < 12; k++) xv[k] = Xs[xyz * 12 + k];
#pragma unroll
        for (int q = 0; q < NT; q++) {
            int n = n0 + q;
            if (n >= nv) break;
            const double2 *vp = evecs + (((long)t * nv + n) * V3 + xyz) * 3;
            double2 v0 = vp[0], v1 = vp[1], v2 = vp[2];
#pragma unroll
            for (int a = 0; a < 4; a++) {
                double2 s = cadd(cadd(cconjmul(v0, xv[a * 3]), cconjmul(v1, xv[a * 3 + 1])), cconjmul(v2, xv[a * 3 + 2]));
                acc[q][a][0] += s.x;
                acc[q][a][1] += s.y;
            }
        }
    }
    // wave reduction, then across the waves of the block
    __shared__ double lds[4][NT * 8];
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NT; q++)
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int p = 0; p < 2; p++) {
                double v = acc[q][a][p];
                for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
                if (lane == 0) lds[wave][(q * 4 + a) * 2 + p] = v;
            }
    __syncthreads();
    if ((int)threadIdx.x < NT * 4) {
        int q = threadIdx.x / 4, a = threadIdx.x % 4;
        int n = n0 + q;
        if (n < nv) {
            double re = 0, im = 0;
            for (int w = 0; w < (int)(blockDim.x / 64); w++) {
                re += lds[w][(q * 4 + a) * 2];
                im += lds[w][(q * 4 + a) * 2 + 1];
            }
            coef[(((long)r * nt + t) * 4 + a) * nv + n] = make_double2(re, im);
        }
    }
}

Dil make_dil(const laph_dilution *dil, int nt, int nv)
{
    Dil d;
    int N[3] = {nt, 4, nv};
    for (int k = 0; k < 3; k++) {
        d.type[k] = dil->type[k];
        d.J[k] = dil->J[k];
        d.N[k] = N[k];
        switch (dil->type[k]) {
        case LAPH_DIL_NONE: d.cnt[k] = 1; break;
        case LAPH_DIL_FULL: d.cnt[k] = N[k]; break;
        default: d.cnt[k] = dil->J[k]; break;
        }
    }
    return d;
}

}  // namespace

static void launch_z4(laph_ctx *c, uint16_t s, uint16_t k, int nv, double2 *rho)
{
    long n = (long)c->g.nt * 4 * nv;
    uint32_t key0 = ((uint32_t)k << 16) | (uint32_t)s;
    hipLaunchKernelGGL(k_z4, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, key0, c->g.nt, nv, rho);
    LAPH_HIP(hipGetLastError());
}

extern "C" int laph_z4_noise(laph_ctx_t c, uint16_t s, uint16_t k, int nv, double *rho)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(rho && nv > 0, LAPH_EINVAL, "null rho or nv <= 0");
    launch_z4(c, s, k, nv, (double2 *)rho);
    LAPH_HIP(hipStreamSynchronize(c->stream));
    LAPH_API_END(c)
}

extern "C" int make_diluted_source(laph_ctx_t c, const double *evecs, int nv, uint16_t s, uint16_t k,
                                   const laph_dilution *dil, int64_t b_first, int n_src, double *eta)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(evecs && eta && dil && nv > 0 && n_src > 0, LAPH_EINVAL, "bad arguments");
    long nb = laph_dilution_count(dil, c->g.nt, nv);
    LAPH_CHECK(nb > 0, LAPH_EDIVIDE, "invalid dilution scheme (N/J not an integer)");
    LAPH_CHECK(b_first >= 0 && b_first + n_src <= nb, LAPH_EINVAL, "projector index out of range");
    double2 *rho = (double2 *)ctx_named(c, "src.rho", sizeof(double2) * c->g.nt * 4 * nv);
    launch_z4(c, s, k, nv, rho);
    Dil d = make_dil(dil, c->g.nt, nv);
    long n = c->g.V * 3 * n_src;
    hipLaunchKernelGGL(k_source, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, (const double2 *)evecs,
                       (const double2 *)rho, d, (long)b_first, n_src, c->g.V3, c->g.nt, nv, (double2 *)eta);
    LAPH_HIP(hipGetLastError());
    LAPH_API_END(c)
}

extern "C" int sink_project(laph_ctx_t c, const double *evecs, int nv, const double *X, int n_rhs, double *coef)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(evecs && X && coef && nv > 0 && n_rhs > 0, LAPH_EINVAL, "bad arguments");
    LAPH_CHECK(n_rhs <= 65535, LAPH_EINVAL, "n_rhs too large for one call");
    dim3 grid(c->g.nt, (nv + NT - 1) / NT, n_rhs);
    hipLaunchKernelGGL(k_sink, grid, dim3(256), 0, c->stream, (const double2 *)evecs, (const double2 *)X, c->g.V3,
                       c->g.nt, nv, (double2 *)coef);
    LAPH_HIP(hipGetLastError());
    LAPH_API_END(c)
}

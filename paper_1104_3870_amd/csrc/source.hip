// Z4 noise, diluted LapH sources and the sink projection V_s^dag X (Sec. II, Sec. IV).
#include <algorithm>
#include <mutex>

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
// T2: double2 (complex128 output) or float2 (complex64: the FP64 sums rounded once)
template <class T2>
__global__ void k_source(const double2 *__restrict__ evecs, const double2 *__restrict__ rho, Dil d, long b_first,
                         int nsrc, long V3, int nt, int nv, T2 *__restrict__ eta)
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
    T2 *out = eta + ((long)j * V3 * nt + s) * 12;
    double2 acc[4] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
    if (member(d, 0, t, bT)) {
        for (int n = 0; n < nv; n++) {
            if (!member(d, 2, n, bL)) continue;
            double2 v = evecs[(((long)t * nv + n) * V3 + xyz) * 3 + c];
            for (int a = 0; a < 4; a++)
                if (member(d, 1, a, bS)) acc[a] = cadd(acc[a], cmul(v, rho[((long)t * 4 + a) * nv + n]));
        }
    }
    for (int a = 0; a < 4; a++) {
        T2 o;
        o.x = acc[a].x;
        o.y = acc[a].y;
        out[a * 3 + c] = o;
    }
}

// LapH coefficients of the diluted quark sources varrho^[b] = V_s P^(b) rho (or, with the
// spin matrix S set, of S varrho^[b]): out[j][t][alpha][n] = sum_beta S[alpha][beta]
// (P^(b) rho)(t, beta, n), b = b_first + j; one lane per (j, t, n)
struct SpinM {
    double2 m[16];
    int identity;
};

__global__ void k_quark_coef(const double2 *__restrict__ rho, Dil d, long b_first, int nsrc, int nt, int nv,
                             SpinM S, double2 *__restrict__ out)
{
    long q = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (q >= (long)nsrc * nt * nv) return;
    const int n = (int)(q % nv);
    const long jt = q / nv;
    const int t = (int)(jt % nt), j = (int)(jt / nt);
    const long b = b_first + j;
    const int bL = (int)(b % d.cnt[2]);
    const int bS = (int)((b / d.cnt[2]) % d.cnt[1]);
    const int bT = (int)(b / ((long)d.cnt[2] * d.cnt[1]));
    const bool on = member(d, 0, t, bT) && member(d, 2, n, bL);
    double2 v[4];
    for (int a = 0; a < 4; a++)
        v[a] = (on && member(d, 1, a, bS)) ? rho[((long)t * 4 + a) * nv + n] : make_double2(0.0, 0.0);
    for (int a = 0; a < 4; a++) {
        double2 o = v[a];
        if (!S.identity) {
            o = make_double2(0.0, 0.0);
            for (int bb = 0; bb < 4; bb++) o = cadd(o, cmul(S.m[a * 4 + bb], v[bb]));
        }
        out[(jt * 4 + a) * nv + n] = o;
    }
}

// Tiled sink projection: per time slice t the coefficients form the product
// C[(r, alpha)][n] = sum_{x, c} X[r][t][x][alpha][c] conj(V[t][n][x][c]), rows (RHS, spin),
// columns eigenvectors, contraction over the slice's sites and colours.  A block owns one
// t, a tile of kSinkM rows (kSinkM / 4 RHS) and all columns of a column tile, and a range
// of sites (split over blockIdx.z); both operands pass through LDS kSinkX sites at a time,
// so X is read once and V once per row tile.  Partial sums per site range are reduced by
// k_sink_reduce in a fixed order.
constexpr int kSinkM = 64;   // rows per block (16 RHS x 4 spins)
constexpr int kSinkN = 112;  // columns per tile (16 lanes x 7)
constexpr int kSinkX = 4;    // sites per LDS stage (K = 12 per stage)

__global__ __launch_bounds__(256) void k_sink_tiled(const double2 *__restrict__ evecs, const double2 *__restrict__ X,
                                                    long V3, int nt, int nv, int nrhs, int xper,
                                                    double2 *__restrict__ part)
{
    __shared__ double2 sa[kSinkM / 4][kSinkX * 12];  // [rhs in tile][site * 12 + alpha * 3 + c]
    __shared__ double2 sb[kSinkN][kSinkX * 3 + 1];   // [column][site * 3 + c] (padded)
    const int t = blockIdx.x;
    const int mt = blockIdx.y % ((nrhs * 4 + kSinkM - 1) / kSinkM);
    const int nt0 = (blockIdx.y / ((nrhs * 4 + kSinkM - 1) / kSinkM)) * kSinkN;
    const int r0 = mt * (kSinkM / 4);
    const long x0 = (long)blockIdx.z * xper, x1 = std::min(V3, x0 + xper);
    const int tm = threadIdx.x >> 4, tn = threadIdx.x & 15;  // rows tm*4 .. +3, columns tn + 16 j
    double acc[4][7][2];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 7; j++) acc[i][j][0] = acc[i][j][1] = 0.0;
    for (long xs = x0; xs < x1; xs += kSinkX) {
        const int nx = (int)std::min((long)kSinkX, x1 - xs);
        // stage X: 16 RHS x nx sites x 12 components (each RHS's sites are contiguous)
        for (int k = threadIdx.x; k < (kSinkM / 4) * kSinkX * 12; k += blockDim.x) {
            const int rr = k / (kSinkX * 12), e = k - rr * (kSinkX * 12);
            const int r = r0 + rr;
            double2 v = make_double2(0.0, 0.0);
            if (r < nrhs && e < nx * 12) v = X[(((long)r * nt + t) * V3 + xs) * 12 + e];
            sa[rr][e] = v;
        }
        // stage V: kSinkN columns x nx sites x 3 colours, conjugated
        for (int k = threadIdx.x; k < kSinkN * kSinkX * 3; k += blockDim.x) {
            const int nn = k / (kSinkX * 3), e = k - nn * (kSinkX * 3);
            const int n = nt0 + nn;
            double2 v = make_double2(0.0, 0.0);
            if (n < nv && e < nx * 3) {
                v = evecs[(((long)t * nv + n) * V3 + xs) * 3 + e];
                v.y = -v.y;
            }
            sb[nn][e] = v;
        }
        __syncthreads();
#pragma unroll 2
        for (int xi = 0; xi < kSinkX; xi++)
#pragma unroll
            for (int cc = 0; cc < 3; cc++) {
                double2 bv[7];
#pragma unroll
                for (int j = 0; j < 7; j++) bv[j] = sb[tn + 16 * j][xi * 3 + cc];
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    // row tm * 4 + i = (rhs (tm * 4 + i) / 4, spin (tm * 4 + i) % 4) = (tm, i)
                    const double2 av = sa[tm][xi * 12 + i * 3 + cc];
#pragma unroll
                    for (int j = 0; j < 7; j++) {
                        acc[i][j][0] = fma(av.x, bv[j].x, fma(-av.y, bv[j].y, acc[i][j][0]));
                        acc[i][j][1] = fma(av.x, bv[j].y, fma(av.y, bv[j].x, acc[i][j][1]));
                    }
                }
            }
        __syncthreads();
    }
    // part[z][r][t][alpha][n]
    const int r = r0 + tm;
    if (r >= nrhs) return;
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 7; j++) {
            const int n = nt0 + tn + 16 * j;
            if (n < nv)
                part[((((long)blockIdx.z * nrhs + r) * nt + t) * 4 + i) * nv + n] =
                    make_double2(acc[i][j][0], acc[i][j][1]);
        }
}

// coef = sum over the site ranges of the partial products, in range order
__global__ void k_sink_reduce(const double2 *__restrict__ part, int nz, long m, double2 *__restrict__ coef)
{
    long q = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (q >= m) return;
    double2 s = make_double2(0.0, 0.0);
    for (int z = 0; z < nz; z++) s = cadd(s, part[(long)z * m + q]);
    coef[q] = s;
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
                                   const laph_dilution *dil, int64_t b_first, int n_src, void *eta, int dtype)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(evecs && eta && dil && nv > 0 && n_src > 0, LAPH_EINVAL, "bad arguments");
    LAPH_CHECK(dtype == LAPH_DTYPE_C128 || dtype == LAPH_DTYPE_C64, LAPH_EINVAL, "unknown dtype");
    long nb = laph_dilution_count(dil, c->g.nt, nv);
    LAPH_CHECK(nb > 0, LAPH_EDIVIDE, "invalid dilution scheme (N/J not an integer)");
    LAPH_CHECK(b_first >= 0 && b_first + n_src <= nb, LAPH_EINVAL, "projector index out of range");
    double2 *rho = (double2 *)ctx_named(c, "src.rho", sizeof(double2) * c->g.nt * 4 * nv);
    launch_z4(c, s, k, nv, rho);
    Dil d = make_dil(dil, c->g.nt, nv);
    long n = c->g.V * 3 * n_src;
    if (dtype == LAPH_DTYPE_C128)
        hipLaunchKernelGGL(k_source<double2>, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream,
                           (const double2 *)evecs, (const double2 *)rho, d, (long)b_first, n_src, c->g.V3, c->g.nt,
                           nv, (double2 *)eta);
    else
        hipLaunchKernelGGL(k_source<float2>, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream,
                           (const double2 *)evecs, (const double2 *)rho, d, (long)b_first, n_src, c->g.V3, c->g.nt,
                           nv, (float2 *)eta);
    LAPH_HIP(hipGetLastError());
    LAPH_API_END(c)
}

// The quark-source coefficients of the gamma_5-Hermitian estimate (Sec. II): varrho-bar =
// -gamma_5 gamma_4 varrho, with the chiral-basis matrices gamma_4 = [[0, 1], [1, 0]] (2x2
// blocks) and gamma_5 = diag(1, 1, -1, -1) written as data and multiplied here.
static SpinM bar_matrix()
{
    const double g4[4][4] = {{0, 0, 1, 0}, {0, 0, 0, 1}, {1, 0, 0, 0}, {0, 1, 0, 0}};
    const double g5[4] = {1, 1, -1, -1};
    SpinM S;
    S.identity = 0;
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++) S.m[a * 4 + b] = make_double2(-g5[a] * g4[a][b], 0.0);
    return S;
}

extern "C" int laph_quark_source(laph_ctx_t c, int nv, uint16_t s, uint16_t k, const laph_dilution *dil,
                                 int64_t b_first, int n_src, int bar, double *out)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(out && dil && nv > 0 && n_src > 0, LAPH_EINVAL, "bad arguments");
    long nb = laph_dilution_count(dil, c->g.nt, nv);
    LAPH_CHECK(nb > 0, LAPH_EDIVIDE, "invalid dilution scheme (N/J not an integer)");
    LAPH_CHECK(b_first >= 0 && b_first + n_src <= nb, LAPH_EINVAL, "projector index out of range");
    double2 *rho = (double2 *)ctx_named(c, "src.rho", sizeof(double2) * c->g.nt * 4 * nv);
    launch_z4(c, s, k, nv, rho);
    Dil d = make_dil(dil, c->g.nt, nv);
    SpinM S{};
    S.identity = 1;
    if (bar) S = bar_matrix();
    const long n = (long)n_src * c->g.nt * nv;
    hipLaunchKernelGGL(k_quark_coef, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, (const double2 *)rho, d,
                       (long)b_first, n_src, c->g.nt, nv, S, (double2 *)out);
    LAPH_HIP(hipGetLastError());
    LAPH_API_END(c)
}

// site ranges (split-K factor) of the tiled sink projection
static long sink_ranges(const Geom &g, int nv, int n_rhs, long &xper)
{
    const int mtiles = (n_rhs * 4 + kSinkM - 1) / kSinkM, ntiles = (nv + kSinkN - 1) / kSinkN;
    const long base = (long)g.nt * mtiles * ntiles;
    long nz = std::max(1L, std::min(g.V3 / (8 * kSinkX), 2048 / std::max(1L, base)));
    xper = (g.V3 + nz - 1) / nz;
    xper = (xper + kSinkX - 1) / kSinkX * kSinkX;
    return (g.V3 + xper - 1) / xper;
}

size_t sink_scratch_bytes(const Geom &g, int nv, int n_rhs)
{
    long xper;
    const long nz = sink_ranges(g, nv, n_rhs, xper);
    return ws_align(sizeof(double2) * (size_t)n_rhs * g.nt * 4 * nv * nz);
}

size_t source_scratch_bytes(const Geom &g, int nv) { return ws_align(sizeof(double2) * g.nt * 4 * nv); }

// the tiled product and the fixed-order reduction of its site ranges, partials in part
// (room for nz_max ranges of m values; the range count is cut to fit)
static void sink_launch(laph_ctx *c, const double *evecs, int nv, const double *X, int n_rhs, double *coef,
                        double2 *part, long nz_max)
{
    const int mtiles = (n_rhs * 4 + kSinkM - 1) / kSinkM, ntiles = (nv + kSinkN - 1) / kSinkN;
    long xper;
    long nz = sink_ranges(c->g, nv, n_rhs, xper);
    if (nz > nz_max) {
        xper = (c->g.V3 + nz_max - 1) / nz_max;
        xper = (xper + kSinkX - 1) / kSinkX * kSinkX;
        nz = (c->g.V3 + xper - 1) / xper;
    }
    LAPH_CHECK(mtiles * ntiles <= 65535 && nz <= 65535, LAPH_EINVAL, "sink projection too large for one call");
    const long m = (long)n_rhs * c->g.nt * 4 * nv;
    hipLaunchKernelGGL(k_sink_tiled, dim3(c->g.nt, mtiles * ntiles, nz), dim3(256), 0, c->stream,
                       (const double2 *)evecs, (const double2 *)X, c->g.V3, c->g.nt, nv, n_rhs, (int)xper, part);
    LAPH_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sink_reduce, dim3(nblocks_for(m, 256)), dim3(256), 0, c->stream, (const double2 *)part,
                       (int)nz, m, (double2 *)coef);
    LAPH_HIP(hipGetLastError());
}

extern "C" int sink_project(laph_ctx_t c, const double *evecs, int nv, const double *X, int n_rhs, double *coef)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(evecs && X && coef && nv > 0 && n_rhs > 0, LAPH_EINVAL, "bad arguments");
    LAPH_CHECK(n_rhs <= 65535, LAPH_EINVAL, "n_rhs too large for one call");
    long xper;
    const long nz = sink_ranges(c->g, nv, n_rhs, xper);
    const long m = (long)n_rhs * c->g.nt * 4 * nv;
    double2 *part = (double2 *)ctx_named(c, "sink.part", sizeof(double2) * m * nz);
    sink_launch(c, evecs, nv, X, n_rhs, coef, part, nz);
    LAPH_API_END(c)
}

// ---------------------------------------------- sink projection without a workspace
// The partial products of sink_project_noalloc live in this array, one copy per device,
// held until the process ends.  Host code must not pass the array's name to a kernel (it
// is a host-side stand-in there): it uses the device address that sink_scratch_init looks
// up once per device.  k_sink_tiled writes every partial it sums, so nothing needs to
// start at zero.
constexpr size_t kSinkScratchBytes = (size_t)LAPH_SINK_NOALLOC_BYTES;
static __device__ __align__(256) double2 scratch[kSinkScratchBytes / sizeof(double2)];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64];  // device address of `scratch` per device ordinal

// once per device, with that device current (laph_create)
void sink_scratch_init(laph_ctx *c)
{
    LAPH_CHECK(c->device >= 0 && c->device < 64, LAPH_EINVAL, "device ordinal %d out of range", c->device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[c->device]) {
        void *ptr = nullptr;
        LAPH_HIP(hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)));
        LAPH_CHECK(ptr != nullptr, LAPH_EHIP, "no device address for the sink scratch array");
        g_scratch_ptr[c->device] = ptr;
    }
    c->sink_scratch = g_scratch_ptr[c->device];
}

extern "C" int sink_project_noalloc(laph_ctx_t c, const double *evecs, int nv, const double *X, int n_rhs,
                                    double *coef)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(evecs && X && coef && nv > 0 && n_rhs > 0, LAPH_EINVAL, "bad arguments");
    LAPH_CHECK(c->sink_scratch, LAPH_EHIP, "sink scratch array not set up on device %d", c->device);
    const size_t m = (size_t)n_rhs * c->g.nt * 4 * nv;
    LAPH_CHECK(m * sizeof(double2) <= kSinkScratchBytes, LAPH_EINVAL,
               "n_rhs * Nt * 4 * nv * 16 = %zu bytes of partial sums exceed the fixed scratch of %zu bytes",
               m * sizeof(double2), kSinkScratchBytes);
    const long nz_max = (long)(kSinkScratchBytes / (m * sizeof(double2)));
    sink_launch(c, evecs, nv, X, n_rhs, coef, (double2 *)c->sink_scratch, nz_max);
    LAPH_API_END(c)
}

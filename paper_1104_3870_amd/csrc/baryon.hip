// Baryon functions in LapH space (Sec. III.A: Eq. baryonfunc, and the baryon correlator
// of Eq. baryoncorr with its six noise orderings).
//
// With the trivial displacement every LapH-smeared quark sink is varphi = V_s f, so
//   B(t) = sum_{abg} c_abg sum_{n1 n2 n3} T[t][n1][n2][n3] f1[t][a][n1] f2[t][b][n2] f3[t][g][n3]
// with the eigenvector tensor T[t][n1][n2][n3] = sum_x e^{-ip.x} eps_abc V_n1(x,a) V_n2(x,b)
// V_n3(x,c) (totally antisymmetric: computed for n1 < n2, the rest by symmetry).  The
// contraction over (n1, n2, n3) for all dilution triples is three batched complex products:
//   X[n1 n2][k g]   = sum_n3 T[n1 n2][n3] F3[n3][k g]
//   Y[n1][j b][k g] = sum_n2 F2[n2][j b] X[n1 n2][k g]
//   Z[i a][j b k g] = sum_n1 F1[n1][i a] Y[n1][j b k g],   B[i][j][k] = sum c_abg Z[i a][j b][k g]
#include <algorithm>
#include <cmath>

#include "laph_impl.h"
#include "zgemm_mfma.h"

namespace {

// ------------------------------------------------------- batched complex product
// C[b](m, n) = sum_k op(A[b](m, k)) B[b](k, n), op = conj when conjA; every operand is
// addressed by strides (in complex elements); the batch index b splits into (b / nbi, b % nbi)
// with a stride per part.  Computed on the FP64 matrix cores (zgemm_mfma.h).
struct Zgemm {
    const double2 *A;
    long sAo, sAi, sAm, sAk;
    const double2 *B;
    long sBo, sBi, sBk, sBn;
    double2 *C;
    long sCo, sCi, sCm, sCn;
    int M, N, K, nbi, conjA;
};

struct GemmS {
    Zgemm g;
    int M, N, K;
    __device__ bool tile(long &bt, int &m0, int &n0) const
    {
        bt = blockIdx.z;
        m0 = blockIdx.x * zg::kTM;
        n0 = blockIdx.y * zg::kTN;
        return true;
    }
    // element q of a lane: e = lane + 256 q; the index running along the operand's unit
    // stride varies fastest across lanes
    template <int KT>
    struct Reg {
        double2 a[zg::kPer<KT>], b[zg::kPer<KT>];
    };
    template <int KT>
    __device__ void am(int e, int &m, int &k) const
    {
        const bool ak = g.sAk == 1;
        m = ak ? e / KT : e % zg::kTM;
        k = ak ? e % KT : e / zg::kTM;
    }
    template <int KT>
    __device__ void load(Reg<KT> &r, long bt, int m0, int n0, int k0) const
    {
        const long bo = bt / g.nbi, bi = bt - bo * g.nbi;
        const double2 *A = g.A + bo * g.sAo + bi * g.sAi;
        const double2 *B = g.B + bo * g.sBo + bi * g.sBi;
#pragma unroll
        for (int q = 0; q < zg::kPer<KT>; q++) {
            const int e = threadIdx.x + 256 * q;
            int m, k;
            am<KT>(e, m, k);
            // explicit branches (a select against a local zero would load through a flat
            // address)
            r.a[q] = r.b[q] = make_double2(0.0, 0.0);
            if (m0 + m < M && k0 + k < K) r.a[q] = A[(m0 + m) * g.sAm + (long)(k0 + k) * g.sAk];
            const int n = e % zg::kTN, kb = e / zg::kTN;
            if (n0 + n < N && k0 + kb < K) r.b[q] = B[(long)(k0 + kb) * g.sBk + (n0 + n) * g.sBn];
        }
    }
    template <int KT>
    __device__ void put(zg::Tile<KT> &t, const Reg<KT> &r) const
    {
        const double sg = g.conjA ? -1.0 : 1.0;
#pragma unroll
        for (int q = 0; q < zg::kPer<KT>; q++) {
            const int e = threadIdx.x + 256 * q;
            int m, k;
            am<KT>(e, m, k);
            t.ar[k][m] = r.a[q].x;
            t.ai[k][m] = sg * r.a[q].y;
            const int n = e % zg::kTN, kb = e / zg::kTN;
            t.br[kb][n] = r.b[q].x;
            t.bi[kb][n] = r.b[q].y;
        }
    }
    __device__ void store(long bt, int m, int n, double re, double im) const
    {
        const long bo = bt / g.nbi, bi = bt - bo * g.nbi;
        g.C[bo * g.sCo + bi * g.sCi + m * g.sCm + n * g.sCn] = make_double2(re, im);
    }
};

void zgemm(laph_ctx *c, const Zgemm &g, long batch)
{
    if (g.M <= 0 || g.N <= 0 || batch <= 0) return;
    const unsigned gm = (g.M + zg::kTM - 1) / zg::kTM, gn = (g.N + zg::kTN - 1) / zg::kTN;
    LAPH_CHECK(gn <= 65535 && batch <= 65535, LAPH_EINVAL, "product too large for one launch");
    GemmS s{g, g.M, g.N, g.K};
    hipLaunchKernelGGL((zg::k_zgemm<16, GemmS>), dim3(gm, gn, (unsigned)batch), dim3(256), 0, c->stream, s);
    LAPH_HIP(hipGetLastError());
}

// ------------------------------------------------------- eigenvector tensor
// T[t][n1][n2][n3] = sum_{x,c} (e^{-ip.x} V_n1(x) x V_n2(x))_c V_n3(x, c), (u x w)_c =
// eps_abc u_a w_b, is totally antisymmetric, so only n1 < n2 < n3 is computed and each
// value is written to its six images (the tensor is zeroed first, which leaves every entry
// with a repeated index at zero).  One block per (n1, slice, chunk of tile pairs): for the
// 16-row tiles a <= b of n2 and n3 that can hold n1 < n2 < n3, the products
// A[n2][(x c)] B[(x c)][n3] with A the cross products (formed while staging) and
// B = V_n3, on the FP64 matrix cores; the rows of A and B from the block's first tile on
// are staged through LDS four sites at a time, and the block's four waves take the pairs
// in turn.  Loading each stage one stage ahead (registers) and staging only the rows the
// block's pairs read took the 24^3 x 128, N_v = 112 tensor from 527 to 470 ms.
constexpr int kBT = 16;  // MFMA tile
constexpr int kBK = 12;  // K per stage: four sites x three colours
constexpr int kBP = 6;   // tile pairs per wave and block

__host__ __device__ inline int tri_pairs(int u) { return u * (u + 1) / 2; }

// SA, SB: staging elements of A (rows x 4 sites) and B (rows x kBK) per lane whose global
// loads are held in registers one stage ahead, so that the loads of stage k + 1 are in
// flight during the matrix products of stage k (SA = 0: staged directly, for row counts
// whose elements would not fit the registers).  The phase-multiplied V_n1 of a stage's
// four sites is formed once per stage into LDS.
template <int SA, int SB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_baryon_tensor_tri(
    const double2 *__restrict__ V, const double2 *__restrict__ ph, int nv, long V3, int T, double2 *__restrict__ out)
{
    extern __shared__ double lds[];
    const int NP = T * kBT + 4;  // LDS row stride (doubles)
    double *ar = lds, *ai = ar + kBK * NP, *br = ai + kBK * NP, *bi = br + kBK * NP;
    __shared__ double2 su[2][kBK];  // e^{-ip.x} V_n1(x) of the stage's sites, double-buffered
    const int n1 = blockIdx.x, t = blockIdx.z;
    const int amin = (n1 + 1) / kBT;  // first n2 tile holding an n2 > n1
    if (amin >= T) return;
    const int np = tri_pairs(T - amin);
    const int p0 = blockIdx.y * 4 * kBP;
    if (p0 >= np) return;  // uniform over the block
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l & 15, lk = l >> 4;
    // this wave's pairs p = p0 + wave + 4 j, decoded to (a, b), a <= b
    int pa[kBP], pb[kBP];
#pragma unroll
    for (int j = 0; j < kBP; j++) {
        int p = p0 + wave + 4 * j, a = amin;
        pa[j] = -1;
        pb[j] = -1;
        if (p < np && p < p0 + 4 * kBP) {
            while (p >= T - a) {
                p -= T - a;
                a++;
            }
            pa[j] = a;
            pb[j] = a + p;
        }
    }
    zg::d4 cr[kBP], ci[kBP];
#pragma unroll
    for (int j = 0; j < kBP; j++) {
        cr[j] = zg::d4{0.0, 0.0, 0.0, 0.0};
        ci[j] = zg::d4{0.0, 0.0, 0.0, 0.0};
    }
    const long K = 3 * V3;
    const double2 *Vt = V + (long)t * nv * K;
    // rows from the first tile any pair of this block reads
    const int rlo = kBT * amin, rows = T * kBT;
    const double2 z2 = make_double2(0.0, 0.0);
    // lanes 0..11: e^{-ip.x} V_n1(x)_c of the stage's (site, colour) k into su[buf][k]
    auto u_stage = [&](long k0, int buf) {
        if (threadIdx.x < kBK) {
            const long kk = k0 + threadIdx.x, x = kk / 3;
            su[buf][threadIdx.x] = kk < K ? cmul(ph[x], Vt[(long)n1 * K + kk]) : z2;
        }
    };
    // A element e = (m, site xs): the cross product of su with V_m(x)
    auto a_in = [&](int e, long k0, double2 (&w)[3]) {
        const int m = rlo + (e >> 2);
        const long x = k0 / 3 + (e & 3);
        if (m < rows && x < V3 && m < nv) {
            const double2 *wp = Vt + ((long)m * V3 + x) * 3;
            w[0] = wp[0];
            w[1] = wp[1];
            w[2] = wp[2];
        } else {
            w[0] = w[1] = w[2] = z2;
        }
    };
    auto a_out = [&](int e, const double2 (&w)[3], int buf) {
        const int m = rlo + (e >> 2), xs = e & 3;
        if (m >= rows) return;
        const double2 u0 = su[buf][3 * xs], u1 = su[buf][3 * xs + 1], u2 = su[buf][3 * xs + 2];
        const double2 c3[3] = {csub(cmul(u1, w[2]), cmul(u2, w[1])), csub(cmul(u2, w[0]), cmul(u0, w[2])),
                               csub(cmul(u0, w[1]), cmul(u1, w[0]))};
#pragma unroll
        for (int cc = 0; cc < 3; cc++) {
            ar[(3 * xs + cc) * NP + m] = c3[cc].x;
            ai[(3 * xs + cc) * NP + m] = c3[cc].y;
        }
    };
    // B element e = (n3, k): V_n3 at K index k0 + k (K contiguous per vector)
    auto b_in = [&](int e, long k0) {
        const int q = e / kBK, n = rlo + q;
        const long kk = k0 + (e - q * kBK);
        // an explicit branch: a select against the local zero would load through a flat
        // address
        double2 v = z2;
        if (n < rows && kk < K && n < nv) v = Vt[(long)n * K + kk];
        return v;
    };
    auto b_out = [&](int e, double2 v) {
        const int q = e / kBK, n = rlo + q, k = e - q * kBK;
        if (n >= rows) return;
        br[k * NP + n] = v.x;
        bi[k * NP + n] = v.y;
    };
    const int na = (rows - rlo) * 4, nb = (rows - rlo) * kBK;
    double2 ra[SA > 0 ? SA : 1][3], rb[SB > 0 ? SB : 1];
    if constexpr (SA > 0) {
#pragma unroll
        for (int q = 0; q < SA; q++) a_in(threadIdx.x + 256 * q, 0, ra[q]);
#pragma unroll
        for (int q = 0; q < SB; q++) rb[q] = b_in(threadIdx.x + 256 * q, 0);
    }
    u_stage(0, 0);
    __syncthreads();
    int buf = 0;
    for (long k0 = 0; k0 < K; k0 += kBK) {
        if constexpr (SA > 0) {
#pragma unroll
            for (int q = 0; q < SA; q++)
                if (threadIdx.x + 256 * q < na) a_out(threadIdx.x + 256 * q, ra[q], buf);
#pragma unroll
            for (int q = 0; q < SB; q++)
                if (threadIdx.x + 256 * q < nb) b_out(threadIdx.x + 256 * q, rb[q]);
        } else {
            for (int e = threadIdx.x; e < na; e += blockDim.x) {
                a_in(e, k0, ra[0]);
                a_out(e, ra[0], buf);
            }
            for (int e = threadIdx.x; e < nb; e += blockDim.x) b_out(e, b_in(e, k0));
        }
        // the next stage's V_n1 goes to the other buffer, read after the next barrier
        if (k0 + kBK < K) u_stage(k0 + kBK, buf ^ 1);
        __syncthreads();
        if constexpr (SA > 0) {
            // the next stage's loads, consumed after this stage's products
            if (k0 + kBK < K) {
#pragma unroll
                for (int q = 0; q < SA; q++) a_in(threadIdx.x + 256 * q, k0 + kBK, ra[q]);
#pragma unroll
                for (int q = 0; q < SB; q++) rb[q] = b_in(threadIdx.x + 256 * q, k0 + kBK);
            }
        }
        // one K step of 4 at a time: its LDS operands of the six pairs (48 registers) are
        // what the compiler keeps in flight, leaving room for the next stage's loads
#pragma unroll 1
        for (int kk = 0; kk < kBK; kk += 4) {
#pragma unroll
            for (int j = 0; j < kBP; j++) {
                if (pa[j] < 0) continue;  // uniform over the wave
                const int ia = (kk + lk) * NP + kBT * pa[j] + lr, ib = (kk + lk) * NP + kBT * pb[j] + lr;
                const double xr = ar[ia], xi = ai[ia], yr = br[ib], yi = bi[ib];
                cr[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr, yr, cr[j], 0, 0, 0);
                cr[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-xi, yi, cr[j], 0, 0, 0);
                ci[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr, yi, ci[j], 0, 0, 0);
                ci[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xi, yr, ci[j], 0, 0, 0);
            }
        }
        __syncthreads();
        buf ^= 1;
    }
    // element v of lane l: C[lk + 4 v][lr] of the pair's tile (see zgemm_mfma.h)
    const long nv2 = (long)nv * nv, base = (long)t * nv * nv2;
#pragma unroll
    for (int j = 0; j < kBP; j++) {
        if (pa[j] < 0) continue;
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int n2 = kBT * pa[j] + lk + 4 * v, n3 = kBT * pb[j] + lr;
            if (n2 <= n1 || n3 <= n2 || n3 >= nv) continue;
            const double2 q = make_double2(cr[j][v], ci[j][v]), mq = make_double2(-cr[j][v], -ci[j][v]);
            out[base + n1 * nv2 + (long)n2 * nv + n3] = q;
            out[base + n1 * nv2 + (long)n3 * nv + n2] = mq;
            out[base + n2 * nv2 + (long)n1 * nv + n3] = mq;
            out[base + n2 * nv2 + (long)n3 * nv + n1] = q;
            out[base + n3 * nv2 + (long)n1 * nv + n2] = q;
            out[base + n3 * nv2 + (long)n2 * nv + n1] = mq;
        }
    }
}

__global__ void k_zero2(double2 *p, long n)
{
    const long q = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (q < n) p[q] = make_double2(0.0, 0.0);
}

__global__ void k_phase3(double2 *ph, int ns, int k0, int k1, int k2)
{
    const long V3 = (long)ns * ns * ns;
    const long x = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (x >= V3) return;
    const int cx = (int)(x % ns), cy = (int)((x / ns) % ns), cz = (int)(x / ((long)ns * ns));
    const long m = (((long)k0 * cx + (long)k1 * cy + (long)k2 * cz) % ns + ns) % ns;
    double s, c;
    sincospi(-2.0 * (double)m / ns, &s, &c);
    ph[x] = make_double2(c, s);
}

// Ft[tl][n][i*4 + alpha] = f[i][t0 + tl][alpha][n] for tc slices
__global__ void k_coef_t(const double2 *__restrict__ f, int nf, int nt, int nv, int t0, int tc,
                         double2 *__restrict__ Ft)
{
    const long q = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const long per = (long)nv * nf * 4;
    if (q >= tc * per) return;
    const int tl = (int)(q / per);
    const long r = q - tl * per;
    const int n = (int)(r / (nf * 4));
    const int ia = (int)(r - (long)n * nf * 4);
    const int i = ia / 4, a = ia % 4;
    Ft[q] = f[(((long)i * nt + t0 + tl) * 4 + a) * nv + n];
}

struct Spin64 {
    double2 c[64];
};

// B[t][i][j][k] = sum_{abg} c_abg Z[tl][(i a)][(j b)(k g)]
__global__ void k_spin3(Spin64 s, const double2 *__restrict__ Z, int n1, int n2, int n3, int t0, int tc,
                        double2 *__restrict__ out)
{
    const long q = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const long per = (long)n1 * n2 * n3;
    if (q >= tc * per) return;
    const int tl = (int)(q / per);
    const long r = q - tl * per;
    const int i = (int)(r / ((long)n2 * n3)), j = (int)((r / n3) % n2), k = (int)(r % n3);
    const long ncol = 16L * n2 * n3;
    const double2 *Zt = Z + (long)tl * (4L * n1) * ncol;
    double2 acc = make_double2(0.0, 0.0);
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++)
            for (int g = 0; g < 4; g++) {
                const double2 cc = s.c[(a * 4 + b) * 4 + g];
                if (cc.x == 0.0 && cc.y == 0.0) continue;
                acc = cadd(acc, cmul(cc, Zt[((long)i * 4 + a) * ncol + ((long)j * 4 + b) * (4L * n3) + k * 4 + g]));
            }
    out[(long)(t0 + tl) * per + r] = acc;
}

// C[tF] = sum_{b1 b2 b3} snk[tF][b1][b2][b3] conj(sum_s sign_s src[s][t0][b_s1][b_s2][b_s3]),
// the six orderings s of Eq. baryoncorr in a fixed order (noise order, sign)
__constant__ int kBPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {2, 1, 0}, {1, 2, 0}, {2, 0, 1}};
__constant__ double kBSign[6] = {1, -1, -1, -1, 1, 1};

__global__ __launch_bounds__(256) void k_baryon_corr(const double2 *__restrict__ snk, const double2 *__restrict__ src,
                                                     int n, int nt, int t0, double2 *__restrict__ out)
{
    const int tf = blockIdx.x;
    const long n3 = (long)n * n * n;
    double2 acc = make_double2(0.0, 0.0);
    for (long q = threadIdx.x; q < n3; q += 256) {
        const int bidx[3] = {(int)(q / ((long)n * n)), (int)((q / n) % n), (int)(q % n)};
        double2 s = make_double2(0.0, 0.0);
        for (int p = 0; p < 6; p++) {
            const long idx = ((long)bidx[kBPerm[p][0]] * n + bidx[kBPerm[p][1]]) * n + bidx[kBPerm[p][2]];
            const double2 v = src[((long)p * nt + t0) * n3 + idx];
            s.x += kBSign[p] * v.x;
            s.y += kBSign[p] * v.y;
        }
        acc = cadd(acc, cconjmul(s, snk[(long)tf * n3 + q]));
    }
    __shared__ double2 red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[tf] = red[0];
}

}  // namespace

// slices per pass of laph_baryon_function: as many as fit a scratch budget of 1 GiB
static int baryon_chunk(int nt, int nv, int n1, int n2, int n3)
{
    const double per = 16.0 * ((double)nv * nv * 4 * n3 + (double)nv * 16 * n2 * n3 + 4.0 * n1 * 16 * n2 * n3 +
                               4.0 * nv * (n1 + n2 + n3));
    int tc = (int)std::max(1.0, std::floor((double)(1u << 30) / per));
    return std::min(tc, nt);
}

size_t baryon_scratch_bytes(const Geom &g, int nv, int n1, int n2, int n3)
{
    const long tc = baryon_chunk(g.nt, nv, n1, n2, n3);
    return ws_align(16 * tc * nv * 4 * n1) + ws_align(16 * tc * nv * 4 * n2) + ws_align(16 * tc * nv * 4 * n3) +
           ws_align(16 * tc * nv * nv * 4 * n3) + ws_align(16 * tc * nv * 16 * n2 * n3) +
           ws_align(16 * tc * 4 * n1 * 16 * n2 * n3);
}

extern "C" int laph_baryon_tensor(laph_ctx_t c, const double *evecs, int nv, const int *k, double *T)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(evecs && k && T && nv > 0, LAPH_EINVAL, "bad arguments");
    const long V3 = c->g.V3;
    double2 *ph = (double2 *)ctx_named(c, "bar.phase", sizeof(double2) * V3);
    hipLaunchKernelGGL(k_phase3, dim3(nblocks_for(V3, 256)), dim3(256), 0, c->stream, ph, c->g.ns, k[0], k[1], k[2]);
    const int tiles = (nv + kBT - 1) / kBT;
    const size_t lds = sizeof(double) * 4 * kBK * (size_t)(tiles * kBT + 4);
    LAPH_CHECK(lds <= 160 * 1024, LAPH_EINVAL, "nv too large: the tensor kernel stages all N_v vectors in LDS");
    LAPH_CHECK(c->g.nt <= 65535 && 3 * V3 < (1L << 31), LAPH_EINVAL, "lattice too large for one launch");
    // up to 128 rows (N_v <= 128) each lane holds two A and six B elements of the next stage
    const bool pre = tiles * kBT <= 128;
    const void *kern = pre ? (const void *)k_baryon_tensor_tri<2, 6> : (const void *)k_baryon_tensor_tri<0, 0>;
    if (lds > 64 * 1024)
        LAPH_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const long total = (long)c->g.nt * nv * nv * nv;
    hipLaunchKernelGGL(k_zero2, dim3(nblocks_for(total, 256)), dim3(256), 0, c->stream, (double2 *)T, total);
    const int chunks = (tri_pairs(tiles) + 4 * kBP - 1) / (4 * kBP);
    const dim3 grid(nv, chunks, c->g.nt);
    if (pre)
        hipLaunchKernelGGL((k_baryon_tensor_tri<2, 6>), grid, dim3(256), lds, c->stream, (const double2 *)evecs,
                           (const double2 *)ph, nv, V3, tiles, (double2 *)T);
    else
        hipLaunchKernelGGL((k_baryon_tensor_tri<0, 0>), grid, dim3(256), lds, c->stream, (const double2 *)evecs,
                           (const double2 *)ph, nv, V3, tiles, (double2 *)T);
    LAPH_HIP(hipGetLastError());
    LAPH_API_END(c)
}

extern "C" int laph_baryon_function(laph_ctx_t c, const double *T, int nv, const double *cs, const double *f1, int n1,
                                    const double *f2, int n2, const double *f3, int n3, double *out)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(T && cs && f1 && f2 && f3 && out && nv > 0 && n1 > 0 && n2 > 0 && n3 > 0, LAPH_EINVAL,
               "bad arguments");
    Spin64 s;
    for (int q = 0; q < 64; q++) {
        LAPH_CHECK(std::isfinite(cs[2 * q]) && std::isfinite(cs[2 * q + 1]), LAPH_EINVAL, "spin tensor not finite");
        s.c[q] = make_double2(cs[2 * q], cs[2 * q + 1]);
    }
    const int nt = c->g.nt;
    const int tc = baryon_chunk(nt, nv, n1, n2, n3);
    const long c1 = 4L * n1, c2 = 4L * n2, c3 = 4L * n3;
    double2 *F1 = (double2 *)ctx_named(c, "bar.F1", 16 * (size_t)tc * nv * c1);
    double2 *F2 = (double2 *)ctx_named(c, "bar.F2", 16 * (size_t)tc * nv * c2);
    double2 *F3 = (double2 *)ctx_named(c, "bar.F3", 16 * (size_t)tc * nv * c3);
    double2 *X = (double2 *)ctx_named(c, "bar.X", 16 * (size_t)tc * nv * nv * c3);
    double2 *Y = (double2 *)ctx_named(c, "bar.Y", 16 * (size_t)tc * nv * c2 * c3);
    double2 *Z = (double2 *)ctx_named(c, "bar.Z", 16 * (size_t)tc * c1 * c2 * c3);
    const double2 *Td = (const double2 *)T;
    for (int t0 = 0; t0 < nt; t0 += tc) {
        const int tcn = std::min(tc, nt - t0);
        hipLaunchKernelGGL(k_coef_t, dim3(nblocks_for((long)tcn * nv * c1, 256)), dim3(256), 0, c->stream,
                           (const double2 *)f1, n1, nt, nv, t0, tcn, F1);
        hipLaunchKernelGGL(k_coef_t, dim3(nblocks_for((long)tcn * nv * c2, 256)), dim3(256), 0, c->stream,
                           (const double2 *)f2, n2, nt, nv, t0, tcn, F2);
        hipLaunchKernelGGL(k_coef_t, dim3(nblocks_for((long)tcn * nv * c3, 256)), dim3(256), 0, c->stream,
                           (const double2 *)f3, n3, nt, nv, t0, tcn, F3);
        LAPH_HIP(hipGetLastError());
        // X[tl][n1 n2][k g] = sum_n3 T[t][n1 n2][n3] F3[tl][n3][k g]
        Zgemm gx{Td + (size_t)t0 * nv * nv * nv, (long)nv * nv * nv, 0, nv, 1,
                 F3, nv * c3, 0, c3, 1,
                 X, (long)nv * nv * c3, 0, c3, 1,
                 nv * nv, (int)c3, nv, 1, 0};
        zgemm(c, gx, tcn);
        // Y[tl][n1][j b][k g] = sum_n2 F2[tl][n2][j b] X[tl][n1 n2][k g]
        Zgemm gy{F2, nv * c2, 0, 1, c2,
                 X, (long)nv * nv * c3, (long)nv * c3, c3, 1,
                 Y, (long)nv * c2 * c3, c2 * c3, c3, 1,
                 (int)c2, (int)c3, nv, nv, 0};
        zgemm(c, gy, (long)tcn * nv);
        // Z[tl][i a][(j b)(k g)] = sum_n1 F1[tl][n1][i a] Y[tl][n1][(j b)(k g)]
        Zgemm gz{F1, nv * c1, 0, 1, c1,
                 Y, (long)nv * c2 * c3, 0, c2 * c3, 1,
                 Z, c1 * c2 * c3, 0, c2 * c3, 1,
                 (int)c1, (int)(c2 * c3), nv, 1, 0};
        zgemm(c, gz, tcn);
        const long nout = (long)tcn * n1 * n2 * n3;
        hipLaunchKernelGGL(k_spin3, dim3(nblocks_for(nout, 256)), dim3(256), 0, c->stream, s, (const double2 *)Z, n1,
                           n2, n3, t0, tcn, (double2 *)out);
        LAPH_HIP(hipGetLastError());
    }
    LAPH_API_END(c)
}

extern "C" int laph_baryon_correlator(laph_ctx_t c, const double *snk, const double *src, int n, int t0, double *out)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(snk && src && out && n > 0, LAPH_EINVAL, "bad arguments");
    LAPH_CHECK(t0 >= 0 && t0 < c->g.nt, LAPH_EINVAL, "t0 out of range");
    hipLaunchKernelGGL(k_baryon_corr, dim3(c->g.nt), dim3(256), 0, c->stream, (const double2 *)snk,
                       (const double2 *)src, n, c->g.nt, t0, (double2 *)out);
    LAPH_HIP(hipGetLastError());
    LAPH_API_END(c)
}

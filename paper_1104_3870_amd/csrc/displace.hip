// Covariant displacements of colour fields and their momentum-projected overlaps (Sec. II:
// displacement types D^(j) of the quark lines D^(j) S Omega^-1 S D^(k)dag; Sec. III.B: the
// momentum projection of the meson function).
//
// A displaced, momentum-projected meson function of LapH-smeared fields D^(j) V_s a and
// D^(k) V_s b factorises through the overlaps O[t][n][m] = sum_x e^{-ip.x} (D^(j) v_n)^dag
// (D^(k) v_m) of displaced eigenvectors: M = e^{-ip.(d_j + d_k)/2} sum c_ab conj(a_an)
// O_nm b_bm, so the fields are displaced once per eigenvector, not once per quark line.
#include <cmath>

#include "laph_impl.h"
#include "zgemm_mfma.h"

namespace {

// out[t][j][x] = (D v_j)(x) for colour fields in the eigenvector layout [Nt][n][Ns^3][3]:
// one lane per site (t, x) forms the path's link product W(x) once (W = U(x) U(x+e) ...
// U(x+(len-1)e), or the product of the adjoints backwards) and applies it to v_j at the
// far end for every j, so each link is read once per site, not once per vector
__global__ void k_displace(const double2 *__restrict__ U, const double2 *__restrict__ v, double2 *__restrict__ out,
                           int ns, int nt, int n, int dir, int sign, int len)
{
    const long V3 = (long)ns * ns * ns;
    const long q = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (q >= (long)nt * V3) return;
    const int t = (int)(q / V3);
    const long xyz = q - (long)t * V3;
    int c[3] = {(int)(xyz % ns), (int)((xyz / ns) % ns), (int)(xyz / ((long)ns * ns))};
    // W = product of the links from x to the far end, left to right
    double2 W[9];
#pragma unroll
    for (int e = 0; e < 9; e++) W[e] = make_double2((e % 4) == 0 ? 1.0 : 0.0, 0.0);
    int cur = c[dir];
    for (int k = 0; k < len; k++) {
        int s3[3] = {c[0], c[1], c[2]};
        const int nxt = ((cur + sign) % ns + ns) % ns;
        s3[dir] = sign > 0 ? cur : nxt;  // forward: U_d(cur); backward: U_d(cur - e)^dag
        const long site = s3[0] + (long)ns * (s3[1] + (long)ns * s3[2]) + V3 * t;
        const double2 *L = U + (site * 4 + dir) * 9;
        double2 Lm[9], R[9];
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) {
                const double2 u = sign > 0 ? L[a * 3 + b] : L[b * 3 + a];
                Lm[a * 3 + b] = sign > 0 ? u : make_double2(u.x, -u.y);
            }
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) {
                double2 acc = make_double2(0.0, 0.0);
#pragma unroll
                for (int m = 0; m < 3; m++) acc = cadd(acc, cmul(W[a * 3 + m], Lm[m * 3 + b]));
                R[a * 3 + b] = acc;
            }
#pragma unroll
        for (int e = 0; e < 9; e++) W[e] = R[e];
        cur = nxt;
    }
    int f[3] = {c[0], c[1], c[2]};
    f[dir] = cur;
    const long far = f[0] + (long)ns * (f[1] + (long)ns * f[2]);
    // four vectors' loads in flight per lane (each lane streams all n vectors of its site)
#pragma unroll 4
    for (int j = 0; j < n; j++) {
        const double2 *vf = v + (((long)t * n + j) * V3 + far) * 3;
        const double2 w0 = vf[0], w1 = vf[1], w2 = vf[2];
        double2 *o = out + (((long)t * n + j) * V3 + xyz) * 3;
#pragma unroll
        for (int a = 0; a < 3; a++)
            o[a] = cadd(cadd(cmul(W[a * 3], w0), cmul(W[a * 3 + 1], w1)), cmul(W[a * 3 + 2], w2));
    }
}

// phase[x] = exp(-2 pi i k.x / Ns) on one slice
__global__ void k_phase(double2 *ph, int ns, int k0, int k1, int k2)
{
    const long V3 = (long)ns * ns * ns;
    const long x = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (x >= V3) return;
    const int cx = (int)(x % ns), cy = (int)((x / ns) % ns), cz = (int)(x / ((long)ns * ns));
    // the integer phase index reduced mod Ns keeps the argument small and exact
    const long m = (((long)k0 * cx + (long)k1 * cy + (long)k2 * cz) % ns + ns) % ns;
    double s, c;
    sincospi(-2.0 * (double)m / ns, &s, &c);
    ph[x] = make_double2(c, s);
}

// O[t][n][m] = sum_{x, c} conj(a[t][n][x][c]) ph[x] b[t][m][x][c]: per slice the product
// A^dag (ph B) over K = 3 Ns^3 on the FP64 matrix cores; one block per slice and 64 x 64
// tile, the conjugate and the phase applied while staging
struct OverlapS {
    const double2 *a, *b, *ph;
    double2 *out;
    int M, N, K;  // na, nb, 3 Ns^3
    __device__ bool tile(long &bt, int &m0, int &n0) const
    {
        bt = blockIdx.z;
        m0 = blockIdx.x * zg::kTM;
        n0 = blockIdx.y * zg::kTN;
        return true;
    }
    // element q of a lane: e = lane + 256 q, row r = e / KT, k = e % KT (k fastest: KT
    // consecutive values of a row)
    template <int KT>
    struct Reg {
        double2 a[zg::kPer<KT>], b[zg::kPer<KT>], p[zg::kPer<KT>];
    };
    template <int KT>
    __device__ void load(Reg<KT> &g, long bt, int m0, int n0, int k0) const
    {
        static_assert(zg::kTM == zg::kTN, "one loop stages both operands");
#pragma unroll
        for (int q = 0; q < zg::kPer<KT>; q++) {
            const int e = threadIdx.x + 256 * q, r = e / KT, k = e - r * KT;
            const long kk = (long)k0 + k;
            // (explicit branches: a select between a global and a local zero would become a
            // select of addresses and a flat load)
            g.a[q] = g.b[q] = g.p[q] = make_double2(0.0, 0.0);
            if (kk < K) {
                if (m0 + r < M) g.a[q] = a[(bt * M + m0 + r) * (long)K + kk];
                if (n0 + r < N) g.b[q] = b[(bt * N + n0 + r) * (long)K + kk];
                g.p[q] = ph[kk / 3];
            }
        }
    }
    template <int KT>
    __device__ void put(zg::Tile<KT> &t, const Reg<KT> &g) const
    {
#pragma unroll
        for (int q = 0; q < zg::kPer<KT>; q++) {
            const int e = threadIdx.x + 256 * q, r = e / KT, k = e - r * KT;
            const double2 vb = cmul(g.p[q], g.b[q]);
            t.ar[k][r] = g.a[q].x;
            t.ai[k][r] = -g.a[q].y;
            t.br[k][r] = vb.x;
            t.bi[k][r] = vb.y;
        }
    }
    __device__ void store(long bt, int m, int n, double re, double im) const
    {
        out[(bt * M + m) * (long)N + n] = make_double2(re, im);
    }
};

// out[j][t][beta][p] = sum_m O[t][p][m] b[j][t][beta][m]; one lane per output element
__global__ void k_overlap_apply(const double2 *__restrict__ O, int na, int nb, const double2 *__restrict__ b,
                                long nrt, double2 *__restrict__ out, int nt)
{
    const long q = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (q >= nrt * 4 * na) return;
    const int p = (int)(q % na);
    const long rb = q / na;  // (j, t, beta)
    const int t = (int)((rb / 4) % nt);
    const double2 *orow = O + ((long)t * na + p) * nb;
    const double2 *bv = b + rb * nb;
    double2 acc = make_double2(0.0, 0.0);
    for (int m = 0; m < nb; m++) acc = cadd(acc, cmul(orow[m], bv[m]));
    out[q] = acc;
}

}  // namespace

extern "C" int laph_displace(laph_ctx_t c, const double *U, int dir, int sign, int length, const double *v, int n,
                             double *out)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(U && v && out && v != out && n > 0, LAPH_EINVAL, "bad arguments");
    LAPH_CHECK(dir >= 0 && dir < 3 && (sign == 1 || sign == -1) && length >= 0, LAPH_EINVAL,
               "direction 0..2, sign +-1, length >= 0");
    const long total = (long)c->g.nt * c->g.V3;
    hipLaunchKernelGGL(k_displace, dim3(nblocks_for(total, 256)), dim3(256), 0, c->stream, (const double2 *)U,
                       (const double2 *)v, (double2 *)out, c->g.ns, c->g.nt, n, dir, sign, length);
    LAPH_HIP(hipGetLastError());
    LAPH_API_END(c)
}

extern "C" int laph_mom_overlap(laph_ctx_t c, const double *a, int na, const double *b, int nb, const int *k,
                                double *out)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(a && b && k && out && na > 0 && nb > 0, LAPH_EINVAL, "bad arguments");
    const long V3 = c->g.V3;
    double2 *ph = (double2 *)ctx_named(c, "ovl.phase", sizeof(double2) * V3);
    hipLaunchKernelGGL(k_phase, dim3(nblocks_for(V3, 256)), dim3(256), 0, c->stream, ph, c->g.ns, k[0], k[1], k[2]);
    const unsigned gn = (na + zg::kTM - 1) / zg::kTM, gm = (nb + zg::kTN - 1) / zg::kTN;
    LAPH_CHECK(gm <= 65535 && c->g.nt <= 65535, LAPH_EINVAL, "too many fields for one launch");
    LAPH_CHECK(3 * V3 < (1L << 31), LAPH_EINVAL, "slice too large");
    OverlapS os{(const double2 *)a, (const double2 *)b, (const double2 *)ph, (double2 *)out, na, nb, (int)(3 * V3)};
    hipLaunchKernelGGL((zg::k_zgemm<16, OverlapS>), dim3(gn, gm, c->g.nt), dim3(256), 0, c->stream, os);
    LAPH_HIP(hipGetLastError());
    LAPH_API_END(c)
}

extern "C" int laph_overlap_apply(laph_ctx_t c, const double *O, int na, int nb, const double *b, int n, double *out)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(O && b && out && b != out && na > 0 && nb > 0 && n > 0, LAPH_EINVAL, "bad arguments");
    const long nrt = (long)n * c->g.nt;
    hipLaunchKernelGGL(k_overlap_apply, dim3(nblocks_for(nrt * 4 * na, 256)), dim3(256), 0, c->stream,
                       (const double2 *)O, na, nb, (const double2 *)b, nrt, (double2 *)out, c->g.nt);
    LAPH_HIP(hipGetLastError());
    LAPH_API_END(c)
}

// Clover term of the anisotropic Wilson-clover matrix and its inverse.
//
// In the chiral basis sigma_mn is block diagonal: sigma_k4 = diag(s_k, -s_k) and
// sigma_kl = -eps_klm diag(s_m, s_m) (s_m Pauli matrices).  With B_m = c_s F_mag,m
// (F_mag = (F_23, F_31, F_12)) and E_k = c_t F_k4 the two chiral 6x6 blocks of
//   A = d - 1/2 [c_t sum_k sigma_k4 F_k4 + c_s sum_{k<l} sigma_kl F_kl],  d = m0 + 1 + 3/xi,
// are  d + 1/2 sum_m s_m (x) G_m  with G = B - E (upper spins) and G = B + E (lower),
// i.e. d + 1/2 [[G_3, G_1 - i G_2], [G_1 + i G_2, -G_3]].
#include "laph_impl.h"

namespace {

struct M3 {
    double2 e[9];
};

__device__ inline M3 ld(const double2 *U, long s, int mu)
{
    M3 m;
    const double2 *p = U + (s * 4 + mu) * 9;
    for (int k = 0; k < 9; k++) m.e[k] = p[k];
    return m;
}
__device__ inline M3 mul(const M3 &a, const M3 &b)
{
    M3 r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double2 acc = cmake(0, 0);
            for (int k = 0; k < 3; k++) acc = cadd(acc, cmul(a.e[i * 3 + k], b.e[k * 3 + j]));
            r.e[i * 3 + j] = acc;
        }
    return r;
}
__device__ inline M3 dag(const M3 &a)
{
    M3 r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) r.e[i * 3 + j] = cmake(a.e[j * 3 + i].x, -a.e[j * 3 + i].y);
    return r;
}

__device__ inline long nbr(long s, int mu, int step, int ns, int nt)
{
    int c[4];
    long r = s;
    c[0] = (int)(r % ns);
    r /= ns;
    c[1] = (int)(r % ns);
    r /= ns;
    c[2] = (int)(r % ns);
    c[3] = (int)(r / ns);
    int L = mu == 3 ? nt : ns;
    c[mu] = (c[mu] + step + L) % L;
    return c[0] + (long)ns * (c[1] + (long)ns * (c[2] + (long)ns * c[3]));
}

// F_mn = traceless part of (Q - Q^dag)/(8i), Q the sum of the four leaves at s
__device__ M3 field_strength(const double2 *U, long s, int mu, int nu, int ns, int nt)
{
    long xpm = nbr(s, mu, 1, ns, nt), xpn = nbr(s, nu, 1, ns, nt);
    long xmm = nbr(s, mu, -1, ns, nt), xmn = nbr(s, nu, -1, ns, nt);
    long xmm_pn = nbr(xmm, nu, 1, ns, nt), xmm_mn = nbr(xmm, nu, -1, ns, nt), xmn_pm = nbr(xmn, mu, 1, ns, nt);
    M3 q1 = mul(mul(ld(U, s, mu), ld(U, xpm, nu)), mul(dag(ld(U, xpn, mu)), dag(ld(U, s, nu))));
    M3 q2 = mul(mul(ld(U, s, nu), dag(ld(U, xmm_pn, mu))), mul(dag(ld(U, xmm, nu)), ld(U, xmm, mu)));
    M3 q3 = mul(mul(dag(ld(U, xmm, mu)), dag(ld(U, xmm_mn, nu))), mul(ld(U, xmm_mn, mu), ld(U, xmn, nu)));
    M3 q4 = mul(mul(dag(ld(U, xmn, nu)), ld(U, xmn, mu)), mul(ld(U, xmn_pm, nu), dag(ld(U, s, mu))));
    M3 F;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            int a = i * 3 + j, b = j * 3 + i;
            double2 q = cadd(cadd(q1.e[a], q2.e[a]), cadd(q3.e[a], q4.e[a]));
            double2 qt = cadd(cadd(q1.e[b], q2.e[b]), cadd(q3.e[b], q4.e[b]));
            // (q - conj(qt)) / (8i) = -i/8 (q - conj(qt))
            double2 d = cmake(q.x - qt.x, q.y + qt.y);
            F.e[a] = cmake(d.y / 8.0, -d.x / 8.0);
        }
    double2 tr = cscale(cadd(cadd(F.e[0], F.e[4]), F.e[8]), 1.0 / 3.0);
    for (int i = 0; i < 3; i++) F.e[i * 4] = csub(F.e[i * 4], tr);
    return F;
}

// Gauss-Jordan inverse of a 6x6 complex matrix with partial pivoting (in place).
__device__ void invert6(double2 (&m)[6][6])
{
    double2 inv[6][6];
    for (int i = 0; i < 6; i++)
        for (int j = 0; j < 6; j++) inv[i][j] = cmake(i == j ? 1.0 : 0.0, 0.0);
    for (int col = 0; col < 6; col++) {
        int piv = col;
        double best = cnorm2(m[col][col]);
        for (int r = col + 1; r < 6; r++) {
            double v = cnorm2(m[r][col]);
            if (v > best) {
                best = v;
                piv = r;
            }
        }
        if (piv != col)
            for (int j = 0; j < 6; j++) {
                double2 t = m[col][j];
                m[col][j] = m[piv][j];
                m[piv][j] = t;
                t = inv[col][j];
                inv[col][j] = inv[piv][j];
                inv[piv][j] = t;
            }
        double2 p = cdiv(cmake(1.0, 0.0), m[col][col]);
        for (int j = 0; j < 6; j++) {
            m[col][j] = cmul(m[col][j], p);
            inv[col][j] = cmul(inv[col][j], p);
        }
        for (int r = 0; r < 6; r++) {
            if (r == col) continue;
            double2 f = m[r][col];
            for (int j = 0; j < 6; j++) {
                m[r][j] = csub(m[r][j], cmul(f, m[col][j]));
                inv[r][j] = csub(inv[r][j], cmul(f, inv[col][j]));
            }
        }
    }
    for (int i = 0; i < 6; i++)
        for (int j = 0; j < 6; j++) m[i][j] = inv[i][j];
}

__device__ void store_packed(double *dst, long stride, const double2 (&m)[6][6])
{
    for (int i = 0; i < 6; i++) dst[i * stride] = m[i][i].x;
    int e = 6;
    for (int i = 1; i < 6; i++)
        for (int j = 0; j < i; j++) {
            // Hermitian part of the computed matrix
            double2 v = cscale(cadd(m[i][j], cmake(m[j][i].x, -m[j][i].y)), 0.5);
            dst[e * stride] = v.x;
            dst[(e + 1) * stride] = v.y;
            e += 2;
        }
}

__global__ void k_clover_build(const double2 *__restrict__ U, double *__restrict__ clov, double *__restrict__ clinv,
                               int ns, int nt, long V, long Vh, double diag, double cs, double ct)
{
    long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (s >= V) return;
    long r = s;
    int x = (int)(r % ns);
    r /= ns;
    int y = (int)(r % ns);
    r /= ns;
    int z = (int)(r % ns);
    int t = (int)(r / ns);
    int par = (x + y + z + t) & 1;
    long cb = s >> 1;
    M3 F01 = field_strength(U, s, 0, 1, ns, nt);
    M3 F02 = field_strength(U, s, 0, 2, ns, nt);
    M3 F12 = field_strength(U, s, 1, 2, ns, nt);
    M3 F03 = field_strength(U, s, 0, 3, ns, nt);
    M3 F13 = field_strength(U, s, 1, 3, ns, nt);
    M3 F23 = field_strength(U, s, 2, 3, ns, nt);
    for (int blk = 0; blk < 2; blk++) {
        double sg = blk == 0 ? -1.0 : 1.0;  // G = B - E (upper), B + E (lower)
        double2 G[3][9];
        for (int e = 0; e < 9; e++) {
            G[0][e] = cadd(cscale(F12.e[e], cs), cscale(F03.e[e], sg * ct));   // B_1 = c_s F_23
            G[1][e] = cadd(cscale(F02.e[e], -cs), cscale(F13.e[e], sg * ct));  // B_2 = c_s F_31
            G[2][e] = cadd(cscale(F01.e[e], cs), cscale(F23.e[e], sg * ct));   // B_3 = c_s F_12
        }
        double2 m[6][6];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                int e = a * 3 + b;
                double dd = (a == b) ? diag : 0.0;
                m[a][b] = cadd(cmake(dd, 0), cscale(G[2][e], 0.5));
                m[3 + a][3 + b] = csub(cmake(dd, 0), cscale(G[2][e], 0.5));
                // 1/2 (G1 - i G2) and 1/2 (G1 + i G2); i*z = (-z.y, z.x)
                m[a][3 + b] = cscale(cmake(G[0][e].x + G[1][e].y, G[0][e].y - G[1][e].x), 0.5);
                m[3 + a][b] = cscale(cmake(G[0][e].x - G[1][e].y, G[0][e].y + G[1][e].x), 0.5);
            }
        store_packed(clov + ((long)(par * 72 + blk * 36)) * Vh + cb, Vh, m);
        invert6(m);
        store_packed(clinv + ((long)(par * 72 + blk * 36)) * Vh + cb, Vh, m);
    }
}

__global__ void k_d_to_f(const double *__restrict__ a, float *__restrict__ b, long n)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

}  // namespace

void clover_build(laph_ctx *c, const double *U, const laph_dirac *d, double *clov, double *clinv)
{
    double diag = d->m0 + 1.0 + 3.0 / d->xi;
    double cs = d->c_sw / d->xi, ct = d->c_sw * (1.0 + 1.0 / d->xi) / 2.0;
    hipLaunchKernelGGL(k_clover_build, dim3(nblocks_for(c->g.V, 128)), dim3(128), 0, c->stream,
                       (const double2 *)U, clov, clinv, c->g.ns, c->g.nt, c->g.V, c->g.Vh, diag, cs, ct);
    LAPH_HIP(hipGetLastError());
}

void clover_to_f32(laph_ctx *c, const double *cl, float *cl32)
{
    long n = 144 * c->g.Vh;
    hipLaunchKernelGGL(k_d_to_f, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, cl, cl32, n);
    LAPH_HIP(hipGetLastError());
}

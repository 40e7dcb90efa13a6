// Temporal gauge for the solver's operator.
//
// The Wilson-clover operator is gauge covariant: for site-local SU(3) rotations G(x),
// U'_mu(x) = G(x) U_mu(x) G(x + mu)^dag gives Omega' = G Omega G^dag, with the clover
// term rotating as A'(x) = G(x) A(x) G(x)^dag.  Solving Omega' x' = G eta and returning
// x = G^dag x' is the same solve.  With G(x, 0) = 1 and G(x, t + 1) = G(x, t) U_4(x, t),
// every time-direction link except those leaving the last slice becomes the unit matrix,
// which the multi-RHS hop then applies without a product (the links of the last slice
// carry the Polyakov line).
#include "laph_impl.h"

namespace {

// c = a b, 3x3 complex, row-major double2
__device__ __forceinline__ void mm3(const double2 *a, const double2 *b, double2 *c)
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double2 s = cmul(a[i * 3], b[j]);
            s = cadd(s, cmul(a[i * 3 + 1], b[3 + j]));
            s = cadd(s, cmul(a[i * 3 + 2], b[6 + j]));
            c[i * 3 + j] = s;
        }
}

// c = a b^dag
__device__ __forceinline__ void mmd3(const double2 *a, const double2 *b, double2 *c)
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double2 s = cmul(a[i * 3], make_double2(b[j * 3].x, -b[j * 3].y));
            s = cadd(s, cmul(a[i * 3 + 1], make_double2(b[j * 3 + 1].x, -b[j * 3 + 1].y)));
            s = cadd(s, cmul(a[i * 3 + 2], make_double2(b[j * 3 + 2].x, -b[j * 3 + 2].y)));
            c[i * 3 + j] = s;
        }
}

// one thread per spatial site walks the time slices: G(t = 0) = 1, G(t + 1) = G(t) U_4(t)
__global__ void k_tg_rotations(const double2 *__restrict__ U, double2 *__restrict__ G, long V3, int nt)
{
    long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (s >= V3) return;
    double2 g[9], n[9];
    for (int k = 0; k < 9; k++) g[k] = make_double2((k % 4 == 0) ? 1.0 : 0.0, 0.0);
    for (int t = 0; t < nt; t++) {
        long site = (long)t * V3 + s;
        for (int k = 0; k < 9; k++) G[site * 9 + k] = g[k];
        mm3(g, U + (site * 4 + 3) * 9, n);
        for (int k = 0; k < 9; k++) g[k] = n[k];
    }
}

// U'_mu(x) = G(x) U_mu(x) G(x + mu)^dag (periodic neighbours), one thread per link
__global__ void k_tg_links(const double2 *__restrict__ U, const double2 *__restrict__ G, double2 *__restrict__ Up,
                           int ns, int nt, long V)
{
    long l = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (l >= 4 * V) return;
    const long s = l >> 2;
    const int mu = (int)(l & 3);
    int x = (int)(s % ns);
    long r = s / ns;
    int y = (int)(r % ns);
    r /= ns;
    int z = (int)(r % ns);
    int t = (int)(r / ns);
    if (mu == 0) x = (x + 1) % ns;
    if (mu == 1) y = (y + 1) % ns;
    if (mu == 2) z = (z + 1) % ns;
    if (mu == 3) t = (t + 1) % nt;
    const long sn = x + (long)ns * (y + (long)ns * (z + (long)ns * t));
    double2 a[9];
    mm3(G + s * 9, U + l * 9, a);
    mmd3(a, G + sn * 9, Up + l * 9);
}

// psi[r][site][alpha][a] <- sum_b G[site][a][b] psi[r][site][alpha][b]  (dag: G^dag)
__global__ void k_tg_spinor(const double2 *__restrict__ G, const double2 *__restrict__ in, double2 *__restrict__ out,
                            long V, long n, int dag)
{
    long q = blockIdx.x * (long)blockDim.x + threadIdx.x;  // (rhs, site, alpha)
    if (q >= n) return;
    const long site = (q >> 2) % V;
    const double2 *g = G + site * 9;
    double2 v[3], o[3];
    for (int b = 0; b < 3; b++) v[b] = in[q * 3 + b];
    for (int a = 0; a < 3; a++) {
        double2 s = make_double2(0, 0);
        for (int b = 0; b < 3; b++) s = cadd(s, dag ? cconjmul(g[b * 3 + a], v[b]) : cmul(g[a * 3 + b], v[b]));
        o[a] = s;
    }
    for (int a = 0; a < 3; a++) out[q * 3 + a] = o[a];
}

}  // namespace

void tgauge_fix(laph_ctx *c, const double *U, double *G, double *Up)
{
    const long V = c->g.V, V3 = c->g.V3;
    hipLaunchKernelGGL(k_tg_rotations, dim3(nblocks_for(V3, 128)), dim3(128), 0, c->stream, (const double2 *)U,
                       (double2 *)G, V3, c->g.nt);
    LAPH_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_tg_links, dim3(nblocks_for(4 * V, 256)), dim3(256), 0, c->stream, (const double2 *)U,
                       (const double2 *)G, (double2 *)Up, c->g.ns, c->g.nt, V);
    LAPH_HIP(hipGetLastError());
}

void tgauge_spinor(laph_ctx *c, const double *G, const double *in, double *out, int nrhs, int dag)
{
    const long V = c->g.V, n = (long)nrhs * V * 4;
    hipLaunchKernelGGL(k_tg_spinor, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, (const double2 *)G,
                       (const double2 *)in, (double2 *)out, V, n, dag);
    LAPH_HIP(hipGetLastError());
}

// Conversions between the canonical ABI layouts and the device SoA layouts.
#include "laph_impl.h"

__global__ void k_links_to_eo(const double2 *__restrict__ U, double2 *__restrict__ g, int ns, int nt, long V,
                              long Vh)
{
    long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (s >= V) return;
    int x = (int)(s % ns);
    long r = s / ns;
    int y = (int)(r % ns);
    r /= ns;
    int z = (int)(r % ns);
    int t = (int)(r / ns);
    int par = (x + y + z + t) & 1;
    long cb = s >> 1;
    for (int mu = 0; mu < 4; mu++)
        for (int k = 0; k < 9; k++) g[((long)(mu * 2 + par) * 9 + k) * Vh + cb] = U[(s * 4 + mu) * 9 + k];
}

void links_to_eo(laph_ctx *c, const double *U, double2 *g64)
{
    long V = c->g.V;
    hipLaunchKernelGGL(k_links_to_eo, dim3(nblocks_for(V, 256)), dim3(256), 0, c->stream,
                       (const double2 *)U, g64, c->g.ns, c->g.nt, V, c->g.Vh);
    LAPH_HIP(hipGetLastError());
}

__global__ void k_d2_to_f2(const double2 *__restrict__ a, float2 *__restrict__ b, long n)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

void eo64_to_eo32(laph_ctx *c, const double2 *g64, float2 *g32, long n)
{
    hipLaunchKernelGGL(k_d2_to_f2, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, g64, g32, n);
    LAPH_HIP(hipGetLastError());
}

// canonical [R][V][4][3] -> parity halves [12][Vh][R]; gam = 4 applies gamma_4 (chiral
// basis: swaps the upper and lower spin pairs), gam = 5 applies gamma_5 = diag(1,1,-1,-1);
// G (may be null): a site-local colour rotation [V][3][3] applied first.
// One lane per (site, RHS) with the RHS fastest: the parity halves are written with
// consecutive RHS at consecutive addresses, every lane reads its site's 192-byte record.
__global__ void k_spinor_to_eo(const double2 *__restrict__ psi, int nrhs, int gam, double2 *__restrict__ ev,
                               double2 *__restrict__ od, int ns, long V, long Vh, const double2 *__restrict__ G)
{
    long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (tid >= V * nrhs) return;
    long s = tid / nrhs;
    int r = (int)(tid - s * nrhs);
    int x = (int)(s % ns);
    long q = s / ns;
    int y = (int)(q % ns);
    q /= ns;
    int z = (int)(q % ns);
    int t = (int)(q / ns);
    int par = (x + y + z + t) & 1;
    long cb = s >> 1;
    double2 *dst = par ? od : ev;
    const double2 *src = psi + ((long)r * V + s) * 12;
    double2 v[12];
    for (int k = 0; k < 12; k++) v[k] = src[k];
    if (G) {
        const double2 *g = G + s * 9;
        for (int a = 0; a < 4; a++) {
            double2 o[3];
            for (int col = 0; col < 3; col++)
                o[col] = cadd(cadd(cmul(g[col * 3], v[a * 3]), cmul(g[col * 3 + 1], v[a * 3 + 1])),
                              cmul(g[col * 3 + 2], v[a * 3 + 2]));
            for (int col = 0; col < 3; col++) v[a * 3 + col] = o[col];
        }
    }
    for (int a = 0; a < 4; a++) {
        int sa = (gam == 4) ? (a ^ 2) : a;
        double sg = (gam == 5 && a >= 2) ? -1.0 : 1.0;
        for (int col = 0; col < 3; col++)
            dst[((long)(a * 3 + col) * Vh + cb) * nrhs + r] = cscale(v[sa * 3 + col], sg);
    }
}

void spinor_to_eo(laph_ctx *c, const double *psi, int nrhs, int gam, double2 *even, double2 *odd, const double *G)
{
    long n = c->g.V * nrhs;
    hipLaunchKernelGGL(k_spinor_to_eo, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, (const double2 *)psi,
                       nrhs, gam, even, odd, c->g.ns, c->g.V, c->g.Vh, (const double2 *)G);
    LAPH_HIP(hipGetLastError());
}

// the inverse of k_spinor_to_eo, same lane order (reads of consecutive RHS coalesced);
// G (may be null): G^dag applied last
__global__ void k_spinor_from_eo(const double2 *__restrict__ ev, const double2 *__restrict__ od, int nrhs, int gam,
                                 double2 *__restrict__ psi, int ns, long V, long Vh, const double2 *__restrict__ G)
{
    long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (tid >= V * nrhs) return;
    long s = tid / nrhs;
    int r = (int)(tid - s * nrhs);
    int x = (int)(s % ns);
    long q = s / ns;
    int y = (int)(q % ns);
    q /= ns;
    int z = (int)(q % ns);
    int t = (int)(q / ns);
    int par = (x + y + z + t) & 1;
    long cb = s >> 1;
    const double2 *src = par ? od : ev;
    double2 *dst = psi + ((long)r * V + s) * 12;
    double2 v[12];
    for (int a = 0; a < 4; a++) {
        int sa = (gam == 4) ? (a ^ 2) : a;
        double sg = (gam == 5 && a >= 2) ? -1.0 : 1.0;
        for (int col = 0; col < 3; col++) v[a * 3 + col] = cscale(src[((long)(sa * 3 + col) * Vh + cb) * nrhs + r], sg);
    }
    if (G) {
        const double2 *g = G + s * 9;
        for (int a = 0; a < 4; a++) {
            double2 o[3];
            for (int col = 0; col < 3; col++)
                o[col] = cadd(cadd(cconjmul(g[col], v[a * 3]), cconjmul(g[3 + col], v[a * 3 + 1])),
                              cconjmul(g[6 + col], v[a * 3 + 2]));
            for (int col = 0; col < 3; col++) v[a * 3 + col] = o[col];
        }
    }
    for (int k = 0; k < 12; k++) dst[k] = v[k];
}

void spinor_from_eo(laph_ctx *c, const double2 *even, const double2 *odd, int nrhs, int gam, double *psi,
                    const double *G)
{
    long n = c->g.V * nrhs;
    hipLaunchKernelGGL(k_spinor_from_eo, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, even, odd, nrhs, gam,
                       (double2 *)psi, c->g.ns, c->g.V, c->g.Vh, (const double2 *)G);
    LAPH_HIP(hipGetLastError());
}

__global__ void k_smeared_to_soa(const double2 *__restrict__ U, double2 *__restrict__ us, long V)
{
    long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (s >= V) return;
    for (int k = 0; k < 3; k++)
        for (int e = 0; e < 9; e++) us[(long)(k * 9 + e) * V + s] = U[(s * 4 + k) * 9 + e];
}

void smeared_links_to_soa(laph_ctx *c, const double *U, double2 *us)
{
    hipLaunchKernelGGL(k_smeared_to_soa, dim3(nblocks_for(c->g.V, 256)), dim3(256), 0, c->stream,
                       (const double2 *)U, us, c->g.V);
    LAPH_HIP(hipGetLastError());
}

// Gauge-covariant 3D Laplacian (Sec. II) and its Chebyshev transform (Sec. IV), batched
// over all time slices.  The fused kernel computes
//     out = alpha * (Lap in) + beta * in + gamma * prev
// which is one step of T_k = 2 B T_{k-1} - T_{k-2}, B = 1 + c (Lap + lambda_C).
#include "laplace.h"

namespace {

// one lane per (slice t, spatial site); vectors of slice t start at base + t * stride
__global__ __launch_bounds__(256) void k_lap(const double2 *__restrict__ us, const double2 *__restrict__ in,
                                             long in_stride, const double2 *__restrict__ prev, long prev_stride,
                                             double2 *__restrict__ out, long out_stride, int ns, int nt, long V,
                                             double alpha, double beta, double gamma, const int *__restrict__ skip)
{
    unsigned b = xcd_block(blockIdx.x, gridDim.x);
    long s = (long)b * blockDim.x + threadIdx.x;
    if (s >= V) return;
    long V3 = V / nt;
    int t = (int)(s / V3);
    if (skip && skip[t]) return;
    long r = s - (long)t * V3;
    int x = (int)(r % ns);
    long q = r / ns;
    int y = (int)(q % ns);
    int z = (int)(q / ns);
    const double2 *vin = in + t * in_stride;
    double2 acc[3];
    double2 self[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        self[a] = vin[r * 3 + a];
        acc[a] = cscale(self[a], -6.0);
    }
#pragma unroll
    for (int k = 0; k < 3; k++) {
        int xp = x, yp = y, zp = z, xm = x, ym = y, zm = z;
        if (k == 0) {
            xp = x + 1 == ns ? 0 : x + 1;
            xm = x == 0 ? ns - 1 : x - 1;
        } else if (k == 1) {
            yp = y + 1 == ns ? 0 : y + 1;
            ym = y == 0 ? ns - 1 : y - 1;
        } else {
            zp = z + 1 == ns ? 0 : z + 1;
            zm = z == 0 ? ns - 1 : z - 1;
        }
        long rp = xp + (long)ns * (yp + (long)ns * zp);
        long rm = xm + (long)ns * (ym + (long)ns * zm);
        long sm = rm + (long)t * V3;
        double2 vp[3], vm[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            vp[a] = vin[rp * 3 + a];
            vm[a] = vin[rm * 3 + a];
        }
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int c = 0; c < 3; c++) {
                acc[a] = cadd(acc[a], cmul(us[(long)(k * 9 + a * 3 + c) * V + s], vp[c]));
                acc[a] = cadd(acc[a], cconjmul(us[(long)(k * 9 + c * 3 + a) * V + sm], vm[c]));
            }
    }
    double2 *vo = out + t * out_stride;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        double2 o = cadd(cscale(acc[a], alpha), cscale(self[a], beta));
        if (prev) o = cadd(o, cscale(prev[t * prev_stride + r * 3 + a], gamma));
        vo[r * 3 + a] = o;
    }
}

}  // namespace

void lap_fused(laph_ctx *c, const double2 *us, const double2 *in, long in_stride, const double2 *prev,
               long prev_stride, double2 *out, long out_stride, double alpha, double beta, double gamma,
               const int *skip)
{
    long V = c->g.V;
    hipLaunchKernelGGL(k_lap, dim3(nblocks_for(V, 256)), dim3(256), 0, c->stream, us, in, in_stride, prev,
                       prev_stride, out, out_stride, c->g.ns, c->g.nt, V, alpha, beta, gamma, skip);
    LAPH_HIP(hipGetLastError());
}

// out = T_order(B) in, B = 1 + cc (Lap + lamC); w0, w1 scratch of the same shape
void cheb_apply(laph_ctx *c, const double2 *us, const double2 *in, long in_stride, double2 *out, long out_stride,
                double2 *w0, double2 *w1, long w_stride, double lamL, double lamC, int order, const int *skip)
{
    double cc = 2.0 / (lamL - lamC);
    double b0 = 1.0 + cc * lamC;  // B = cc * Lap + b0
    if (order == 0) {
        lap_fused(c, us, in, in_stride, nullptr, 0, out, out_stride, 0.0, 1.0, 0.0, skip);
        return;
    }
    if (order == 1) {
        lap_fused(c, us, in, in_stride, nullptr, 0, out, out_stride, cc, b0, 0.0, skip);
        return;
    }
    // T_1 -> w0; then T_k = 2 B T_{k-1} - T_{k-2}, rotating buffers so T_order lands in out
    const double2 *tm2 = in;
    long s2 = in_stride;
    double2 *bufs[2] = {w0, w1};
    lap_fused(c, us, in, in_stride, nullptr, 0, w0, w_stride, cc, b0, 0.0, skip);
    const double2 *tm1 = w0;
    long s1 = w_stride;
    int nb = 1;
    for (int k = 2; k <= order; k++) {
        double2 *dst;
        long sd;
        if (k == order) {
            dst = out;
            sd = out_stride;
        } else {
            dst = bufs[nb];
            sd = w_stride;
            nb ^= 1;
        }
        lap_fused(c, us, tm1, s1, tm2, s2, dst, sd, 2.0 * cc, 2.0 * b0, -1.0, skip);
        tm2 = tm1;
        s2 = s1;
        tm1 = dst;
        s1 = sd;
    }
}

static double2 *prepare_soa(laph_ctx *c, const double *U)
{
    double2 *us = (double2 *)ctx_named(c, "lap.us", (size_t)27 * c->g.V * 16);
    smeared_links_to_soa(c, U, us);
    return us;
}

extern "C" int laph_laplacian_apply(laph_ctx_t c, const double *U, const double *v, double *out)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(U && v && out && v != out, LAPH_EINVAL, "bad arguments");
    double2 *us = prepare_soa(c, U);
    long V3 = c->g.V3;
    // one launch covers all slices: a "slice stride" of V3*3 makes the layout contiguous
    lap_fused(c, us, (const double2 *)v, V3 * 3, nullptr, 0, (double2 *)out, V3 * 3, 1.0, 0.0, 0.0, nullptr);
    LAPH_API_END(c)
}

extern "C" int laph_chebyshev_apply(laph_ctx_t c, const double *U, double lamL, double lamC, int order,
                                    const double *v, double *out)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(U && v && out && v != out && order >= 0 && lamL > lamC, LAPH_EINVAL, "bad arguments");
    double2 *us = prepare_soa(c, U);
    long V3 = c->g.V3;
    size_t bytes = (size_t)c->g.V * 3 * 16;
    double2 *w0 = (double2 *)ctx_named(c, "cheb.w0", bytes), *w1 = (double2 *)ctx_named(c, "cheb.w1", bytes);
    cheb_apply(c, us, (const double2 *)v, V3 * 3, (double2 *)out, V3 * 3, w0, w1, V3 * 3, lamL, lamC, order, nullptr);
    LAPH_API_END(c)
}

// Spatial stout smearing (Sec. II: stout links with spatial staples only, time links
// untouched).  exp(iQ) uses the Cayley-Hamilton closed form of Morningstar & Peardon,
// Phys. Rev. D 69, 054501 (2004): exp(iQ) = f0 + f1 Q + f2 Q^2 with f_j from c0 = det Q,
// c1 = tr Q^2 / 2.
#include <cmath>

#include "laph_impl.h"

namespace {

struct Mat {
    double2 e[9];
};

__device__ inline Mat mload(const double2 *U, long s, int mu)
{
    Mat m;
    for (int k = 0; k < 9; k++) m.e[k] = U[(s * 4 + mu) * 9 + k];
    return m;
}
__device__ inline Mat mmul(const Mat &a, const Mat &b)
{
    Mat r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double2 acc = cmake(0, 0);
            for (int k = 0; k < 3; k++) acc = cadd(acc, cmul(a.e[i * 3 + k], b.e[k * 3 + j]));
            r.e[i * 3 + j] = acc;
        }
    return r;
}
__device__ inline Mat mdag(const Mat &a)
{
    Mat r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) r.e[i * 3 + j] = cmake(a.e[j * 3 + i].x, -a.e[j * 3 + i].y);
    return r;
}

__device__ inline long shift(long s, int mu, int step, int ns)
{
    int c[4];
    long r = s;
    c[0] = (int)(r % ns);
    r /= ns;
    c[1] = (int)(r % ns);
    r /= ns;
    c[2] = (int)(r % ns);
    c[3] = (int)(r / ns);
    c[mu] = (c[mu] + step + ns) % ns;  // spatial directions only
    return c[0] + (long)ns * (c[1] + (long)ns * (c[2] + (long)ns * c[3]));
}

// exp(iQ) for Hermitian traceless Q
__device__ Mat expiq(const Mat &Q)
{
    Mat Q2 = mmul(Q, Q);
    double c1 = 0.5 * (Q2.e[0].x + Q2.e[4].x + Q2.e[8].x);
    Mat Q3 = mmul(Q2, Q);
    double c0 = (Q3.e[0].x + Q3.e[4].x + Q3.e[8].x) / 3.0;
    double2 f0, f1, f2;
    if (c1 < 1e-14) {
        // |Q| tiny: Taylor series through Q^4 with Q^3 = c1 Q + c0 (Cayley-Hamilton)
        f0 = cmake(1.0, -c0 / 6.0);
        f1 = cmake(c0 / 24.0, 1.0 - c1 / 6.0);
        f2 = cmake(-0.5 + c1 / 24.0, 0.0);
    } else {
        bool neg = c0 < 0;
        double c0a = fabs(c0);
        double c0max = 2.0 * pow(c1 / 3.0, 1.5);
        double ratio = fmin(1.0, c0a / c0max);
        double theta = acos(ratio);
        double u = sqrt(c1 / 3.0) * cos(theta / 3.0);
        double w = sqrt(c1) * sin(theta / 3.0);
        double u2 = u * u, w2 = w * w;
        double xi0 = fabs(w) < 0.05 ? 1.0 - w2 / 6.0 * (1.0 - w2 / 20.0 * (1.0 - w2 / 42.0)) : sin(w) / w;
        double cw = cos(w);
        double2 e2iu = cmake(cos(2 * u), sin(2 * u));
        double2 emiu = cmake(cos(u), -sin(u));
        double2 h0 = cadd(cscale(e2iu, u2 - w2), cmul(emiu, cmake(8 * u2 * cw, 2 * u * (3 * u2 + w2) * xi0)));
        double2 h1 = csub(cscale(e2iu, 2 * u), cmul(emiu, cmake(2 * u * cw, -(3 * u2 - w2) * xi0)));
        double2 h2 = csub(e2iu, cmul(emiu, cmake(cw, 3 * u * xi0)));
        double den = 9 * u2 - w2;
        f0 = cscale(h0, 1.0 / den);
        f1 = cscale(h1, 1.0 / den);
        f2 = cscale(h2, 1.0 / den);
        if (neg) {  // f_j(-c0) = (-1)^j conj(f_j(c0))
            f0 = cmake(f0.x, -f0.y);
            f1 = cmake(-f1.x, f1.y);
            f2 = cmake(f2.x, -f2.y);
        }
    }
    Mat E;
    for (int k = 0; k < 9; k++) E.e[k] = cadd(cmul(f1, Q.e[k]), cmul(f2, Q2.e[k]));
    for (int i = 0; i < 3; i++) E.e[i * 4] = cadd(E.e[i * 4], f0);
    return E;
}

__global__ void k_stout(const double2 *__restrict__ in, double2 *__restrict__ out, int ns, long V, double rho)
{
    long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (tid >= V * 4) return;
    long s = tid >> 2;
    int k = (int)(tid & 3);
    if (k == 3) {  // time link: copy
        for (int e = 0; e < 9; e++) out[(s * 4 + 3) * 9 + e] = in[(s * 4 + 3) * 9 + e];
        return;
    }
    Mat C;
    for (int e = 0; e < 9; e++) C.e[e] = cmake(0, 0);
    for (int j = 0; j < 3; j++) {
        if (j == k) continue;
        long sj = shift(s, j, 1, ns), sk = shift(s, k, 1, ns), smj = shift(s, j, -1, ns);
        long smjk = shift(smj, k, 1, ns);
        Mat up = mmul(mmul(mload(in, s, j), mload(in, sj, k)), mdag(mload(in, sk, j)));
        Mat dn = mmul(mmul(mdag(mload(in, smj, j)), mload(in, smj, k)), mload(in, smjk, j));
        for (int e = 0; e < 9; e++) C.e[e] = cadd(C.e[e], cadd(up.e[e], dn.e[e]));
    }
    Mat Uk = mload(in, s, k);
    Mat Om = mmul(C, mdag(Uk));
    for (int e = 0; e < 9; e++) Om.e[e] = cscale(Om.e[e], rho);
    // Q = (i/2)(Om^dag - Om) - (i/6) tr(Om^dag - Om)
    Mat Q;
    double2 tr = cmake(0, 0);
    for (int i = 0; i < 3; i++) {
        double2 d = csub(cmake(Om.e[i * 4].x, -Om.e[i * 4].y), Om.e[i * 4]);
        tr = cadd(tr, d);
    }
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double2 d = csub(cmake(Om.e[j * 3 + i].x, -Om.e[j * 3 + i].y), Om.e[i * 3 + j]);
            Q.e[i * 3 + j] = cmake(-0.5 * d.y, 0.5 * d.x);  // (i/2) d
        }
    for (int i = 0; i < 3; i++) Q.e[i * 4] = csub(Q.e[i * 4], cmake(-tr.y / 6.0, tr.x / 6.0));
    Mat E = mmul(expiq(Q), Uk);
    for (int e = 0; e < 9; e++) out[(s * 4 + k) * 9 + e] = E.e[e];
}

}  // namespace

void stout_smear_device(laph_ctx *c, const double *U, double rho, int nsteps, double *out)
{
    long V = c->g.V;
    size_t bytes = (size_t)V * 36 * 16;
    double2 *tmp = (double2 *)ctx_named(c, "stout.tmp", bytes);
    if (nsteps <= 0) {
        LAPH_HIP(hipMemcpyAsync(out, U, bytes, hipMemcpyDeviceToDevice, c->stream));
        return;
    }
    // ping-pong so that the last step lands in out
    const double2 *src = (const double2 *)U;
    for (int st = 0; st < nsteps; st++) {
        double2 *dst = ((nsteps - 1 - st) % 2 == 0) ? (double2 *)out : tmp;
        hipLaunchKernelGGL(k_stout, dim3(nblocks_for(V * 4, 128)), dim3(128), 0, c->stream, src, dst, c->g.ns, V,
                           rho);
        LAPH_HIP(hipGetLastError());
        src = dst;
    }
}

extern "C" int laph_stout_smear(laph_ctx_t c, const double *U, const laph_stout *st, double *out)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(U && st && out && U != out, LAPH_EINVAL, "bad arguments");
    LAPH_CHECK(st->nsteps >= 0 && std::isfinite(st->rho), LAPH_EINVAL, "bad stout parameters");
    stout_smear_device(c, U, st->rho, st->nsteps, out);
    LAPH_API_END(c)
}

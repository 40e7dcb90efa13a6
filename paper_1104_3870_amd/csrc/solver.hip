// dirac_solve: Omega x = eta through the even-odd Schur system (Sec. IV: BiCGStab with
// even-odd preconditioning, mixed precision, CG on the normal equations as fallback).
//
//   K x = b with b = gamma_4 eta (since Omega = gamma_4 K),
//   M = 1 - A_oo^-1 D_oe A_ee^-1 D_eo,  bhat = A_oo^-1 (b_o - D_oe A_ee^-1 b_e),
//   M x_o = bhat,  x_e = A_ee^-1 (b_e - D_eo x_o).
// R right-hand sides are iterated together, each with its own Krylov scalars (BiCGStab, or
// CG on the normal equations of M, the form used near the critical mass, where BiCGStab
// diverges); a converged right-hand side is frozen by its mask.  Lower-precision inner
// iterations keep the solution increment in FP32 and fold it into the FP64 solution at
// every reliable update, which also replaces the iterated residual by the FP64 true
// residual of M.
// Every answer is judged by the FP64 true residual |b - K x| / |b| of the full system.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include <complex>

#include "dslash_mr.h"
#include "ptnet.h"
#include "spinor_io.h"

// largest power-of-two block (<= 32) the hopping kernels of this precision can address
static int max_block_rhs(laph_ctx *c, int prec)
{
    if (prec != LAPH_PREC_F64) return lds_max_rhs(c, prec);
    int R = 32;
    while (R >= 1 && (unsigned long long)c->g.Vh * R * sizeof(double2) >= (1ull << 32)) R /= 2;
    return R;
}

namespace {

int laph_verbose_level()
{
    static int v = -1;
    if (v < 0) {
        const char *e = getenv("LAPH_VERBOSE");
        v = (e && *e) ? atoi(e) : 0;
    }
    return v;
}
bool laph_verbose() { return laph_verbose_level() > 0; }

constexpr int kBS = 256;
constexpr int kMaxBlocks = 1024;


struct Vec {
    void *d = nullptr;
    float *n = nullptr;  // per-site scale (FP16 storage only)
};

inline unsigned red_blocks(long n) { return (unsigned)std::min<long>(kMaxBlocks, (n + kBS - 1) / kBS); }

// reduce NV doubles per right-hand side over the block; lanes with equal tid % R share r
template <int NV>
__device__ __forceinline__ void block_partial(double (&v)[NV], int R, double *partial)
{
    for (int off = 32; off >= R; off >>= 1)
#pragma unroll
        for (int k = 0; k < NV; k++) v[k] += __shfl_down(v[k], off, 64);
    __shared__ double lds[kBS / 64][32][NV];
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < R)
#pragma unroll
        for (int k = 0; k < NV; k++) lds[wave][lane][k] = v[k];
    __syncthreads();
    if ((int)threadIdx.x < R) {
#pragma unroll
        for (int k = 0; k < NV; k++) {
            double s = 0;
            for (int w = 0; w < kBS / 64; w++) s += lds[w][threadIdx.x][k];
            partial[((long)blockIdx.x * R + threadIdx.x) * NV + k] = s;
        }
    }
}

// deterministic sum of the partials of right-hand side r (one block per r)
template <int NV>
__device__ __forceinline__ void sum_partials(const double *partial, int nblk, int R, int r, double (&out)[NV])
{
    __shared__ double lds[kBS][NV];
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; k++) v[k] = 0;
    for (int b = threadIdx.x; b < nblk; b += kBS)
#pragma unroll
        for (int k = 0; k < NV; k++) v[k] += partial[((long)b * R + r) * NV + k];
#pragma unroll
    for (int k = 0; k < NV; k++) lds[threadIdx.x][k] = v[k];
    __syncthreads();
    for (int s = kBS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int k = 0; k < NV; k++) lds[threadIdx.x][k] += lds[threadIdx.x + s][k];
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < NV; k++) out[k] = lds[0][k];
}

// load / store a whole site-spinor as doubles (the BLAS arithmetic is FP64)
template <class SP>
__device__ __forceinline__ void ld_site(const Vec &v, long Vh, int R, long i, int r, Cx<double> (&o)[12])
{
    ld_spinor12<SP, double>((const typename SP::E *)v.d, v.n, Vh, R, i, r, o);
}
template <class SP>
__device__ __forceinline__ void st_site(Vec &v, long Vh, int R, long i, int r, const Cx<double> (&o)[12])
{
    st_spinor12<SP, double>((typename SP::E *)v.d, v.n, Vh, R, i, r, o);
}

// CG directions whose steps the solution increment still owes, latest first: d[0] takes
// the current alpha, d[j] (j >= 1) the alpha of j iterations back
struct Dirs {
    Vec d[kMaxDirs];
    int n = 0;
};

// o += sum_{j < n} coef_j d_j (static indices: the list stays in kernel arguments)
template <class SP>
__device__ __forceinline__ void add_steps(const Dirs &dirs, int n, const Scal &s, long Vh, int R, long i, int r,
                                          Cx<double> (&o)[12])
{
#pragma unroll
    for (int j = 0; j < kMaxDirs; j++) {
        if (j >= n) break;
        const double al = j ? s.alpha_prev[j - 1] : s.alpha.x;
        Cx<double> b[12];
        ld_site<SP>(dirs.d[j], Vh, R, i, r, b);
#pragma unroll
        for (int k = 0; k < 12; k++) o[k] = o[k] + al * b[k];
    }
}

__device__ __forceinline__ double2 c2(Cx<double> a) { return make_double2(a.re, a.im); }
__device__ __forceinline__ Cx<double> cx(double2 a) { return {a.x, a.y}; }

// ------------------------------------------------------------------ BiCGStab kernels
// r = r0 = p = convert(rhi); x = 0; partial |r|^2
template <class SP, class XP>
__global__ __launch_bounds__(kBS) void k_bicg_init(Vec rhi, Vec r, Vec r0, Vec p, Vec x, long Vh, int R,
                                                   double *partial, const Scal *sc)
{
    double acc[1] = {0};
    long n = Vh * R, stride = (long)gridDim.x * kBS;
    int rr = (int)((blockIdx.x * (long)kBS + threadIdx.x) % R);
    for (long tid = blockIdx.x * (long)kBS + threadIdx.x; tid < n; tid += stride) {
        long i = tid / R;
        Cx<double> v[12], z[12];
        if (!sc[rr].active) {
            // the increment of a frozen right-hand side is folded at the end: keep it zero
#pragma unroll
            for (int k = 0; k < 12; k++) z[k] = {0, 0};
            st_site<XP>(x, Vh, R, i, rr, z);
            continue;
        }
        ld_site<S64>(rhi, Vh, R, i, rr, v);
        st_site<SP>(r, Vh, R, i, rr, v);
        ld_site<SP>(r, Vh, R, i, rr, v);  // the value actually stored
        st_site<SP>(r0, Vh, R, i, rr, v);
        st_site<SP>(p, Vh, R, i, rr, v);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            z[k] = {0, 0};
            acc[0] += v[k].re * v[k].re + v[k].im * v[k].im;
        }
        st_site<XP>(x, Vh, R, i, rr, z);
    }
    block_partial<1>(acc, R, partial);
}

__global__ void k_fin_init(const double *partial, int nblk, int R, Scal *sc)
{
    int r = blockIdx.x;
    double s[1];
    sum_partials<1>(partial, nblk, R, r, s);
    if (threadIdx.x == 0 && sc[r].active) {
        sc[r].rho = make_double2(s[0], 0);
        sc[r].r2 = s[0];
    }
}

// partial <a, b> (complex)
template <class SP>
__global__ __launch_bounds__(kBS) void k_dot(Vec a, Vec b, long Vh, int R, double *partial)
{
    double acc[2] = {0, 0};
    long n = Vh * R, stride = (long)gridDim.x * kBS;
    int rr = (int)((blockIdx.x * (long)kBS + threadIdx.x) % R);
    for (long tid = blockIdx.x * (long)kBS + threadIdx.x; tid < n; tid += stride) {
        long i = tid / R;
        Cx<double> u[12], w[12];
        ld_site<SP>(a, Vh, R, i, rr, u);
        ld_site<SP>(b, Vh, R, i, rr, w);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            acc[0] += u[k].re * w[k].re + u[k].im * w[k].im;
            acc[1] += u[k].re * w[k].im - u[k].im * w[k].re;
        }
    }
    block_partial<2>(acc, R, partial);
}

__global__ void k_fin_alpha(const double *partial, int nblk, int R, Scal *sc)
{
    int r = blockIdx.x;
    double s[2];
    sum_partials<2>(partial, nblk, R, r, s);
    if (threadIdx.x) return;
    Scal &q = sc[r];
    double2 den = make_double2(s[0], s[1]);
    if (!q.active) {
        q.alpha = make_double2(0, 0);
        return;
    }
    if (cnorm2(den) == 0.0 || !std::isfinite(den.x) || !std::isfinite(den.y)) {
        q.alpha = make_double2(0, 0);
        q.breakdown = 1;
        q.active = 0;
        return;
    }
    q.alpha = cdiv(q.rho, den);
}

// s = r - alpha v
template <class SP>
__global__ __launch_bounds__(kBS) void k_s_update(Vec r, Vec v, Vec s, long Vh, int R, const Scal *sc)
{
    long n = Vh * R;
    long tid = blockIdx.x * (long)kBS + threadIdx.x;
    if (tid >= n) return;
    long i = tid / R;
    int rr = (int)(tid - i * R);
    if (!sc[rr].active) return;
    Cx<double> al = cx(sc[rr].alpha), a[12], b[12];
    ld_site<SP>(r, Vh, R, i, rr, a);
    ld_site<SP>(v, Vh, R, i, rr, b);
#pragma unroll
    for (int k = 0; k < 12; k++) a[k] = a[k] - al * b[k];
    st_site<SP>(s, Vh, R, i, rr, a);
}

// partial <t, s> and |t|^2
template <class SP>
__global__ __launch_bounds__(kBS) void k_dot_ts(Vec t, Vec s, long Vh, int R, double *partial)
{
    double acc[3] = {0, 0, 0};
    long n = Vh * R, stride = (long)gridDim.x * kBS;
    int rr = (int)((blockIdx.x * (long)kBS + threadIdx.x) % R);
    for (long tid = blockIdx.x * (long)kBS + threadIdx.x; tid < n; tid += stride) {
        long i = tid / R;
        Cx<double> u[12], w[12];
        ld_site<SP>(t, Vh, R, i, rr, u);
        ld_site<SP>(s, Vh, R, i, rr, w);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            acc[0] += u[k].re * w[k].re + u[k].im * w[k].im;
            acc[1] += u[k].re * w[k].im - u[k].im * w[k].re;
            acc[2] += u[k].re * u[k].re + u[k].im * u[k].im;
        }
    }
    block_partial<3>(acc, R, partial);
}

__global__ void k_fin_omega(const double *partial, int nblk, int R, Scal *sc)
{
    int r = blockIdx.x;
    double s[3];
    sum_partials<3>(partial, nblk, R, r, s);
    if (threadIdx.x) return;
    Scal &q = sc[r];
    if (!q.active) {
        q.omega = make_double2(0, 0);
        return;
    }
    if (!(s[2] > 0.0) || !std::isfinite(s[2])) {
        q.omega = make_double2(0, 0);
        q.breakdown = 1;
        q.active = 0;
        return;
    }
    q.omega = make_double2(s[0] / s[2], s[1] / s[2]);
}

// x += alpha p + omega s;  r = s - omega t;  partial <r0, r>, |r|^2
template <class SP, class XP>
__global__ __launch_bounds__(kBS) void k_xr_update(Vec x, Vec p, Vec s, Vec t, Vec r, Vec r0, long Vh, int R,
                                                   double *partial, const Scal *sc)
{
    double acc[3] = {0, 0, 0};
    long n = Vh * R, stride = (long)gridDim.x * kBS;
    int rr = (int)((blockIdx.x * (long)kBS + threadIdx.x) % R);
    bool act = sc[rr].active;
    Cx<double> al = cx(sc[rr].alpha), om = cx(sc[rr].omega);
    for (long tid = blockIdx.x * (long)kBS + threadIdx.x; tid < n; tid += stride) {
        if (!act) break;
        long i = tid / R;
        Cx<double> xv[12], pv[12], sv[12], tv[12], z[12];
        ld_site<XP>(x, Vh, R, i, rr, xv);
        ld_site<SP>(p, Vh, R, i, rr, pv);
        ld_site<SP>(s, Vh, R, i, rr, sv);
#pragma unroll
        for (int k = 0; k < 12; k++) xv[k] = xv[k] + al * pv[k] + om * sv[k];
        st_site<XP>(x, Vh, R, i, rr, xv);
        ld_site<SP>(t, Vh, R, i, rr, tv);
#pragma unroll
        for (int k = 0; k < 12; k++) sv[k] = sv[k] - om * tv[k];
        st_site<SP>(r, Vh, R, i, rr, sv);
        ld_site<SP>(r, Vh, R, i, rr, sv);  // stored value
        ld_site<SP>(r0, Vh, R, i, rr, z);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            acc[0] += z[k].re * sv[k].re + z[k].im * sv[k].im;
            acc[1] += z[k].re * sv[k].im - z[k].im * sv[k].re;
            acc[2] += sv[k].re * sv[k].re + sv[k].im * sv[k].im;
        }
    }
    block_partial<3>(acc, R, partial);
}

// rho_new = <r0, r>, beta = (rho_new / rho)(alpha / omega), |r|^2; with hi_conv the
// iterated residual alone may declare convergence (plain FP64 iteration)
__global__ void k_fin_beta(const double *partial, int nblk, int R, Scal *sc, int hi_conv)
{
    int r = blockIdx.x;
    double s[3];
    sum_partials<3>(partial, nblk, R, r, s);
    if (threadIdx.x) return;
    Scal &q = sc[r];
    if (!q.active) {
        q.beta = make_double2(0, 0);
        return;
    }
    double2 rn = make_double2(s[0], s[1]);
    q.iters += 1;
    q.r2 = s[2];
    if (!std::isfinite(s[2]) || cnorm2(q.rho) == 0.0 || cnorm2(q.omega) == 0.0) {
        q.breakdown = 1;
        q.active = 0;
        q.beta = make_double2(0, 0);
        return;
    }
    q.beta = cmul(cdiv(rn, q.rho), cdiv(q.alpha, q.omega));
    q.rho = rn;
    if (hi_conv && s[2] <= q.tol2) q.active = 0;
}

// p = r + beta (p - omega v)
template <class SP>
__global__ __launch_bounds__(kBS) void k_p_update(Vec p, Vec r, Vec v, long Vh, int R, const Scal *sc)
{
    long n = Vh * R;
    long tid = blockIdx.x * (long)kBS + threadIdx.x;
    if (tid >= n) return;
    long i = tid / R;
    int rr = (int)(tid - i * R);
    if (!sc[rr].active) return;
    Cx<double> be = cx(sc[rr].beta), om = cx(sc[rr].omega), pv[12], rv[12], vv[12];
    ld_site<SP>(p, Vh, R, i, rr, pv);
    ld_site<SP>(r, Vh, R, i, rr, rv);
    ld_site<SP>(v, Vh, R, i, rr, vv);
#pragma unroll
    for (int k = 0; k < 12; k++) pv[k] = rv[k] + be * (pv[k] - om * vv[k]);
    st_site<SP>(p, Vh, R, i, rr, pv);
}

// ------------------------------------------------------------ FP64 / reliable updates
// xhi += xlo; xlo = 0 (right-hand sides with mask set, or all when all_rhs)
template <class XP>
__global__ __launch_bounds__(kBS) void k_fold_x(Vec xhi, Vec xlo, long Vh, int R, const Scal *sc, int all_rhs)
{
    long n = Vh * R;
    long tid = blockIdx.x * (long)kBS + threadIdx.x;
    if (tid >= n) return;
    long i = tid / R;
    int rr = (int)(tid - i * R);
    if (!all_rhs && !sc[rr].active) return;
    Cx<double> a[12], b[12], z[12];
    ld_site<S64>(xhi, Vh, R, i, rr, a);
    ld_site<XP>(xlo, Vh, R, i, rr, b);
#pragma unroll
    for (int k = 0; k < 12; k++) {
        a[k] = a[k] + b[k];
        z[k] = {0, 0};
    }
    st_site<S64>(xhi, Vh, R, i, rr, a);
    st_site<XP>(xlo, Vh, R, i, rr, z);
}

// the same fold with the steps the direction update still owes x:
// xhi += xlo + sum_j coef_j d_j (right-hand sides with mask set)
template <class XP, class SP>
__global__ __launch_bounds__(kBS) void k_fold_x_step(Vec xhi, Vec xlo, Dirs dirs, long Vh, int R, const Scal *sc)
{
    long n = Vh * R;
    long tid = blockIdx.x * (long)kBS + threadIdx.x;
    if (tid >= n) return;
    long i = tid / R;
    int rr = (int)(tid - i * R);
    if (!sc[rr].active) return;
    Cx<double> a[12], b[12], z[12];
    ld_site<S64>(xhi, Vh, R, i, rr, a);
    ld_site<XP>(xlo, Vh, R, i, rr, b);
#pragma unroll
    for (int k = 0; k < 12; k++) {
        a[k] = a[k] + b[k];
        z[k] = {0, 0};
    }
    add_steps<SP>(dirs, dirs.n, sc[rr], Vh, R, i, rr, a);
    st_site<S64>(xhi, Vh, R, i, rr, a);
    st_site<XP>(xlo, Vh, R, i, rr, z);
}

// r = b - m (FP64; m.d null: m = 0), partial |r|^2; restricted to masked right-hand sides
// unless all_rhs; with rlo.d set also r converted to the storage precision SP (r.d null:
// that conversion alone is stored)
template <class SP>
__global__ __launch_bounds__(kBS) void k_resid64(Vec b, Vec m, Vec r, Vec rlo, long Vh, int R, double *partial,
                                                 const Scal *sc, int all_rhs)
{
    double acc[1] = {0};
    long n = Vh * R, stride = (long)gridDim.x * kBS;
    int rr = (int)((blockIdx.x * (long)kBS + threadIdx.x) % R);
    bool act = all_rhs || sc[rr].active;
    for (long tid = blockIdx.x * (long)kBS + threadIdx.x; tid < n; tid += stride) {
        if (!act) break;
        long i = tid / R;
        Cx<double> a[12], c[12];
        ld_site<S64>(b, Vh, R, i, rr, a);
        if (m.d) {
            ld_site<S64>(m, Vh, R, i, rr, c);
        } else {
#pragma unroll
            for (int k = 0; k < 12; k++) c[k] = {0, 0};
        }
#pragma unroll
        for (int k = 0; k < 12; k++) {
            a[k] = a[k] - c[k];
            acc[0] += a[k].re * a[k].re + a[k].im * a[k].im;
        }
        if (r.d) st_site<S64>(r, Vh, R, i, rr, a);
        if (rlo.d) st_site<SP>(rlo, Vh, R, i, rr, a);
    }
    block_partial<1>(acc, R, partial);
}

// mode 0: r2hi = sum, and mask off converged (r2hi <= tol2); mode 1: b2 = sum
// the steps the direction update still owes x go into the increment:
// xlo += sum_j coef_j d_j (right-hand sides with mask set)
template <class XP, class SP>
__global__ __launch_bounds__(kBS) void k_owe_xlo(Vec xlo, Dirs dirs, long Vh, int R, const Scal *sc)
{
    long n = Vh * R;
    long tid = blockIdx.x * (long)kBS + threadIdx.x;
    if (tid >= n) return;
    long i = tid / R;
    int rr = (int)(tid - i * R);
    if (!sc[rr].active) return;
    Cx<double> a[12];
    ld_site<XP>(xlo, Vh, R, i, rr, a);
    add_steps<SP>(dirs, dirs.n, sc[rr], Vh, R, i, rr, a);
    st_site<XP>(xlo, Vh, R, i, rr, a);
}

__global__ void k_fin_r2hi(const double *partial, int nblk, int R, Scal *sc, int mode)
{
    int r = blockIdx.x;
    double s[1];
    sum_partials<1>(partial, nblk, R, r, s);
    if (threadIdx.x) return;
    Scal &q = sc[r];
    if (mode == 1) {
        q.b2 = s[0];
        return;
    }
    if (!q.active) return;
    q.r2hi = s[0];
    if (s[0] <= q.tol2) q.active = 0;
}

__global__ void k_fin_rho(const double *partial, int nblk, int R, Scal *sc)
{
    int r = blockIdx.x;
    double s[3];
    sum_partials<3>(partial, nblk, R, r, s);
    if (threadIdx.x) return;
    Scal &q = sc[r];
    if (!q.active) return;
    q.rho = make_double2(s[0], s[1]);
    q.r2 = s[2];
}

// ------------------------------------------------------------------- CGNR kernels
// CG on the normal equations Mhat^dag Mhat x = Mhat^dag bhat (the paper's fallback,
// Sec. IV).  r is the normal-equation residual, res = bhat - Mhat x the even-odd residual
// (both by recursion between FP64 reliable updates); rho holds |r|^2.

// start of CG from r = M^dag res already in storage precision: p = r, x = 0; partial |r|^2,
// |res|^2 (masked RHS only)
template <class SP, class XP>
__global__ __launch_bounds__(kBS) void k_cg_start(Vec r, Vec p, Vec res, Vec x, long Vh, int R, double *partial,
                                                  const Scal *sc)
{
    double acc[2] = {0, 0};
    long n = Vh * R, stride = (long)gridDim.x * kBS;
    int rr = (int)((blockIdx.x * (long)kBS + threadIdx.x) % R);
    bool act = sc[rr].active;
    for (long tid = blockIdx.x * (long)kBS + threadIdx.x; tid < n; tid += stride) {
        long i = tid / R;
        Cx<double> v[12];
#pragma unroll
        for (int k = 0; k < 12; k++) v[k] = {0, 0};
        st_site<XP>(x, Vh, R, i, rr, v);
        if (!act) continue;
        ld_site<SP>(r, Vh, R, i, rr, v);
        st_site<SP>(p, Vh, R, i, rr, v);
#pragma unroll
        for (int k = 0; k < 12; k++) acc[0] += v[k].re * v[k].re + v[k].im * v[k].im;
        ld_site<SP>(res, Vh, R, i, rr, v);
#pragma unroll
        for (int k = 0; k < 12; k++) acc[1] += v[k].re * v[k].re + v[k].im * v[k].im;
    }
    block_partial<2>(acc, R, partial);
}

// rho = |r|^2, r2 = |res|^2 (masked RHS only)
__global__ void k_fin_cg_init(const double *partial, int nblk, int R, Scal *sc)
{
    int r = blockIdx.x;
    double s[2];
    sum_partials<2>(partial, nblk, R, r, s);
    if (threadIdx.x || !sc[r].active) return;
    sc[r].rho = make_double2(s[0], 0);
    sc[r].r2 = s[1];
}

// partial |a|^2
template <class SP>
__global__ __launch_bounds__(kBS) void k_normsq(Vec a, long Vh, int R, double *partial)
{
    double acc[1] = {0};
    long n = Vh * R, stride = (long)gridDim.x * kBS;
    int rr = (int)((blockIdx.x * (long)kBS + threadIdx.x) % R);
    for (long tid = blockIdx.x * (long)kBS + threadIdx.x; tid < n; tid += stride) {
        long i = tid / R;
        Cx<double> v[12];
        ld_site<SP>(a, Vh, R, i, rr, v);
#pragma unroll
        for (int k = 0; k < 12; k++) acc[0] += v[k].re * v[k].re + v[k].im * v[k].im;
    }
    block_partial<1>(acc, R, partial);
}

// alpha = rho / |q|^2
// deterministic sum of right-hand-side-major partials partial[r * nblk + b]
__device__ __forceinline__ double sum_partials_rmajor(const double *partial, int nblk, int r)
{
    __shared__ double lds[kBS];
    double v = 0;
    for (int b = threadIdx.x; b < nblk; b += kBS) v += partial[(long)r * nblk + b];
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int s = kBS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    return lds[0];
}

// partial[b][row] (nrow values per block, block-major as the fused epilogues write them)
// -> out[row][kChunks], chunk ch = fixed-order sum of its contiguous share of the blocks
// (the first stage of a deterministic two-stage reduction; nrow <= kBS)
constexpr int kChunks = 1024;
// every caller reduces at most three values for each of at most 32 fields: one block holds
// a group of all nrow rows
static_assert(3 * 32 <= kBS, "k_prereduce needs nrow <= kBS");
__global__ __launch_bounds__(kBS) void k_prereduce(const double *partial, int nblk, int nrow, double *out)
{
    const int ch = blockIdx.x, t = threadIdx.x;
    const long beg = (long)nblk * ch / kChunks, end = (long)nblk * (ch + 1) / kChunks;
    const int G = kBS / nrow, g = t / nrow, row = t - g * nrow;  // G groups of nrow lanes
    // four independent partial sums per lane keep four loads in flight
    double v0 = 0, v1 = 0, v2 = 0, v3 = 0;
    if (g < G) {
        long b = beg + g;
        for (; b + 3 * G < end; b += 4 * G) {
            v0 += partial[b * nrow + row];
            v1 += partial[(b + G) * nrow + row];
            v2 += partial[(b + 2 * G) * nrow + row];
            v3 += partial[(b + 3 * G) * nrow + row];
        }
        for (; b < end; b += G) v0 += partial[b * nrow + row];
    }
    const double v = (v0 + v1) + (v2 + v3);
    __shared__ double lds[kBS];
    lds[t] = v;
    __syncthreads();
    if (t < nrow) {
        double s2 = 0;
        for (int q = 0; q < G; q++) s2 += lds[q * nrow + t];
        out[(long)t * kChunks + ch] = s2;
    }
}

// ------------------------------------------------- fused multi-RHS BiCGStab (Sec. IV)
// The low-precision BiCGStab iteration takes its inner products <r0, v>, <t, s>, |t|^2 from
// the epilogues of the hops that form v = M p and t = M s (M_INV_AFTER_DOT), and keeps its
// solution steps alpha p + omega s owed in a ring of K (p, s) buffer pairs, taken K at a
// time, as the CG loop does with its directions.

// (p, s) pairs whose steps the solution increment still owes, latest first: pair 0 takes
// the current alpha and omega, pair j >= 1 those of j iterations back
struct BsDirs {
    Vec p[kMaxDirs], s[kMaxDirs];
    int n = 0;
};

// o += sum_{j < n} alpha_j p_j + omega_j s_j
template <class SP>
__device__ __forceinline__ void add_bs_steps(const BsDirs &d, int n, const Scal &q, long Vh, int R, long i, int r,
                                             Cx<double> (&o)[12])
{
#pragma unroll
    for (int j = 0; j < kMaxDirs; j++) {
        if (j >= n) break;
        const Cx<double> al = cx(j ? q.bs_alpha_prev[j - 1] : q.alpha);
        const Cx<double> om = cx(j ? q.bs_omega_prev[j - 1] : q.omega);
        Cx<double> b[12];
        ld_site<SP>(d.p[j], Vh, R, i, r, b);
#pragma unroll
        for (int k = 0; k < 12; k++) o[k] = o[k] + al * b[k];
        ld_site<SP>(d.s[j], Vh, R, i, r, b);
#pragma unroll
        for (int k = 0; k < 12; k++) o[k] = o[k] + om * b[k];
    }
}

// the three value rows of right-hand side r in prereduced partials [(e R + r) * nblk + b]
__device__ __forceinline__ void sum_rows3(const double *partial, int nblk, int R, int r, double (&out)[3])
{
    __shared__ double lds[3][kBS];
    double v[3] = {0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += kBS)
#pragma unroll
        for (int e = 0; e < 3; e++) v[e] += partial[((long)e * R + r) * nblk + b];
#pragma unroll
    for (int e = 0; e < 3; e++) lds[e][threadIdx.x] = v[e];
    __syncthreads();
    for (int h = kBS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
#pragma unroll
            for (int e = 0; e < 3; e++) lds[e][threadIdx.x] += lds[e][threadIdx.x + h];
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < 3; e++) out[e] = lds[e][0];
}

// alpha = rho / <r0, v> from the epilogue partials of v = M p; the previous alpha and
// omega move into the step history first
__global__ void k_fin_bs_alpha(const double *partial, int nblk, int R, Scal *sc)
{
    const int r = blockIdx.x;
    double s[3];
    sum_rows3(partial, nblk, R, r, s);
    if (threadIdx.x) return;
    Scal &q = sc[r];
    if (!q.active) {
        q.alpha = make_double2(0, 0);
        return;
    }
    for (int j = kMaxDirs - 2; j > 0; j--) {
        q.bs_alpha_prev[j] = q.bs_alpha_prev[j - 1];
        q.bs_omega_prev[j] = q.bs_omega_prev[j - 1];
    }
    q.bs_alpha_prev[0] = q.alpha;
    q.bs_omega_prev[0] = q.omega;
    const double2 den = make_double2(s[0], s[1]);
    if (cnorm2(den) == 0.0 || !std::isfinite(den.x) || !std::isfinite(den.y)) {
        q.alpha = make_double2(0, 0);
        q.breakdown = 1;
        q.active = 0;
        return;
    }
    q.alpha = cdiv(q.rho, den);
}

// omega = <t, s> / |t|^2 from the epilogue partials of t = M s, which hold <s, t> = conj <t, s>
__global__ void k_fin_bs_omega(const double *partial, int nblk, int R, Scal *sc)
{
    const int r = blockIdx.x;
    double s[3];
    sum_rows3(partial, nblk, R, r, s);
    if (threadIdx.x) return;
    Scal &q = sc[r];
    if (!q.active) {
        q.omega = make_double2(0, 0);
        return;
    }
    if (!(s[2] > 0.0) || !std::isfinite(s[2])) {
        q.omega = make_double2(0, 0);
        q.breakdown = 1;
        q.active = 0;
        return;
    }
    q.omega = make_double2(s[0] / s[2], -s[1] / s[2]);
}

// r = s - omega t; per-block partials of <r0, r> and |r|^2 of the stored r, laid out as
// the hopping epilogues write them, [block][value][RHS] (a block: kBS / R sites x R RHS)
template <class SP>
__global__ __launch_bounds__(kBS) void k_bs_r(Vec s, Vec t, Vec r, Vec r0, long Vh, int R, double *partial,
                                              const Scal *sc)
{
    const long tid = blockIdx.x * (long)kBS + threadIdx.x;
    const long i = tid / R;
    const int rr = (int)(threadIdx.x & (R - 1));
    double acc[3] = {0, 0, 0};
    if (i < Vh && sc[rr].active) {
        const Cx<double> om = cx(sc[rr].omega);
        Cx<double> a[12], b[12];
        ld_site<SP>(s, Vh, R, i, rr, a);
        ld_site<SP>(t, Vh, R, i, rr, b);
#pragma unroll
        for (int k = 0; k < 12; k++) a[k] = a[k] - om * b[k];
        st_site<SP>(r, Vh, R, i, rr, a);
        ld_site<SP>(r, Vh, R, i, rr, a);  // the stored value
        ld_site<SP>(r0, Vh, R, i, rr, b);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            acc[0] += b[k].re * a[k].re + b[k].im * a[k].im;
            acc[1] += b[k].re * a[k].im - b[k].im * a[k].re;
            acc[2] += a[k].re * a[k].re + a[k].im * a[k].im;
        }
    }
    __shared__ double red[3][kBS];
#pragma unroll
    for (int e = 0; e < 3; e++) red[e][threadIdx.x] = acc[e];
    __syncthreads();
    if ((int)threadIdx.x < R) {
#pragma unroll
        for (int e = 0; e < 3; e++) {
            double v = 0.0;
            for (int q = threadIdx.x; q < kBS; q += R) v += red[e][q];
            partial[((long)blockIdx.x * 3 + e) * R + threadIdx.x] = v;
        }
    }
}

// rho_new = <r0, r>, beta = (rho_new / rho)(alpha / omega), |r|^2 from the prereduced
// partials of k_bs_r
__global__ void k_fin_bs_beta(const double *partial, int nblk, int R, Scal *sc)
{
    const int r = blockIdx.x;
    double s[3];
    sum_rows3(partial, nblk, R, r, s);
    if (threadIdx.x) return;
    Scal &q = sc[r];
    if (!q.active) {
        q.beta = make_double2(0, 0);
        return;
    }
    const double2 rn = make_double2(s[0], s[1]);
    q.iters += 1;
    q.r2 = s[2];
    if (!std::isfinite(s[0]) || !std::isfinite(s[1]) || !std::isfinite(s[2]) || cnorm2(q.rho) == 0.0 ||
        cnorm2(q.omega) == 0.0) {
        q.breakdown = 1;
        q.active = 0;
        q.beta = make_double2(0, 0);
        return;
    }
    q.beta = cmul(cdiv(rn, q.rho), cdiv(q.alpha, q.omega));
    q.rho = rn;
}

// pout = r + beta (p - omega v) with p = d.p[0]; pout may be d.p[0] or, when the owed steps
// are taken first (nsteps > 0: x += the steps of pairs 0 .. nsteps - 1), the oldest pair's p
template <class SP, class XP>
__global__ __launch_bounds__(kBS) void k_bs_p(Vec pout, BsDirs d, Vec r, Vec v, Vec x, long Vh, int R,
                                              const Scal *sc, int nsteps)
{
    long n = Vh * R;
    long tid = blockIdx.x * (long)kBS + threadIdx.x;
    if (tid >= n) return;
    long i = tid / R;
    int rr = (int)(tid - i * R);
    if (!sc[rr].active) return;
    const Cx<double> be = cx(sc[rr].beta), om = cx(sc[rr].omega);
    Cx<double> a[12], b[12];
    if (nsteps) {
        ld_site<XP>(x, Vh, R, i, rr, b);
        add_bs_steps<SP>(d, nsteps, sc[rr], Vh, R, i, rr, b);
        st_site<XP>(x, Vh, R, i, rr, b);
    }
    ld_site<SP>(d.p[0], Vh, R, i, rr, a);
    ld_site<SP>(v, Vh, R, i, rr, b);
#pragma unroll
    for (int k = 0; k < 12; k++) a[k] = a[k] - om * b[k];
    ld_site<SP>(r, Vh, R, i, rr, b);
#pragma unroll
    for (int k = 0; k < 12; k++) a[k] = b[k] + be * a[k];
    st_site<SP>(pout, Vh, R, i, rr, a);
}

// xhi += xlo + the owed steps; xlo = 0 (right-hand sides with mask set)
template <class XP, class SP>
__global__ __launch_bounds__(kBS) void k_fold_x_bs(Vec xhi, Vec xlo, BsDirs d, long Vh, int R, const Scal *sc)
{
    long n = Vh * R;
    long tid = blockIdx.x * (long)kBS + threadIdx.x;
    if (tid >= n) return;
    long i = tid / R;
    int rr = (int)(tid - i * R);
    if (!sc[rr].active) return;
    Cx<double> a[12], b[12], z[12];
    ld_site<S64>(xhi, Vh, R, i, rr, a);
    ld_site<XP>(xlo, Vh, R, i, rr, b);
#pragma unroll
    for (int k = 0; k < 12; k++) {
        a[k] = a[k] + b[k];
        z[k] = {0, 0};
    }
    add_bs_steps<SP>(d, d.n, sc[rr], Vh, R, i, rr, a);
    st_site<S64>(xhi, Vh, R, i, rr, a);
    st_site<XP>(xlo, Vh, R, i, rr, z);
}

// partial <a, b>, |b|^2
template <class SP>
__global__ __launch_bounds__(kBS) void k_dot_nb(Vec a, Vec b, long Vh, int R, double *partial, const Scal *sc)
{
    double acc[3] = {0, 0, 0};
    long n = Vh * R, stride = (long)gridDim.x * kBS;
    int rr = (int)((blockIdx.x * (long)kBS + threadIdx.x) % R);
    const bool act = sc[rr].active;
    for (long tid = blockIdx.x * (long)kBS + threadIdx.x; tid < n; tid += stride) {
        if (!act) break;
        long i = tid / R;
        Cx<double> u[12], w[12];
        ld_site<SP>(a, Vh, R, i, rr, u);
        ld_site<SP>(b, Vh, R, i, rr, w);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            acc[0] += u[k].re * w[k].re + u[k].im * w[k].im;
            acc[1] += u[k].re * w[k].im - u[k].im * w[k].re;
            acc[2] += w[k].re * w[k].re + w[k].im * w[k].im;
        }
    }
    block_partial<3>(acc, R, partial);
}

// the host's divergence verdicts, in stream order: right-hand sides in mask stop with a
// breakdown (handed to the fallback)
__global__ void k_bs_drop(Scal *sc, int R, unsigned mask)
{
    const int r = threadIdx.x;
    if (r < R && ((mask >> r) & 1u) && sc[r].active) {
        sc[r].active = 0;
        sc[r].breakdown = 1;
    }
}

// rmajor: partials of the fused hopping epilogue (one value per block and RHS)
__global__ void k_fin_cg_alpha(const double *partial, int nblk, int R, Scal *sc, int rmajor)
{
    int r = blockIdx.x;
    double s[1];
    if (rmajor)
        s[0] = sum_partials_rmajor(partial, nblk, r);
    else
        sum_partials<1>(partial, nblk, R, r, s);
    if (threadIdx.x) return;
    Scal &q = sc[r];
    if (!q.active) {
        q.alpha = make_double2(0, 0);
        return;
    }
    for (int j = kMaxDirs - 2; j > 0; j--) q.alpha_prev[j] = q.alpha_prev[j - 1];
    q.alpha_prev[0] = q.alpha.x;
    if (!(s[0] > 0) || !std::isfinite(s[0])) {
        q.alpha = make_double2(0, 0);
        q.breakdown = 1;
        q.active = 0;
        return;
    }
    q.alpha = make_double2(q.rho.x / s[0], 0);
}

// x += alpha p; res -= alpha q; r -= alpha y;  partial |r|^2, |res|^2
// kRes = false: the even-odd residual is not carried as a vector; its norm follows
// |res'|^2 = |res|^2 - alpha |r|^2 (k_fin_cg_beta) between reliable updates
template <class SP, class XP, bool kRes>
__global__ __launch_bounds__(kBS) void k_cg_update(Vec x, Vec p, Vec res, Vec q, Vec r, Vec y, long Vh, int R,
                                                   double *partial, const Scal *sc)
{
    double acc[2] = {0, 0};
    long n = Vh * R, stride = (long)gridDim.x * kBS;
    int rr = (int)((blockIdx.x * (long)kBS + threadIdx.x) % R);
    bool act = sc[rr].active;
    double al = sc[rr].alpha.x;
    for (long tid = blockIdx.x * (long)kBS + threadIdx.x; tid < n; tid += stride) {
        if (!act) break;
        long i = tid / R;
        Cx<double> a[12], b[12];
        ld_site<XP>(x, Vh, R, i, rr, a);
        ld_site<SP>(p, Vh, R, i, rr, b);
#pragma unroll
        for (int k = 0; k < 12; k++) a[k] = a[k] + al * b[k];
        st_site<XP>(x, Vh, R, i, rr, a);
        if constexpr (kRes) {
            ld_site<SP>(res, Vh, R, i, rr, a);
            ld_site<SP>(q, Vh, R, i, rr, b);
#pragma unroll
            for (int k = 0; k < 12; k++) a[k] = a[k] - al * b[k];
            st_site<SP>(res, Vh, R, i, rr, a);
            ld_site<SP>(res, Vh, R, i, rr, a);
#pragma unroll
            for (int k = 0; k < 12; k++) acc[1] += a[k].re * a[k].re + a[k].im * a[k].im;
        }
        ld_site<SP>(r, Vh, R, i, rr, a);
        ld_site<SP>(y, Vh, R, i, rr, b);
#pragma unroll
        for (int k = 0; k < 12; k++) a[k] = a[k] - al * b[k];
        st_site<SP>(r, Vh, R, i, rr, a);
        ld_site<SP>(r, Vh, R, i, rr, a);
#pragma unroll
        for (int k = 0; k < 12; k++) acc[0] += a[k].re * a[k].re + a[k].im * a[k].im;
    }
    block_partial<2>(acc, R, partial);
}

// beta = |r|^2 / rho; rho = |r|^2; r2 = |res|^2; with hi_conv the recursive even-odd
// residual alone may declare convergence (plain FP64 iteration)
__global__ void k_fin_cg_beta(const double *partial, int nblk, int R, Scal *sc, int hi_conv, int recur,
                              int rmajor)
{
    int r = blockIdx.x;
    double s[2];
    if (rmajor) {
        s[0] = sum_partials_rmajor(partial, nblk, r);
        s[1] = 0.0;
    } else {
        sum_partials<2>(partial, nblk, R, r, s);
    }
    if (threadIdx.x) return;
    Scal &q = sc[r];
    if (!q.active) {
        q.beta = make_double2(0, 0);
        return;
    }
    q.iters += 1;
    // rho still holds the previous |r|^2 here
    q.r2 = recur ? fmax(q.r2 - q.alpha.x * q.rho.x, 0.0) : s[1];
    if (!std::isfinite(s[0]) || !std::isfinite(s[1]) || !(q.rho.x > 0)) {
        q.breakdown = 1;
        q.active = 0;
        q.beta = make_double2(0, 0);
        return;
    }
    q.beta = make_double2(s[0] / q.rho.x, 0);
    q.rho_prev = q.rho.x;
    q.rho = make_double2(s[0], 0);
    if (hi_conv && (s[1] <= q.tol2 || !(s[0] > 0))) q.active = 0;
}

// direction update pout = r + beta d_0 (real beta); pout may be d_0, the oldest direction
// d_{n-1}, or another buffer.  With nsteps > 0 the solution increment first takes the steps
// still owed along the directions: x += sum_{j < nsteps} coef_j d_j.  orth (after a reliable
// update): d_0 is first made orthogonal to the new r, d_0 - aux r, so that
// pout = (1 - beta aux) r + beta d_0
template <class SP, class XP>
__global__ __launch_bounds__(kBS) void k_cg_p(Vec pout, Dirs dirs, Vec r, Vec x, long Vh, int R, const Scal *sc,
                                              int nsteps, int orth)
{
    long n = Vh * R;
    long tid = blockIdx.x * (long)kBS + threadIdx.x;
    if (tid >= n) return;
    long i = tid / R;
    int rr = (int)(tid - i * R);
    if (!sc[rr].active) return;
    double be = sc[rr].beta.x;
    Cx<double> a[12], b[12];
    if (nsteps) {
        ld_site<XP>(x, Vh, R, i, rr, b);
        add_steps<SP>(dirs, nsteps, sc[rr], Vh, R, i, rr, b);
        st_site<XP>(x, Vh, R, i, rr, b);
    }
    ld_site<SP>(dirs.d[0], Vh, R, i, rr, a);
    ld_site<SP>(r, Vh, R, i, rr, b);
    if (orth) {
        const Cx<double> g = {1.0 - be * sc[rr].aux.x, -be * sc[rr].aux.y};
#pragma unroll
        for (int k = 0; k < 12; k++) a[k] = g * b[k] + be * a[k];
    } else {
#pragma unroll
        for (int k = 0; k < 12; k++) a[k] = b[k] + be * a[k];
    }
    st_site<SP>(pout, Vh, R, i, rr, a);
}

// after the residual was replaced: rho = |r|^2, r2 = |res|^2, beta = |r|^2 / rho_prev
__global__ void k_fin_cg_reset(const double *partial, int nblk, int R, Scal *sc)
{
    int r = blockIdx.x;
    double s[2];
    sum_partials<2>(partial, nblk, R, r, s);
    if (threadIdx.x || !sc[r].active) return;
    Scal &q = sc[r];
    q.rho = make_double2(s[0], 0);
    q.r2 = s[1];
    q.beta = make_double2(q.rho_prev > 0 ? s[0] / q.rho_prev : 0.0, 0);
}

// aux = <r, p> / |r|^2 (rho holds |r|^2)
__global__ void k_fin_orth(const double *partial, int nblk, int R, Scal *sc)
{
    int r = blockIdx.x;
    double s[2];
    sum_partials<2>(partial, nblk, R, r, s);
    if (threadIdx.x) return;
    Scal &q = sc[r];
    q.aux = (q.active && q.rho.x > 0) ? make_double2(s[0] / q.rho.x, s[1] / q.rho.x) : make_double2(0, 0);
}

// b = convert(a) (FP64 -> storage precision) for active right-hand sides
template <class SP>
__global__ __launch_bounds__(kBS) void k_convert_masked(Vec a, Vec b, long Vh, int R, const Scal *sc)
{
    long n = Vh * R;
    long tid = blockIdx.x * (long)kBS + threadIdx.x;
    if (tid >= n) return;
    long i = tid / R;
    int rr = (int)(tid - i * R);
    if (!sc[rr].active) return;
    Cx<double> v[12];
    ld_site<S64>(a, Vh, R, i, rr, v);
    st_site<SP>(b, Vh, R, i, rr, v);
}

// partial |a|^2, |b|^2 per right-hand side
template <class SP>
__global__ __launch_bounds__(kBS) void k_normsq2(Vec a, Vec b, long Vh, int R, double *partial)
{
    double acc[2] = {0, 0};
    long n = Vh * R, stride = (long)gridDim.x * kBS;
    int rr = (int)((blockIdx.x * (long)kBS + threadIdx.x) % R);
    for (long tid = blockIdx.x * (long)kBS + threadIdx.x; tid < n; tid += stride) {
        long i = tid / R;
        Cx<double> v[12];
        ld_site<SP>(a, Vh, R, i, rr, v);
#pragma unroll
        for (int k = 0; k < 12; k++) acc[0] += v[k].re * v[k].re + v[k].im * v[k].im;
        ld_site<SP>(b, Vh, R, i, rr, v);
#pragma unroll
        for (int k = 0; k < 12; k++) acc[1] += v[k].re * v[k].re + v[k].im * v[k].im;
    }
    block_partial<2>(acc, R, partial);
}

// r = convert(rhi), res = convert(reshi) for masked RHS; partial |r|^2, |res|^2
template <class SP>
__global__ __launch_bounds__(kBS) void k_cg_replace(Vec rhi, Vec reshi, Vec r, Vec res, long Vh, int R,
                                                    double *partial, const Scal *sc)
{
    double acc[2] = {0, 0};
    long n = Vh * R, stride = (long)gridDim.x * kBS;
    int rr = (int)((blockIdx.x * (long)kBS + threadIdx.x) % R);
    bool act = sc[rr].active;
    for (long tid = blockIdx.x * (long)kBS + threadIdx.x; tid < n; tid += stride) {
        if (!act) break;
        long i = tid / R;
        Cx<double> v[12];
        ld_site<S64>(rhi, Vh, R, i, rr, v);
        st_site<SP>(r, Vh, R, i, rr, v);
        ld_site<SP>(r, Vh, R, i, rr, v);
#pragma unroll
        for (int k = 0; k < 12; k++) acc[0] += v[k].re * v[k].re + v[k].im * v[k].im;
        ld_site<S64>(reshi, Vh, R, i, rr, v);
        st_site<SP>(res, Vh, R, i, rr, v);
        ld_site<SP>(res, Vh, R, i, rr, v);
#pragma unroll
        for (int k = 0; k < 12; k++) acc[1] += v[k].re * v[k].re + v[k].im * v[k].im;
    }
    block_partial<2>(acc, R, partial);
}

// copy (masked) a -> b, both FP64
__global__ __launch_bounds__(kBS) void k_copy64(Vec a, Vec b, long Vh, int R, const Scal *sc, int all_rhs)
{
    long n = Vh * R;
    long tid = blockIdx.x * (long)kBS + threadIdx.x;
    if (tid >= n) return;
    long i = tid / R;
    int rr = (int)(tid - i * R);
    if (!all_rhs && !sc[rr].active) return;
    for (int k = 0; k < 12; k++) {
        long idx = ((long)k * Vh + i) * R + rr;
        ((double2 *)b.d)[idx] = ((const double2 *)a.d)[idx];
    }
}

// ---------------------------------------------------------------- operator helper
template <class SP>
constexpr int prec_of()
{
    return std::is_same<SP, S16>::value    ? LAPH_PREC_F16
           : std::is_same<SP, SB16>::value ? LAPH_PREC_BF16
           : std::is_same<SP, S32>::value  ? LAPH_PREC_F32
                                           : LAPH_PREC_F64;
}

template <class SP, class GP, class CP>
struct Op {
    laph_ctx *c;
    hipStream_t st;
    long Vh;
    int R;
    const void *g;
    const char *clinv;  // packed inverse, parity p at clinv + p * 72 * Vh * sizeof(CP::E)
    const char *clov;   // packed clover (FP64 operator only)
    double ws, wt, bct;
    Vec te;  // even temporary
    // low-precision multi-RHS layouts (used whenever SP is not FP64)
    const float4 *lk12 = nullptr;
    const float4 *claos = nullptr;  // per-site clover inverse, parity p at claos + p * Vh * 18
    int tgauge = 0;                 // temporal gauge: unit time links off the last slice

    static constexpr bool kLow = !std::is_same<SP, S64>::value;

    DslashArgs base(int par) const
    {
        DslashArgs a{};
        a.gauge = g;
        a.ns = c->g.ns;
        a.nt = c->g.nt;
        a.Vh = Vh;
        a.R = R;
        a.par = par;
        a.wt = wt;
        a.ws = ws;
        a.bct = bct;
        return a;
    }
    const void *cinv(int par) const { return clinv + (size_t)par * 72 * Vh * sizeof(typename CP::E); }
    const void *cl(int par) const { return clov + (size_t)par * 72 * Vh * sizeof(typename CP::E); }

    // arguments of the multi-RHS low-precision hopping kernel
    MrArgs mr_args(int par, Vec in, Vec out, const Vec *x, double a, double cc, int g5d) const
    {
        MrArgs m{};
        m.out = out.d;
        m.out_nrm = out.n;
        m.in = in.d;
        m.in_nrm = in.n;
        m.x = x ? x->d : nullptr;
        m.x_nrm = x ? x->n : nullptr;
        m.links = lk12;
        m.clov = claos + (size_t)par * Vh * 18;
        m.ns = c->g.ns;
        m.nt = c->g.nt;
        m.Vh = Vh;
        m.R = R;
        m.par = par;
        m.a = a;
        m.c = cc;
        m.wt = wt;
        m.ws = ws;
        m.bct = bct;
        m.g5d = g5d;
        m.tgauge = tgauge;
        return m;
    }
    // hopping term with epilogue; mode M_PLAIN or M_INV_AFTER
    void dslash(int mode, int par, Vec in, Vec out, const Vec *x, double a, double cc, int g5d) const
    {
        dslash_ext(mode, par, in, out, x, a, cc, g5d, nullptr, nullptr);
    }
    // as dslash; with mode M_INV_AFTER_DAG (low precision) also out2 = A^-1 gamma_5 out and
    // per-block |out|^2 partials
    void dslash_ext(int mode, int par, Vec in, Vec out, const Vec *x, double a, double cc, int g5d, const Vec *out2,
                    double *partial) const
    {
        if constexpr (kLow) {
            MrArgs m = mr_args(par, in, out, x, a, cc, g5d);
            if (out2) {
                m.out2 = out2->d;
                m.out2_nrm = out2->n;
                m.partial = partial;
            }
            launch_dslash_mr<SP>(c, mode, m, st);
        } else {
            LAPH_CHECK(mode != M_INV_AFTER_DAG, LAPH_EINVAL, "fused epilogue is low precision only");
            DslashArgs d = base(par);
            d.in = in.d;
            d.in_nrm = in.n;
            d.out = out.d;
            d.out_nrm = out.n;
            d.x = x ? x->d : nullptr;
            d.x_nrm = x ? x->n : nullptr;
            d.clov = cinv(par);
            d.a = a;
            d.c = cc;
            d.g5d = g5d;
            launch_dslash<SP, GP, CP>(c, mode, d, st);
        }
    }
    void clover_inv(int par, Vec in, Vec out, int g5_in) const
    {
        if constexpr (kLow)
            launch_clover_mr<SP>(c, claos + (size_t)par * Vh * 18, in.d, in.n, out.d, out.n, Vh, R, g5_in, st);
        else
            launch_clover_apply<SP, CP>(c, cinv(par), in.d, in.n, out.d, out.n, Vh, R, g5_in, st);
    }

    // out_o = in_o - A_oo^-1 D_oe A_ee^-1 D_eo in_o
    void mhat(Vec in, Vec out) const
    {
        dslash(M_INV_AFTER, 0, in, te, nullptr, 0.0, 1.0, 0);
        dslash(M_INV_AFTER, 1, te, out, &in, 1.0, -1.0, 0);
    }
    // out_o = Mhat^dag in_o = in_o - gamma_5 D_oe A_ee^-1 D_eo A_oo^-1 gamma_5 in_o
    void mhat_dag(Vec in, Vec out, Vec to) const
    {
        clover_inv(1, in, to, 1);
        mhat_dag_rest(in, to, out);
    }
    // the part of mhat_dag after to = A_oo^-1 gamma_5 in
    void mhat_dag_rest(Vec in, Vec to, Vec out) const
    {
        dslash(M_INV_AFTER, 0, to, te, nullptr, 0.0, 1.0, 0);
        dslash(M_PLAIN, 1, te, out, &in, 1.0, -1.0, 1);
    }
    // mhat_dag_rest whose last hop feeds the CG residual update r -= alpha (M^dag in)
    // directly (low precision, LDS-staged kernel); per-block |r|^2 partials
    void mhat_dag_cg(Vec in, Vec to, Vec r, const Scal *sc, double *partial) const
    {
        dslash(M_INV_AFTER, 0, to, te, nullptr, 0.0, 1.0, 0);
        if constexpr (kLow) {
            MrArgs m = mr_args(1, te, Vec{}, &in, 1.0, -1.0, 1);
            m.partial = partial;
            m.sc = sc;
            m.cg_r = r.d;
            m.cg_r_nrm = r.n;
            launch_dslash_mr<SP>(c, M_PLAIN_CG, m, st);
        } else {
            laph_fail(LAPH_EINVAL, "fused CG update is low precision only");
        }
    }
    // mhat with the second hop's epilogue also forming to = A_oo^-1 gamma_5 out (the start of
    // mhat_dag) and per-block |out|^2 partials (low precision, LDS-staged kernel)
    void mhat_prep(Vec in, Vec out, Vec to, double *partial) const
    {
        dslash(M_INV_AFTER, 0, in, te, nullptr, 0.0, 1.0, 0);
        dslash_ext(M_INV_AFTER_DAG, 1, te, out, &in, 1.0, -1.0, 0, &to, partial);
    }
    // mhat with per-block partials of <y, out> and |out|^2 from the second hop's epilogue
    // (low precision, LDS-staged kernel; partials [block][value][RHS], see MrArgs)
    void mhat_dot(Vec in, Vec out, Vec y, double *partial) const
    {
        dslash(M_INV_AFTER, 0, in, te, nullptr, 0.0, 1.0, 0);
        if constexpr (kLow) {
            MrArgs m = mr_args(1, te, out, &in, 1.0, -1.0, 0);
            m.dot_y = y.d;
            m.dot_y_nrm = y.n;
            m.partial = partial;
            launch_dslash_mr<SP>(c, M_INV_AFTER_DOT, m, st);
        } else {
            laph_fail(LAPH_EINVAL, "fused BiCGStab products are low precision only");
        }
    }
};

using Op64 = Op<S64, G64, C64>;

struct Work {
    laph_ctx *c;
    long Vh;
    int R;
    Scal *sc;      // device
    double *part;  // device partials [kMaxBlocks][R][4]
    bool use_graph = false;  // capture the CG iteration body in a HIP graph
    double delta2 = 0.01;    // reliable update when |res|^2 fell below delta2 times its last FP64 value
    int dirs = 0;            // direction buffers of the fused CG loop (0: the default)
    bool x_zero = false;     // x_hi is known to be zero (the first residual is bhat itself)
    Vec make(const char *name, int bytes, bool norm)
    {
        Vec v;
        v.d = ctx_named(c, std::string("slv.") + name, (size_t)12 * Vh * R * bytes);
        if (norm) v.n = (float *)ctx_named(c, std::string("slv.") + name + ".n", (size_t)Vh * R * 4);
        return v;
    }
};

template <class K, class... Args>
void launch_red(laph_ctx *c, K kern, long n, Args... args)
{
    hipLaunchKernelGGL(kern, dim3(red_blocks(n)), dim3(kBS), 0, c->stream, args...);
    LAPH_HIP(hipGetLastError());
}
template <class K, class... Args>
void launch_el(laph_ctx *c, K kern, long n, Args... args)
{
    hipLaunchKernelGGL(kern, dim3(nblocks_for(n, kBS)), dim3(kBS), 0, c->stream, args...);
    LAPH_HIP(hipGetLastError());
}
template <class K, class... Args>
void launch_fin(laph_ctx *c, K kern, int R, Args... args)
{
    hipLaunchKernelGGL(kern, dim3(R), dim3(kBS), 0, c->stream, args...);
    LAPH_HIP(hipGetLastError());
}

void read_scal(laph_ctx *c, const Scal *d, std::vector<Scal> &h)
{
    LAPH_HIP(hipMemcpyAsync(h.data(), d, sizeof(Scal) * h.size(), hipMemcpyDeviceToHost, c->stream));
    LAPH_HIP(hipStreamSynchronize(c->stream));
}
// pinned two-slot scalar readback for the CG loop (grown on demand, owned by the context)
static Scal *pinned_scal(laph_ctx *c, int R)
{
    const size_t need = 2 * sizeof(Scal) * (size_t)R;
    if (c->pin_bytes < need) {
        if (c->pin) LAPH_HIP(hipHostFree(c->pin));
        c->pin = nullptr;
        c->pin_bytes = 0;
        LAPH_HIP(hipHostMalloc(&c->pin, need, hipHostMallocDefault));
        c->pin_bytes = need;
    }
    for (hipEvent_t &e : c->pin_ev)
        if (!e) LAPH_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return (Scal *)c->pin;
}

// direction buffers of the fused CG loop where the solver parameters leave them open: the
// FP32 solution increment takes the owed steps every that many iterations
constexpr int kDefaultDirs = 8;

// A reliable update serves the whole block, so it waits until this percentage of the
// active right-hand sides want one: their iterated residual fell below reliable_delta of
// its last FP64 value, or below the target (a candidate for convergence, which only the
// FP64 residual can confirm and which meanwhile keeps iterating with the block).  It comes
// at once when one non-candidate fell 100 times further (the storage precision could no
// longer follow it) or every active one is a candidate, and after reliable_every
// iterations.  On 32 LapH sources of the 24^3 x 128 workload (FP16 inner vectors)
// counting candidates into the quorum instead of updating for each cut the updates of
// BiCGStab, whose right-hand sides reach the target over a wider spread of iterations,
// from 22-30 to 15-16 per solve (reliable_delta 0.03); at reliable_delta 0.1 a half
// instead of a quarter cut them from 19-21 to 15 at the same iteration count.  CG needs
// 9 to 11 either way.
constexpr int kUpdateQuorum = 50;

// the rule above on the scalars of one iteration (active right-hand sides only)
struct UpdateVote {
    int nact = 0, nwant = 0, nconv = 0;
    bool deep = false;
    double worst = 0;  // largest |res| / target
    void add(const Scal &q, double r2_last, double delta2)
    {
        nact++;
        worst = std::max(worst, q.tol2 > 0 ? std::sqrt(q.r2 / q.tol2) : 0.0);
        if (q.r2 <= q.tol2) {
            nconv++;
            nwant++;
        } else if (q.r2 < delta2 * r2_last) {
            nwant++;
            deep |= q.r2 < 0.01 * delta2 * r2_last;
        }
    }
    bool quorum() const { return nwant > 0 && nwant * 100 >= kUpdateQuorum * nact; }
    bool all_conv() const { return nact > 0 && nconv == nact; }
    bool want() const { return deep || all_conv() || quorum(); }
};

void write_scal(laph_ctx *c, Scal *d, const std::vector<Scal> &h)
{
    LAPH_HIP(hipMemcpyAsync(d, h.data(), sizeof(Scal) * h.size(), hipMemcpyHostToDevice, c->stream));
}

// rhi = bhat - Mhat xhi for masked RHS (FP64), then r2hi / masks (rlo: the residual in
// storage precision SP instead of rhi, for the right-hand sides it is formed for)
template <class SP = S64>
void true_eo_residual(Work &w, const Op64 &hi, Vec bhat, Vec xhi, Vec tmp, Vec rhi, int all_rhs, Vec rlo = Vec{})
{
    // with x_hi known to be zero (the first residual of a solve) the operator is skipped
    Vec m = tmp;
    if (w.x_zero)
        m = Vec{};
    else
        hi.mhat(xhi, tmp);
    w.x_zero = false;  // the caller goes on to change x_hi
    long n = w.Vh * w.R;
    // with a storage-precision copy requested the callers use that copy alone
    launch_red(w.c, k_resid64<SP>, n, bhat, m, rlo.d ? Vec{} : rhi, rlo, w.Vh, w.R, w.part, (const Scal *)w.sc,
               all_rhs);
    launch_fin(w.c, k_fin_r2hi, w.R, (const double *)w.part, (int)red_blocks(n), w.R, w.sc, 0);
}

// Low-precision BiCGStab (Sec. IV) on the even-odd system, fused for the multi-RHS
// kernels: per iteration two hops form v = M p with <r0, v> from its epilogue, a pass forms
// s = r - alpha v, two hops form t = M s with <t, s> and |t|^2 from its epilogue, a pass
// forms r = s - omega t with <r0, r> and |r|^2, and the direction update forms
// p = r + beta (p - omega v).  The steps alpha p + omega s are owed to the FP32 increment
// in a ring of K (p, s) pairs and taken K at a time; FP64 reliable updates (quorum rule of
// the CG loop) fold them with the increment into x_hi and replace r by the FP64 residual.
// Decisions read the previous iteration's scalars, as in the CG loop.
template <class SP, class GP, class CP, class XP>
void bicgstab_fused(Work &w, const Op<SP, GP, CP> &lo, const Op64 &hi, Vec bhat, Vec xhi, Vec rhi, Vec tmp64,
                    int maxiter, int reliable_every, std::vector<Scal> &hs)
{
    const bool nrm = SP::kNorm;
    laph_ctx *c = w.c;
    const long n = w.Vh * w.R;
    const int nblk = (int)red_blocks(n);
    const int K = w.dirs > 0 ? w.dirs : kDefaultDirs;
    Vec r = w.make("r", SP::bytes, nrm), r0 = w.make("r0", SP::bytes, nrm);
    Vec v = w.make("v", SP::bytes, nrm), t = w.make("t", SP::bytes, nrm);
    Vec pb[kMaxDirs], sb[kMaxDirs];
    pb[0] = w.make("p", SP::bytes, nrm);
    sb[0] = w.make("s", SP::bytes, nrm);
    for (int j = 1; j < K; j++) {
        pb[j] = w.make(("p" + std::to_string(j + 1)).c_str(), SP::bytes, nrm);
        sb[j] = w.make(("s" + std::to_string(j + 1)).c_str(), SP::bytes, nrm);
    }
    Vec xlo = w.make("xlo", XP::bytes, false);
    // per-block partials of the hopping epilogues and of the residual update (three rows
    // per RHS each), then kChunks per row
    const int nblk_hop = (int)lds_dag_blocks(c, prec_of<SP>(), w.R), nblk_el = (int)nblocks_for(n, kBS);
    double *part_hop =
        (double *)ctx_named(c, "slv.bs_part_hop", sizeof(double) * 3 * std::max(nblk_hop, nblk_el) * w.R);
    double *part_pre = (double *)ctx_named(c, "slv.bs_part_pre", sizeof(double) * 3 * kChunks * w.R);
    // r = r0 = p = the FP64 residual in storage precision, x = 0
    launch_red(c, k_bicg_init<SP, XP>, n, rhi, r, r0, pb[0], xlo, w.Vh, w.R, w.part, (const Scal *)w.sc);
    launch_fin(c, k_fin_init, w.R, (const double *)w.part, nblk, w.R, w.sc);
    read_scal(c, w.sc, hs);
    std::vector<double> r2_last(w.R), r2_min(w.R);
    for (int q = 0; q < w.R; q++) r2_last[q] = r2_min[q] = hs[q].r2;
    int cur = 0;    // p is pb[cur]; this iteration's s goes to sb[cur]
    int nowed = 0;  // steps owed to x by earlier iterations, pairs cur - 1, ..., cur - nowed
    // cnt pairs, latest first, starting first pairs behind cur
    auto owed = [&](int first, int cnt) {
        BsDirs d;
        for (int j = 0; j < cnt; j++) {
            const int b = ((cur - first - j) % K + K) % K;
            d.p[j] = pb[b];
            d.s[j] = sb[b];
        }
        d.n = cnt;
        return d;
    };
    auto body = [&](const Op<SP, GP, CP> &op, int b) {
        op.mhat_dot(pb[b], v, r0, part_hop);
        hipLaunchKernelGGL(k_prereduce, dim3(kChunks), dim3(kBS), 0, c->stream, (const double *)part_hop, nblk_hop,
                           3 * w.R, part_pre);
        launch_fin(c, k_fin_bs_alpha, w.R, (const double *)part_pre, kChunks, w.R, w.sc);
        launch_el(c, k_s_update<SP>, n, r, v, sb[b], w.Vh, w.R, (const Scal *)w.sc);
        op.mhat_dot(sb[b], t, sb[b], part_hop);
        hipLaunchKernelGGL(k_prereduce, dim3(kChunks), dim3(kBS), 0, c->stream, (const double *)part_hop, nblk_hop,
                           3 * w.R, part_pre);
        launch_fin(c, k_fin_bs_omega, w.R, (const double *)part_pre, kChunks, w.R, w.sc);
        launch_el(c, k_bs_r<SP>, n, sb[b], t, r, r0, w.Vh, w.R, part_hop, (const Scal *)w.sc);
        hipLaunchKernelGGL(k_prereduce, dim3(kChunks), dim3(kBS), 0, c->stream, (const double *)part_hop, nblk_el,
                           3 * w.R, part_pre);
        launch_fin(c, k_fin_bs_beta, w.R, (const double *)part_pre, kChunks, w.R, w.sc);
    };
    Scal *pin = pinned_scal(c, w.R);
    int slot = 0;
    bool prev_ok = false;
    hipGraphExec_t gexecs[kMaxDirs] = {};  // the body captured for each ring position
    const bool graph_ok = w.use_graph && !c->timing;
    if (graph_ok && !c->cap_stream) LAPH_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    struct GraphGuard {
        hipGraphExec_t *g;
        ~GraphGuard()
        {
            for (int k = 0; k < kMaxDirs; k++)
                if (g[k]) (void)hipGraphExecDestroy(g[k]);
        }
    } guard{gexecs};
    const double kDelta2 = w.delta2;
    int since = 0;
    int why[4] = {0, 0, 0, 0};  // reliable updates by trigger: all converged, deep drop, quorum, count
    for (int it = 0; it < maxiter; it++) {
        hipGraphExec_t &gexec = gexecs[cur];
        if (gexec) {
            LAPH_HIP(hipGraphLaunch(gexec, c->stream));
        } else if (graph_ok) {
            hipStream_t main = c->stream;
            Op<SP, GP, CP> cap = lo;
            cap.st = c->cap_stream;
            c->stream = c->cap_stream;
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
            if (e == hipSuccess) {
                body(cap, cur);
                e = hipStreamEndCapture(c->cap_stream, &g);
            }
            c->stream = main;
            LAPH_HIP(e);
            e = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            LAPH_HIP(e);
            LAPH_HIP(hipGraphLaunch(gexec, c->stream));
        } else {
            body(lo, cur);
        }
        // the direction update writes the next pair's p; with every pair owed it first
        // takes all K steps (the oldest pair is the one overwritten)
        const bool take = nowed + 1 == K;
        const int nxt = (cur + 1) % K;
        launch_el(c, k_bs_p<SP, XP>, n, pb[nxt], owed(0, take ? K : 1), r, v, xlo, w.Vh, w.R, (const Scal *)w.sc,
                  take ? K : 0);
        cur = nxt;
        nowed = take ? 0 : nowed + 1;
        since++;
        LAPH_HIP(hipMemcpyAsync(pin + (size_t)slot * w.R, w.sc, sizeof(Scal) * w.R, hipMemcpyDeviceToHost,
                                c->stream));
        LAPH_HIP(hipEventRecord(c->pin_ev[slot], c->stream));
        const int use = prev_ok ? slot ^ 1 : slot;
        LAPH_HIP(hipEventSynchronize(c->pin_ev[use]));
        std::copy(pin + (size_t)use * w.R, pin + (size_t)use * w.R + w.R, hs.begin());
        prev_ok = true;
        slot ^= 1;
        // divergence: the iterated residual grew 1e4-fold above its minimum; the RHS is
        // handed to the fallback
        unsigned drop = 0;
        UpdateVote vote;
        for (int q = 0; q < w.R; q++) {
            if (!hs[q].active) continue;
            r2_min[q] = std::min(r2_min[q], hs[q].r2);
            if (!(hs[q].r2 <= 1e8 * r2_min[q])) {
                drop |= 1u << q;
                continue;
            }
            vote.add(hs[q], r2_last[q], kDelta2);
        }
        const bool any = vote.nact > 0, want_update = vote.want();
        const int nact = vote.nact;
        const double worst = vote.worst;
        if (drop) {
            hipLaunchKernelGGL(k_bs_drop, dim3(1), dim3(32), 0, c->stream, w.sc, w.R, drop);
            LAPH_HIP(hipGetLastError());
        }
        if (laph_verbose() && (it % 256 == 0 || !any || laph_verbose_level() > 1))
            fprintf(stderr, "[laph] bicgstab it=%d active=%d/%d max |r|/target=%.3g upd=%d\n", it, nact, w.R, worst,
                    (int)want_update);
        if (!any) break;
        if (want_update || since >= reliable_every) {
            why[vote.all_conv() ? 0 : vote.deep ? 1 : vote.quorum() ? 2 : 3]++;
            // reliable update: x_hi += x_lo + the owed steps, r = the FP64 residual in storage
            // precision, rho = <r0, r>; p is kept
            launch_el(c, k_fold_x_bs<XP, SP>, n, xhi, xlo, owed(1, nowed), w.Vh, w.R, (const Scal *)w.sc);
            nowed = 0;
            true_eo_residual<SP>(w, hi, bhat, xhi, tmp64, rhi, 0, r);
            launch_red(c, k_dot_nb<SP>, n, r0, r, w.Vh, w.R, w.part, (const Scal *)w.sc);
            launch_fin(c, k_fin_rho, w.R, (const double *)w.part, nblk, w.R, w.sc);
            since = 0;
            read_scal(c, w.sc, hs);
            prev_ok = false;  // the slots predate the update
            bool left = false;
            for (int q = 0; q < w.R; q++) {
                left |= hs[q].active != 0;
                r2_last[q] = hs[q].r2;
                r2_min[q] = std::min(r2_min[q], hs[q].r2);
            }
            if (!left) break;
        }
    }
    if (laph_verbose())
        fprintf(stderr, "[laph] bicgstab reliable updates: all converged %d, deep drop %d, quorum %d, count %d\n", why[0],
                why[1], why[2], why[3]);
    // steps still owed after the last iteration, then the increment of every RHS (inactive
    // ones hold what they had when they stopped)
    if (nowed) launch_el(c, k_fold_x_bs<XP, SP>, n, xhi, xlo, owed(1, nowed), w.Vh, w.R, (const Scal *)w.sc);
    launch_el(c, k_fold_x<XP>, n, xhi, xlo, w.Vh, w.R, (const Scal *)w.sc, 1);
}

// FP64 BiCGStab (Sec. IV) on the even-odd system for the masked RHS, x_hi accumulating the
// solution (through an FP64 increment folded at the end); the iterated residual decides
// convergence (the full system's true residual judges the answer afterwards).  Returns
// when every RHS is inactive or maxiter is reached.
template <class GP, class CP>
void bicgstab_plain(Work &w, const Op<S64, GP, CP> &op, Vec xhi, Vec rhi, int maxiter, int check_every,
                    std::vector<Scal> &hs)
{
    using SP = S64;
    Vec r = w.make("r", SP::bytes, false), r0 = w.make("r0", SP::bytes, false), p = w.make("p", SP::bytes, false);
    Vec v = w.make("v", SP::bytes, false), s = w.make("s", SP::bytes, false), t = w.make("t", SP::bytes, false);
    Vec xlo = w.make("xlo", SP::bytes, false);
    long n = w.Vh * w.R;
    int nblk = (int)red_blocks(n);
    laph_ctx *c = w.c;
    // r_hi holds the current FP64 residual of the masked RHS
    launch_red(c, k_bicg_init<SP, SP>, n, rhi, r, r0, p, xlo, w.Vh, w.R, w.part, (const Scal *)w.sc);
    launch_fin(c, k_fin_init, w.R, (const double *)w.part, nblk, w.R, w.sc);
    read_scal(c, w.sc, hs);
    std::vector<double> r2_min(w.R);
    for (int q = 0; q < w.R; q++) r2_min[q] = hs[q].r2;
    for (int it = 0; it < maxiter;) {
        int chunk = std::min(check_every, maxiter - it);
        for (int k = 0; k < chunk; k++) {
            op.mhat(p, v);
            launch_red(c, k_dot<SP>, n, r0, v, w.Vh, w.R, w.part);
            launch_fin(c, k_fin_alpha, w.R, (const double *)w.part, nblk, w.R, w.sc);
            launch_el(c, k_s_update<SP>, n, r, v, s, w.Vh, w.R, (const Scal *)w.sc);
            op.mhat(s, t);
            launch_red(c, k_dot_ts<SP>, n, t, s, w.Vh, w.R, w.part);
            launch_fin(c, k_fin_omega, w.R, (const double *)w.part, nblk, w.R, w.sc);
            launch_red(c, k_xr_update<SP, SP>, n, xlo, p, s, t, r, r0, w.Vh, w.R, w.part, (const Scal *)w.sc);
            launch_fin(c, k_fin_beta, w.R, (const double *)w.part, nblk, w.R, w.sc, 1);
            launch_el(c, k_p_update<SP>, n, p, r, v, w.Vh, w.R, (const Scal *)w.sc);
        }
        it += chunk;
        read_scal(c, w.sc, hs);
        // divergence: the iterated residual grew 1e4-fold above its minimum; the RHS is
        // handed to the fallback
        bool diverged = false, any = false;
        int nact = 0;
        double worst = 0;
        for (int q = 0; q < w.R; q++) {
            if (!hs[q].active) continue;
            r2_min[q] = std::min(r2_min[q], hs[q].r2);
            if (!(hs[q].r2 <= 1e8 * r2_min[q])) {
                hs[q].active = 0;
                hs[q].breakdown = 1;
                diverged = true;
                continue;
            }
            any = true;
            nact++;
            worst = std::max(worst, hs[q].tol2 > 0 ? std::sqrt(hs[q].r2 / hs[q].tol2) : 0.0);
        }
        if (diverged) write_scal(c, w.sc, hs);
        if (laph_verbose() && (it % 256 < check_every || !any))
            fprintf(stderr, "[laph] bicgstab it=%d active=%d/%d max |r|/target=%.3g\n", it, nact, w.R, worst);
        if (!any) break;
    }
    // fold the increment (all RHS: inactive ones hold their last increment)
    launch_el(c, k_fold_x<SP>, n, xhi, xlo, w.Vh, w.R, (const Scal *)w.sc, 1);
}

// BiCGStab in storage SP on the even-odd system: the fused low-precision iteration with
// FP64 reliable updates, or plain FP64
template <class SP, class GP, class CP, class XP>
void bicgstab(Work &w, const Op<SP, GP, CP> &lo, const Op64 &hi, Vec bhat, Vec xhi, Vec rhi, Vec tmp64,
              int maxiter, int reliable_every, int check_every, std::vector<Scal> &hs)
{
    if constexpr (std::is_same<SP, S64>::value) {
        (void)hi;
        (void)bhat;
        (void)tmp64;
        (void)reliable_every;
        bicgstab_plain<GP, CP>(w, lo, xhi, rhi, maxiter, check_every, hs);
    } else {
        (void)check_every;
        bicgstab_fused<SP, GP, CP, XP>(w, lo, hi, bhat, xhi, rhi, tmp64, maxiter, reliable_every, hs);
    }
}

// CG on Mhat^dag Mhat x = Mhat^dag bhat in storage SP for the masked RHS, starting from
// xhi (FP64).  Lower precisions fold their FP32 increment into xhi at FP64 reliable
// updates (every reliable_every iterations, after a drop of the recursive residual by
// kDelta, or when it reaches the target); the FP64 even-odd residual decides.
template <class SP, class GP, class CP, class XP>
void cgnr(Work &w, const Op<SP, GP, CP> &lo, const Op64 &hi, Vec bhat, Vec xhi, Vec reshi, Vec rhi, Vec tmp64,
          int maxiter, int reliable_every, int check_every, std::vector<Scal> &hs)
{
    constexpr bool plain = std::is_same<SP, S64>::value;
    const bool nrm = SP::kNorm;
    laph_ctx *c = w.c;
    long n = w.Vh * w.R;
    int nblk = (int)red_blocks(n);
    Vec r = w.make("cg.r", SP::bytes, nrm), p = w.make("cg.p", SP::bytes, nrm), res = w.make("cg.res", SP::bytes, nrm);
    Vec q = w.make("cg.q", SP::bytes, nrm), to = w.make("cg.to", SP::bytes, nrm);
    Vec y = plain ? w.make("cg.y", SP::bytes, nrm) : Vec{};  // M^dag q (the fused form never stores it)
    Vec xlo = w.make("cg.xlo", XP::bytes, false);
    // FP64 residual of the masked RHS reshi = bhat - M xhi (res: the same in storage
    // precision); the normal residual r = M^dag res by the storage-precision operator, as
    // in the reliable updates
    (void)rhi;
    true_eo_residual<SP>(w, hi, bhat, xhi, tmp64, reshi, 0, res);
    lo.mhat_dag(res, r, to);
    launch_red(c, k_cg_start<SP, XP>, n, r, p, res, xlo, w.Vh, w.R, w.part, (const Scal *)w.sc);
    launch_fin(c, k_fin_cg_init, w.R, (const double *)w.part, nblk, w.R, w.sc);
    const double kDelta2 = w.delta2;
    read_scal(c, w.sc, hs);
    if (laph_verbose())
        fprintf(stderr, "[laph] cgnr init rhs0: active=%d r2hi=%.3e rho=%.3e r2=%.3e b2=%.3e tol2=%.3e\n", hs[0].active,
                hs[0].r2hi, hs[0].rho.x, hs[0].r2, hs[0].b2, hs[0].tol2);
    std::vector<double> r2_last(w.R);
    for (int k = 0; k < w.R; k++) r2_last[k] = hs[k].r2;
    int since = 0;
    // lower precisions test the update rule after every iteration: between two tests the
    // recursive residual must not fall far below what the storage precision can follow
    if (!plain) check_every = 1;
    // one iteration: q = M p, alpha, y = M^dag q, x/res/r updates, beta (plain: and p)
    // low precision with the LDS-staged kernel: |q|^2 and the first step of M^dag q come
    // from the epilogue of the hop that forms q
    // (the caller picks R so that the multi-RHS kernel fits: every low-precision solve
    // runs the fused form)
    const bool fuse = !plain;
    double *part_hop = nullptr, *part_pre = nullptr;
    int nblk_hop = 0;
    if (fuse) {
        nblk_hop = (int)lds_dag_blocks(c, prec_of<SP>(), w.R);
        part_hop = (double *)ctx_named(c, "slv.part_hop", sizeof(double) * nblk_hop * w.R);
        part_pre = (double *)ctx_named(c, "slv.part_pre", sizeof(double) * kChunks * w.R);
    }
    // the fused body leaves the steps x += alpha p to the direction update; with K direction
    // buffers (a ring) each update writes the new direction into the next buffer and keeps
    // the old ones, and every K-th update takes the K owed steps at once: the FP32 increment
    // is read and written every K-th iteration only (graph replay keeps one captured body per
    // direction buffer)
    const int K = !fuse ? 1 : w.dirs > 0 ? w.dirs : kDefaultDirs;
    Vec pb[kMaxDirs];
    pb[0] = p;
    for (int j = 1; j < K; j++) pb[j] = w.make(("cg.p" + std::to_string(j + 1)).c_str(), SP::bytes, nrm);
    int cur = 0;            // p is pb[cur]
    bool step_now = false;  // this iteration's step is owed to x
    bool orth = false;      // the next direction update first makes p orthogonal to r
    int nowed = 0;          // earlier steps owed too, their directions in pb[cur - 1], ..., pb[cur - nowed]
    // cnt directions, latest first, starting first buffers behind p's
    auto owed_dirs = [&](int first, int cnt) {
        Dirs d;
        for (int j = 0; j < cnt; j++) d.d[j] = K == 1 ? p : pb[((cur - first - j) % K + K) % K];
        d.n = cnt;
        return d;
    };
    auto body = [&](const Op<SP, GP, CP> &op) {
        if constexpr (!plain) {
            // M p with |q|^2 and A^-1 gamma_5 q from its epilogue; M^dag q feeding the CG
            // update directly (partials of the fused epilogues are block-major, pre-reduced
            // to kChunks per RHS)
            op.mhat_prep(p, q, to, part_hop);
            hipLaunchKernelGGL(k_prereduce, dim3(kChunks), dim3(kBS), 0, c->stream, (const double *)part_hop,
                               nblk_hop, w.R, part_pre);
            launch_fin(c, k_fin_cg_alpha, w.R, (const double *)part_pre, kChunks, w.R, w.sc, 1);
            op.mhat_dag_cg(q, to, r, (const Scal *)w.sc, part_hop);
            hipLaunchKernelGGL(k_prereduce, dim3(kChunks), dim3(kBS), 0, c->stream, (const double *)part_hop,
                               nblk_hop, w.R, part_pre);
            launch_fin(c, k_fin_cg_beta, w.R, (const double *)part_pre, kChunks, w.R, w.sc, 0, 1, 1);
        } else {
            op.mhat(p, q);
            launch_red(c, k_normsq<SP>, n, q, w.Vh, w.R, w.part);
            launch_fin(c, k_fin_cg_alpha, w.R, (const double *)w.part, nblk, w.R, w.sc, 0);
            op.mhat_dag(q, y, to);
            launch_red(c, k_cg_update<SP, XP, true>, n, xlo, p, res, q, r, y, w.Vh, w.R, w.part, (const Scal *)w.sc);
            launch_fin(c, k_fin_cg_beta, w.R, (const double *)w.part, nblk, w.R, w.sc, 1, 0, 0);
            launch_el(c, k_cg_p<SP, XP>, n, p, owed_dirs(0, 1), r, xlo, w.Vh, w.R, (const Scal *)w.sc, 0, 0);
        }
    };
    // lagged decisions (low precision): the scalars of iteration k are copied to a pinned
    // slot behind its hops; the update rule at iteration k reads iteration k - 1's slot,
    // long complete, so the host never waits for the queue to drain (an update or the
    // convergence test comes one iteration later, which the rule tolerates)
    const bool lag = !plain;
    int nupd = 0;  // reliable updates (reported under LAPH_VERBOSE)
    Scal *pin = lag ? pinned_scal(c, w.R) : nullptr;
    int slot = 0;
    bool prev_ok = false;  // the other slot holds the previous iteration's scalars
    hipGraphExec_t gexecs[kMaxDirs] = {};  // body captured with p in each buffer
    const bool graph_ok = w.use_graph && !c->timing;
    if (graph_ok && !c->cap_stream) LAPH_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    struct GraphGuard {
        hipGraphExec_t *g;
        ~GraphGuard()
        {
            for (int k = 0; k < kMaxDirs; k++)
                if (g[k]) (void)hipGraphExecDestroy(g[k]);
        }
    } guard{gexecs};
    for (int it = 0; it < maxiter;) {
        int chunk = std::min(check_every, maxiter - it);
        for (int k = 0; k < chunk; k++) {
            hipGraphExec_t &gexec = gexecs[cur];
            if (gexec) {
                LAPH_HIP(hipGraphLaunch(gexec, c->stream));
            } else if (graph_ok) {
                // record the body once on the capture stream, then replay it
                hipStream_t main = c->stream;
                bool timing = c->timing;
                Op<SP, GP, CP> cap = lo;
                cap.st = c->cap_stream;
                c->stream = c->cap_stream;
                c->timing = false;
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
                if (e == hipSuccess) {
                    body(cap);
                    e = hipStreamEndCapture(c->cap_stream, &g);
                }
                c->stream = main;
                c->timing = timing;
                LAPH_HIP(e);
                e = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                LAPH_HIP(e);
                LAPH_HIP(hipGraphLaunch(gexec, c->stream));
            } else {
                body(lo);
            }
        }
        it += chunk;
        since += chunk;
        step_now = fuse;
        if (lag) {
            LAPH_HIP(hipMemcpyAsync(pin + (size_t)slot * w.R, w.sc, sizeof(Scal) * w.R, hipMemcpyDeviceToHost,
                                    c->stream));
            LAPH_HIP(hipEventRecord(c->pin_ev[slot], c->stream));
            const int use = prev_ok ? slot ^ 1 : slot;
            LAPH_HIP(hipEventSynchronize(c->pin_ev[use]));
            std::copy(pin + (size_t)use * w.R, pin + (size_t)use * w.R + w.R, hs.begin());
            prev_ok = true;
            slot ^= 1;
        } else {
            read_scal(c, w.sc, hs);
        }
        UpdateVote vote;
        for (int k = 0; k < w.R; k++)
            if (hs[k].active) vote.add(hs[k], r2_last[k], kDelta2);
        const bool any = vote.nact > 0, want_update = vote.want();
        const int nact = vote.nact;
        const double worst = vote.worst;
        if (laph_verbose() && (it % 256 < check_every || !any || laph_verbose_level() > 1))
            fprintf(stderr, "[laph] cgnr it=%d active=%d/%d max |res|/target=%.3g rhs0: rho=%.3e alpha=%.3e r2=%.3e "
                    "aux=%.3e upd=%d\n", it, nact, w.R, worst, hs[0].rho.x, hs[0].alpha.x, hs[0].r2, hs[0].aux.x,
                    (int)want_update);
        if (!any) break;
        if (plain) continue;
        if (want_update || since >= reliable_every) {
            nupd++;
            // reliable update between the residual and the direction update: fold the
            // increment, replace r and res by FP64 residuals, take beta from the new |r|^2
            // and keep the old direction orthogonal to the new residual
            // FP64 true residual of the even-odd system; the normal residual M^dag res is
            // computed by the low-precision operator, in which r is stored anyway
            if (step_now)  // the fold takes the steps still owed to x
                launch_el(c, k_fold_x_step<XP, SP>, n, xhi, xlo, owed_dirs(0, 1 + nowed), w.Vh, w.R,
                          (const Scal *)w.sc);
            else
                launch_el(c, k_fold_x<XP>, n, xhi, xlo, w.Vh, w.R, (const Scal *)w.sc, 0);
            // the FP64 residual, and res = the same in storage precision
            true_eo_residual<SP>(w, hi, bhat, xhi, tmp64, reshi, 0, res);
            step_now = false;
            nowed = 0;
            lo.mhat_dag(res, r, to);
            launch_red(c, k_normsq2<SP>, n, r, res, w.Vh, w.R, w.part);
            launch_fin(c, k_fin_cg_reset, w.R, (const double *)w.part, nblk, w.R, w.sc);
            launch_red(c, k_dot<SP>, n, r, p, w.Vh, w.R, w.part);
            launch_fin(c, k_fin_orth, w.R, (const double *)w.part, nblk, w.R, w.sc);
            orth = true;  // the direction update makes p orthogonal to the new r
            since = 0;
            read_scal(c, w.sc, hs);
            prev_ok = false;  // the slots predate the update
            bool left = false;
            for (int k = 0; k < w.R; k++) {
                left |= hs[k].active != 0;
                r2_last[k] = hs[k].r2;
            }
            if (!left) break;
        }
        if (K == 1 || !step_now) {
            launch_el(c, k_cg_p<SP, XP>, n, p, owed_dirs(0, 1), r, xlo, w.Vh, w.R, (const Scal *)w.sc,
                      step_now ? 1 : 0, orth ? 1 : 0);
            orth = false;
        } else {
            // the new direction goes into the next buffer: a free one, or with every buffer
            // holding an owed direction the oldest, whose step (with all others) is taken now
            const bool take = nowed + 1 == K;
            const int nxt = (cur + 1) % K;
            launch_el(c, k_cg_p<SP, XP>, n, pb[nxt], owed_dirs(0, 1 + nowed), r, xlo, w.Vh, w.R, (const Scal *)w.sc,
                      take ? K : 0, 0);
            cur = nxt;
            p = pb[cur];
            nowed = take ? 0 : nowed + 1;
        }
    }
    if (laph_verbose() && !plain) fprintf(stderr, "[laph] cgnr reliable updates: %d\n", nupd);
    // steps still owed after the last iteration (the latest takes the current alpha)
    if (nowed)
        launch_el(c, k_fold_x_step<XP, SP>, n, xhi, xlo, owed_dirs(1, nowed), w.Vh, w.R, (const Scal *)w.sc);
    launch_el(c, k_fold_x<XP>, n, xhi, xlo, w.Vh, w.R, (const Scal *)w.sc, 1);
}

// ----------------------------------------------------------- full-system helpers
// b (canonical) -> b_e, b_o (gamma_4 applied), bhat
void prepare_rhs(laph_ctx *c, const Op64 &hi, const double *eta, int R, Vec be, Vec bo, Vec bhat, Vec te)
{
    spinor_to_eo(c, eta, R, 4, (double2 *)be.d, (double2 *)bo.d, c->tg_in);
    launch_clover_apply<S64, C64>(c, hi.cinv(0), be.d, nullptr, te.d, nullptr, hi.Vh, R, 0, c->stream);
    DslashArgs a = hi.base(1);
    a.in = te.d;
    a.out = bhat.d;
    a.x = bo.d;
    a.clov = hi.cinv(1);
    a.a = 1;
    a.c = -1;
    launch_dslash<S64, G64, C64>(c, M_INV_OF_SUM, a, c->stream);
}

// x_e = A_ee^-1 (b_e - D_eo x_o)
void reconstruct(laph_ctx *c, const Op64 &hi, Vec be, Vec xo, Vec xe)
{
    DslashArgs a = hi.base(0);
    a.in = xo.d;
    a.out = xe.d;
    a.x = be.d;
    a.clov = hi.cinv(0);
    a.a = 1;
    a.c = -1;
    launch_dslash<S64, G64, C64>(c, M_INV_OF_SUM, a, c->stream);
}

// K x for EO halves: out_p = A_pp x_p + D x_other
void apply_K(laph_ctx *c, const Op64 &hi, Vec xe, Vec xo, Vec oe, Vec oo)
{
    for (int par = 0; par < 2; par++) {
        DslashArgs a = hi.base(par);
        a.in = par ? xe.d : xo.d;
        a.x = par ? xo.d : xe.d;
        a.out = par ? oo.d : oe.d;
        a.clov = hi.cl(par);
        a.a = 1;
        a.c = 1;
        launch_dslash<S64, G64, C64>(c, M_CLOV_ADD, a, c->stream);
    }
}

// per-RHS |b - K x|^2 and |b|^2 over both parities (host result)
void full_residual(Work &w, const Op64 &hi, Vec be, Vec bo, Vec xe, Vec xo, Vec te, Vec to, Vec re,
                   std::vector<double> &r2, std::vector<double> &b2)
{
    laph_ctx *c = w.c;
    long n = w.Vh * w.R;
    int nblk = (int)red_blocks(n);
    apply_K(c, hi, xe, xo, te, to);
    std::vector<double> part((size_t)nblk * w.R);
    r2.assign(w.R, 0.0);
    b2.assign(w.R, 0.0);
    for (int par = 0; par < 2; par++) {
        launch_red(c, k_resid64<S64>, n, par ? bo : be, par ? to : te, re, Vec{}, w.Vh, w.R, w.part, (const Scal *)w.sc,
                   1);
        LAPH_HIP(hipMemcpyAsync(part.data(), w.part, sizeof(double) * part.size(), hipMemcpyDeviceToHost, c->stream));
        LAPH_HIP(hipStreamSynchronize(c->stream));
        for (int q = 0; q < w.R; q++)
            for (int b = 0; b < nblk; b++) r2[q] += part[(size_t)b * w.R + q];
        launch_red(c, k_normsq<S64>, n, par ? bo : be, w.Vh, w.R, w.part);
        LAPH_HIP(hipMemcpyAsync(part.data(), w.part, sizeof(double) * part.size(), hipMemcpyDeviceToHost, c->stream));
        LAPH_HIP(hipStreamSynchronize(c->stream));
        for (int q = 0; q < w.R; q++)
            for (int b = 0; b < nblk; b++) b2[q] += part[(size_t)b * w.R + q];
    }
}

// ------------------------------------------------------------------ flexible GMRES
// One right-hand side, FP64 basis.  Kernels over n = 12 Vh complex numbers.
constexpr int kFgBS = 256;

// part[i][b] = sum over chunk b of conj(v_i) w, i = blockIdx.y (v_i at vb + i * n)
__global__ __launch_bounds__(kFgBS) void k_fg_dots(const double2 *__restrict__ vb, const double2 *__restrict__ w,
                                                   long n, long chunk, double2 *__restrict__ part)
{
    const double2 *v = vb + (size_t)blockIdx.y * n;
    long beg = blockIdx.x * chunk, end = std::min(n, beg + chunk);
    double re = 0, im = 0;
    for (long e = beg + threadIdx.x; e < end; e += blockDim.x) {
        double2 a = v[e], b = w[e];
        re += a.x * b.x + a.y * b.y;
        im += a.x * b.y - a.y * b.x;
    }
    __shared__ double sr[kFgBS], si[kFgBS];
    sr[threadIdx.x] = re;
    si[threadIdx.x] = im;
    __syncthreads();
    for (int h = kFgBS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sr[threadIdx.x] += sr[threadIdx.x + h];
            si[threadIdx.x] += si[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = make_double2(sr[0], si[0]);
}

// w -= sum_i h_i v_i  (nv vectors at vb + i * n, h on the device)
__global__ void k_fg_axpy(double2 *__restrict__ w, const double2 *__restrict__ vb, const double2 *__restrict__ h,
                          int nv, long n)
{
    long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (e >= n) return;
    double2 acc = w[e];
    for (int i = 0; i < nv; i++) acc = csub(acc, cmul(h[i], vb[(size_t)i * n + e]));
    w[e] = acc;
}

// dst = s (a - b)   (b may be null)
__global__ void k_fg_lin(double2 *dst, const double2 *a, const double2 *b, double s, long n)
{
    long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (e >= n) return;
    double2 v = a[e];
    if (b) v = csub(v, b[e]);
    dst[e] = cscale(v, s);
}

struct Fgmres {
    laph_ctx *c;
    const Op64 &hi;
    laph_ptnet *net;
    float bct;
    long n;
    int nblk;
    long chunk;
    double2 *part, *hdev;
    std::vector<double2> hpart;

    // h[i] = <v_i, w> for i < nv (host result, fixed summation order)
    void dots(const double2 *vb, int nv, const double2 *w, std::vector<std::complex<double>> &h)
    {
        hipLaunchKernelGGL(k_fg_dots, dim3(nblk, nv), dim3(kFgBS), 0, c->stream, vb, w, n, chunk, part);
        LAPH_HIP(hipGetLastError());
        hpart.resize((size_t)nblk * nv);
        LAPH_HIP(hipMemcpyAsync(hpart.data(), part, sizeof(double2) * hpart.size(), hipMemcpyDeviceToHost,
                                c->stream));
        LAPH_HIP(hipStreamSynchronize(c->stream));
        h.assign(nv, 0.0);
        for (int i = 0; i < nv; i++)
            for (int b = 0; b < nblk; b++) h[i] += std::complex<double>(hpart[(size_t)i * nblk + b].x,
                                                                          hpart[(size_t)i * nblk + b].y);
    }
    void axpy(double2 *w, const double2 *vb, const std::vector<std::complex<double>> &h)
    {
        std::vector<double2> hh(h.size());
        for (size_t i = 0; i < h.size(); i++) hh[i] = make_double2(h[i].real(), h[i].imag());
        LAPH_HIP(hipMemcpyAsync(hdev, hh.data(), sizeof(double2) * hh.size(), hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(k_fg_axpy, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, w, vb, (const double2 *)hdev,
                           (int)h.size(), n);
        LAPH_HIP(hipGetLastError());
        LAPH_HIP(hipStreamSynchronize(c->stream));  // hh is reused by the next call
    }
    double norm(const double2 *w)
    {
        std::vector<std::complex<double>> h;
        dots(w, 1, w, h);
        return std::sqrt(std::max(h[0].real(), 0.0));
    }
    void lin(double2 *dst, const double2 *a, const double2 *b, double s)
    {
        hipLaunchKernelGGL(k_fg_lin, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, dst, a, b, s, n);
        LAPH_HIP(hipGetLastError());
    }
    // z = P_o N(E_o A_oo v): the net approximates K^-1 and Mhat^-1 = (K^-1)_oo A_oo
    void precondition(const double2 *v, double2 *z, double2 *tmp, float2 *na, float2 *nb)
    {
        launch_clover_apply<S64, C64>(c, hi.cl(1), v, nullptr, tmp, nullptr, hi.Vh, 1, 0, c->stream);
        eo_to_net(c, tmp, 1, na);
        ptnet_forward(c, net, bct, na, nb, 1, 0);
        net_to_eo(c, nb, 1, z);
    }
};

// Right-preconditioned flexible GMRES(m) (Saad) on Mhat x = bhat with classical Gram-Schmidt
// applied twice; restarts recompute the FP64 residual.  Returns the iterations spent and
// whether |bhat - Mhat x| <= tol_abs was reached.
int fgmres(laph_ctx *c, const Op64 &hi, laph_ptnet *net, Vec bhat, Vec x, Vec r, double tol_abs, int maxiter,
           int m, bool &reached)
{
    long Vh = c->g.Vh;
    long n = 12 * Vh;
    Fgmres f{c, hi, net, (float)c->cur->prm.bc_t, n, 0, 0, nullptr, nullptr, {}};
    f.chunk = std::max<long>(kFgBS * 16, (n + 511) / 512);
    f.chunk = (f.chunk + kFgBS - 1) / kFgBS * kFgBS;
    f.nblk = (int)((n + f.chunk - 1) / f.chunk);
    f.part = (double2 *)ctx_named(c, "fg.part", sizeof(double2) * f.nblk * (m + 1));
    f.hdev = (double2 *)ctx_named(c, "fg.h", sizeof(double2) * (m + 1));
    double2 *vb = (double2 *)ctx_named(c, "fg.V", sizeof(double2) * n * (m + 1));
    double2 *zb = (double2 *)ctx_named(c, "fg.Z", sizeof(double2) * n * m);
    double2 *tmp = (double2 *)ctx_named(c, "fg.tmp", sizeof(double2) * n);
    float2 *na = (float2 *)ctx_named(c, "fg.na", sizeof(float2) * 12 * c->g.V);
    float2 *nb = (float2 *)ctx_named(c, "fg.nb", sizeof(float2) * 12 * c->g.V);
    double2 *xd = (double2 *)x.d, *rd = (double2 *)r.d;
    using C = std::complex<double>;
    int it = 0;
    reached = false;
    while (it < maxiter) {
        hi.mhat(x, r);
        f.lin(rd, (const double2 *)bhat.d, rd, 1.0);
        double beta = f.norm(rd);
        if (laph_verbose_level() > 1) fprintf(stderr, "[laph] fgmres it %d: |r| = %.3e (target %.3e)\n", it, beta, tol_abs);
        if (!(beta > tol_abs)) {
            reached = std::isfinite(beta);
            break;
        }
        f.lin(vb, rd, nullptr, 1.0 / beta);
        std::vector<std::vector<C>> H(m + 1, std::vector<C>(m, 0.0));
        std::vector<double> cs(m);
        std::vector<C> sn(m), g(m + 1, 0.0);
        g[0] = beta;
        int k = 0;
        bool stop = false;
        for (int j = 0; j < m && it < maxiter; j++) {
            double2 *vj = vb + (size_t)j * n, *zj = zb + (size_t)j * n, *w = vb + (size_t)(j + 1) * n;
            f.precondition(vj, zj, tmp, na, nb);
            hi.mhat(Vec{zj}, Vec{w});
            std::vector<C> h1, h2;
            f.dots(vb, j + 1, w, h1);
            f.axpy(w, vb, h1);
            f.dots(vb, j + 1, w, h2);
            f.axpy(w, vb, h2);
            for (int i = 0; i <= j; i++) H[i][j] = h1[i] + h2[i];
            double hn = f.norm(w);
            H[j + 1][j] = hn;
            it++;
            k = j + 1;
            if (hn > 0 && std::isfinite(hn)) f.lin(w, w, nullptr, 1.0 / hn);
            for (int i = 0; i < j; i++) {  // previous rotations
                C t = cs[i] * H[i][j] + sn[i] * H[i + 1][j];
                H[i + 1][j] = -std::conj(sn[i]) * H[i][j] + cs[i] * H[i + 1][j];
                H[i][j] = t;
            }
            C a = H[j][j];
            double bb = hn, rr = std::sqrt(std::norm(a) + bb * bb);
            if (std::abs(a) == 0.0) {
                cs[j] = 0;
                sn[j] = 1;
            } else {
                cs[j] = std::abs(a) / rr;
                sn[j] = (a / std::abs(a)) * bb / rr;
            }
            H[j][j] = cs[j] * a + sn[j] * bb;
            H[j + 1][j] = 0;
            g[j + 1] = -std::conj(sn[j]) * g[j];
            g[j] = cs[j] * g[j];
            double est = std::abs(g[j + 1]);
            if (!std::isfinite(est) || !(hn > 0)) {
                stop = true;
                break;
            }
            if (est <= tol_abs) break;
        }
        // y = H^-1 g (upper triangular), x += Z y
        std::vector<C> y(k);
        for (int i = k - 1; i >= 0; i--) {
            C s2 = g[i];
            for (int l = i + 1; l < k; l++) s2 -= H[i][l] * y[l];
            y[i] = s2 / H[i][i];
        }
        bool finite = true;
        for (auto &v : y) finite = finite && std::isfinite(v.real()) && std::isfinite(v.imag());
        if (!finite) break;
        for (auto &v : y) v = -v;
        f.axpy(xd, zb, y);
        if (stop) break;
    }
    if (it >= maxiter || !reached) {
        hi.mhat(x, r);
        f.lin(rd, (const double2 *)bhat.d, rd, 1.0);
        double beta = f.norm(rd);
        reached = std::isfinite(beta) && beta <= tol_abs;
    }
    return it;
}

// ------------------------------------------------------------- hop_apply helpers
// b = a in storage precision SP for every right-hand side (FP64 parity layout in)
template <class SP>
__global__ __launch_bounds__(kBS) void k_store_lo(Vec a, Vec b, long Vh, int R)
{
    long tid = blockIdx.x * (long)kBS + threadIdx.x;
    if (tid >= Vh * R) return;
    long i = tid / R;
    int rr = (int)(tid - i * R);
    Cx<double> v[12];
    ld_site<S64>(a, Vh, R, i, rr, v);
    st_site<SP>(b, Vh, R, i, rr, v);
}

// b = a as FP64 (storage precision SP in, FP64 parity layout out)
template <class SP>
__global__ __launch_bounds__(kBS) void k_load_lo(Vec a, Vec b, long Vh, int R)
{
    long tid = blockIdx.x * (long)kBS + threadIdx.x;
    if (tid >= Vh * R) return;
    long i = tid / R;
    int rr = (int)(tid - i * R);
    Cx<double> v[12];
    ld_site<SP>(a, Vh, R, i, rr, v);
    st_site<S64>(b, Vh, R, i, rr, v);
}

// ------------------------------------------------------------------ autotuning
// Times the even-odd hopping kernel (fused clover-inverse epilogue, the launch that
// dominates an iteration) for every block size R and, for the LDS-staged kernel, every
// tile of S sites x R lanes with S R in {64, 128, 256}; keeps the fastest tile per R and
// the R with the lowest time per right-hand side.
template <class SP, class GP, class CP>
std::vector<laph_tune_entry> tune_hopping(laph_ctx *c, int prec)
{
    DiracCache &dc = *c->cur;
    const long Vh = c->g.Vh;
    const bool low = !std::is_same<SP, S64>::value;
    std::vector<int> Rs;
    for (int R : low ? std::vector<int>{4, 8, 16, 32} : std::vector<int>{1, 2, 4, 8, 16, 32})
        if (R <= max_block_rhs(c, prec)) Rs.push_back(R);
    LAPH_CHECK(!Rs.empty(), LAPH_EINVAL, "lattice too large for the hopping kernels' 32-bit offsets");
    std::vector<laph_tune_entry> out;
    hipEvent_t e0, e1;
    LAPH_HIP(hipEventCreate(&e0));
    LAPH_HIP(hipEventCreate(&e1));
    const bool timing = c->timing;
    c->timing = false;
    double best = 1e300;
    int bestR = Rs.back();
    try {
        for (int R : Rs) {
            Work w{c, Vh, R, nullptr, nullptr};
            Vec in = w.make("tune.in", SP::bytes, SP::kNorm), o = w.make("tune.out", SP::bytes, SP::kNorm);
            Vec x = w.make("tune.x", SP::bytes, SP::kNorm), te = w.make("tune.te", SP::bytes, SP::kNorm);
            for (Vec v : {in, x}) {
                LAPH_HIP(hipMemsetAsync(v.d, 0, (size_t)12 * Vh * R * SP::bytes, c->stream));
                if (v.n) LAPH_HIP(hipMemsetAsync(v.n, 0, (size_t)Vh * R * 4, c->stream));
            }
            Op<SP, GP, CP> op{c, c->stream, Vh, R,
                              std::is_same<GP, G64>::value ? dc.g64.p : nullptr,
                              std::is_same<CP, C64>::value ? (const char *)dc.clinv.p : nullptr,
                              nullptr, -0.5 / dc.prm.xi, -0.5, dc.prm.bc_t, te};
            op.lk12 = (const float4 *)dc.lk12.p;
            op.claos = (const float4 *)dc.claos.p;
            op.tgauge = dc.tgauge ? 1 : 0;
            std::vector<int> Ss;
            if (low)
                for (int S = std::max(1, 64 / R); S * R <= 256; S *= 2) Ss.push_back(S);
            else
                Ss.push_back(0);
            int bestS = Ss.front();
            double bestR_ms = 1e300;
            for (int S : Ss) {
                if (low) c->lds_tile[{prec, R}] = S;
                op.dslash(M_INV_AFTER, 1, in, o, &x, 1.0, -1.0, 0);  // warm-up
                const int reps = 3;
                LAPH_HIP(hipEventRecord(e0, c->stream));
                for (int k = 0; k < reps; k++) op.dslash(M_INV_AFTER, 1, in, o, &x, 1.0, -1.0, 0);
                LAPH_HIP(hipEventRecord(e1, c->stream));
                LAPH_HIP(hipEventSynchronize(e1));
                float ms = 0;
                LAPH_HIP(hipEventElapsedTime(&ms, e0, e1));
                double per = ms / reps / R;
                out.push_back(laph_tune_entry{R, S, per});
                if (per < bestR_ms) {
                    bestR_ms = per;
                    bestS = S;
                }
            }
            if (low) c->lds_tile[{prec, R}] = bestS;
            if (bestR_ms < best) {
                best = bestR_ms;
                bestR = R;
            }
        }
    } catch (...) {
        c->timing = timing;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    c->timing = timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->tuned_R[prec] = bestR;
    return out;
}

std::vector<laph_tune_entry> tune_for(laph_ctx *c, int prec)
{
    switch (prec) {
    case LAPH_PREC_F64: return tune_hopping<S64, G64, C64>(c, prec);
    case LAPH_PREC_F32: return tune_hopping<S32, G32, C32>(c, prec);
    case LAPH_PREC_F16: return tune_hopping<S16, G32, C32>(c, prec);
    default: return tune_hopping<SB16, G32, C32>(c, prec);
    }
}

template <class SP, class GP, class CP, class XP>
void solve_batch(laph_ctx *c, const double *eta, double *x, int R, int nreal, const laph_solver *sv,
                 laph_solve_stats *stats)
{
    long Vh = c->g.Vh;
    DiracCache &dc = *c->cur;
    Work w{c, Vh, R, nullptr, nullptr};
    w.use_graph = sv->use_graph != 0;
    if (sv->reliable_delta > 0) w.delta2 = sv->reliable_delta * sv->reliable_delta;
    w.dirs = sv->dir_buffers;
    w.sc = (Scal *)ctx_named(c, "slv.scal", sizeof(Scal) * R);
    w.part = (double *)ctx_named(c, "slv.part", sizeof(double) * kMaxBlocks * R * 4);

    Op64 hi{c, c->stream, Vh, R, dc.g64.p, (const char *)dc.clinv.p, (const char *)dc.clov.p,
            -0.5 / dc.prm.xi, -0.5, dc.prm.bc_t, w.make("te64", 16, false)};
    Vec be = w.make("be", 16, false), bo = w.make("bo", 16, false), bhat = w.make("bhat", 16, false);
    Vec xe = w.make("xe", 16, false), xo = w.make("xo", 16, false), rhi = w.make("rhi", 16, false);
    Vec tmp = w.make("tmp64", 16, false), tmp2 = w.make("tmp64b", 16, false);

    prepare_rhs(c, hi, eta, R, be, bo, bhat, hi.te);

    std::vector<Scal> hs(R);
    // |bhat|^2
    long n = Vh * R;
    launch_red(c, k_normsq<S64>, n, bhat, Vh, R, w.part);
    launch_fin(c, k_fin_r2hi, R, (const double *)w.part, (int)red_blocks(n), R, w.sc, 1);
    read_scal(c, w.sc, hs);
    std::vector<double> eo_tol(R, 0.5 * sv->tol);
    for (int q = 0; q < R; q++) {
        double b2 = hs[q].b2;
        hs[q] = Scal{};
        hs[q].b2 = b2;
        hs[q].active = (q < nreal && b2 > 0) ? 1 : 0;
        hs[q].tol2 = eo_tol[q] * eo_tol[q] * b2;
    }
    write_scal(c, w.sc, hs);
    // x_hi = 0 or the network's guess, r_hi = bhat
    if (sv->net && sv->solver != LAPH_SOLVER_FGMRES)
        ptnet_initial_guess(c, (laph_ptnet *)sv->net, (float)dc.prm.bc_t, eta, R, (double2 *)xo.d);
    else
        LAPH_HIP(hipMemsetAsync(xo.d, 0, (size_t)12 * Vh * R * 16, c->stream));
    w.x_zero = !(sv->net && sv->solver != LAPH_SOLVER_FGMRES);
    launch_el(c, k_copy64, n, bhat, rhi, Vh, R, (const Scal *)w.sc, 1);

    std::vector<int> iters(R, 0), fallback(R, 0);
    std::vector<double> r2, b2;
    const int check_every = 8;
    int reliable = sv->reliable_every > 0 ? sv->reliable_every : 50;
    std::vector<int> done(R, 0);
    for (int q = 0; q < R; q++) done[q] = !hs[q].active;

    Op<SP, GP, CP> lo{c, c->stream, Vh, R,
                      std::is_same<GP, G64>::value ? dc.g64.p : nullptr,
                      std::is_same<CP, C64>::value ? (const char *)dc.clinv.p : nullptr,
                      nullptr, -0.5 / dc.prm.xi, -0.5, dc.prm.bc_t,
                      w.make("te_lo", SP::bytes, SP::kNorm)};
    lo.lk12 = (const float4 *)dc.lk12.p;
    lo.claos = (const float4 *)dc.claos.p;
    lo.tgauge = dc.tgauge ? 1 : 0;

    // Attempts: BiCGStab (Sec. IV) for every RHS that has not failed it, then CG on the
    // normal equations (the paper's fallback) in the same precision for the RHS whose
    // BiCGStab broke down or diverged; the last attempt is plain FP64 CGNR.  After each
    // attempt the FP64 true residual of the full system decides, and an RHS that misses
    // the bar continues from its current x with a tighter even-odd target.
    std::vector<int> bicg_failed(R, 0), fg_failed(R, 0);
    Vec reshi = w.make("reshi", 16, false);
    auto set_active = [&](auto pred) {
        int na = 0;
        for (int q = 0; q < R; q++) {
            hs[q].active = (!done[q] && pred(q)) ? 1 : 0;
            hs[q].iters = 0;
            hs[q].breakdown = 0;
            na += hs[q].active;
        }
        write_scal(c, w.sc, hs);
        return na;
    };
    for (int attempt = 0; attempt < 4; attempt++) {
        const bool last = attempt == 3;
        const char *what = "";
        if (sv->solver == LAPH_SOLVER_FGMRES && !last && R == 1 && !done[0] && !fg_failed[0]) {
            bool ok = false;
            int m = sv->restart > 0 ? sv->restart : 24;
            iters[0] += fgmres(c, hi, (laph_ptnet *)sv->net, bhat, xo, rhi, eo_tol[0] * std::sqrt(hs[0].b2),
                               sv->maxiter, m, ok);
            w.x_zero = false;
            if (!ok) fg_failed[0] = 1;
            what = "fgmres";
        }
        if (sv->solver == LAPH_SOLVER_BICGSTAB && !last &&
            set_active([&](int q) { return !bicg_failed[q]; }) > 0) {
            true_eo_residual(w, hi, bhat, xo, tmp, rhi, 0);
            read_scal(c, w.sc, hs);
            bicgstab<SP, GP, CP, XP>(w, lo, hi, bhat, xo, rhi, tmp, sv->maxiter, reliable, check_every, hs);
            read_scal(c, w.sc, hs);
            for (int q = 0; q < R; q++)
                if (!done[q] && !bicg_failed[q]) {
                    iters[q] += hs[q].iters;
                    if (hs[q].breakdown) bicg_failed[q] = 1;
                }
            what = "bicgstab";
        }
        bool cg_all = sv->solver == LAPH_SOLVER_CGNR || last;
        if (set_active([&](int q) { return cg_all || bicg_failed[q] || fg_failed[q]; }) > 0) {
            if (last)
                cgnr<S64, G64, C64, S64>(w, hi, hi, bhat, xo, reshi, rhi, tmp, std::max(sv->maxiter, 5000), 0,
                                         check_every, hs);
            else
                cgnr<SP, GP, CP, XP>(w, lo, hi, bhat, xo, reshi, rhi, tmp, std::max(sv->maxiter, 5000), reliable,
                                     check_every, hs);
            read_scal(c, w.sc, hs);
            for (int q = 0; q < R; q++)
                if (!done[q] && (cg_all || bicg_failed[q] || fg_failed[q])) {
                    iters[q] += hs[q].iters;
                    if (sv->solver != LAPH_SOLVER_CGNR || last) fallback[q] = 1;
                }
            what = last ? "cgnr-fp64" : "cgnr";
        }
        reconstruct(c, hi, be, xo, xe);
        full_residual(w, hi, be, bo, xe, xo, tmp, tmp2, rhi, r2, b2);
        if (laph_verbose()) {
            double mx = 0;
            int mi = 0;
            for (int q = 0; q < R; q++) {
                double rel = b2[q] > 0 ? std::sqrt(r2[q] / b2[q]) : 0.0;
                if (rel > mx) mx = rel;
                mi = std::max(mi, iters[q]);
            }
            fprintf(stderr, "[laph] attempt %d (%s): max true residual %.3e, max iters %d\n", attempt, what, mx, mi);
        }
        bool all = true;
        for (int q = 0; q < R; q++) {
            if (done[q]) continue;
            double rel = b2[q] > 0 ? std::sqrt(r2[q] / b2[q]) : 0.0;
            if (rel <= sv->tol) {
                done[q] = 1;
            } else {
                all = false;
                // tighten the even-odd target by the observed ratio and continue from x
                double eo_rel = hs[q].b2 > 0 ? std::sqrt(std::max(hs[q].r2hi, hs[q].r2) / hs[q].b2) : 0;
                double ratio = (eo_rel > 0 && rel > 0 && std::isfinite(eo_rel)) ? eo_rel / rel : 1.0;
                eo_tol[q] = std::min(eo_tol[q] * 0.5, sv->tol * ratio * 0.5);
                hs[q].tol2 = eo_tol[q] * eo_tol[q] * hs[q].b2;
            }
        }
        if (all) break;
    }
    spinor_from_eo(c, (const double2 *)xe.d, (const double2 *)xo.d, R, 0, x, c->tg_out);
    for (int q = 0; q < nreal; q++) {
        if (!stats) break;
        double rel = b2[q] > 0 ? std::sqrt(r2[q] / b2[q]) : 0.0;
        stats[q].iters = iters[q];
        stats[q].fallback_used = fallback[q];
        stats[q].true_resid = rel;
        stats[q].status = rel <= sv->tol ? LAPH_OK : LAPH_ENOCONV;
    }
    for (int q = 0; q < nreal; q++) {
        double rel = b2[q] > 0 ? std::sqrt(r2[q] / b2[q]) : 0.0;
        if (!(rel <= sv->tol)) laph_fail(LAPH_ENOCONV, "rhs %d: true residual %.3e > tol %.3e", q, rel, sv->tol);
    }
}

}  // namespace

// ------------------------------------------------------------------- setup / ABI

static bool dirac_cache_holds(const DiracCache &dc, const double *U, uint64_t fp, const laph_dirac *d)
{
    return dc.valid && dc.U == U && dc.fp == fp && dc.prm.m0 == d->m0 && dc.prm.xi == d->xi &&
           dc.prm.c_sw == d->c_sw && dc.prm.bc_t == d->bc_t;
}

// (re)build cache dc for the field Ub when it does not hold the operator of the caller's
// field Ukey (fingerprint fp) with parameters d.  The cache is keyed by the field's
// contents as well as its address: a caller may free a field and allocate another one at
// the same address.
static void prepare_cache(laph_ctx *c, DiracCache &dc, const double *Ukey, uint64_t fp, const double *Ub,
                          const laph_dirac *d, bool need_f32)
{
    const bool f32 = need_f32 || dc.has_f32;
    const size_t need = cache_unit_bytes(c->g, dc.tgauge, f32);
    const void *held = dc.unit.p;
    cache_unit(c, dc, need);  // pins the unit; a new or moved unit is rebuilt
    if (dc.unit.p != held || dc.has_f32 != f32) {
        dc.valid = false;
        dc.f32 = false;
        cache_carve(c, dc, dc.tgauge, f32);
    }
    if (!dirac_cache_holds(dc, Ukey, fp, d)) {
        links_to_eo(c, Ub, (double2 *)dc.g64.p);
        clover_build(c, Ub, d, (double *)dc.clov.p, (double *)dc.clinv.p);
        dc.valid = true;
        dc.U = Ukey;
        dc.fp = fp;
        dc.prm = *d;
        dc.f32 = false;
    }
    if (need_f32 && !dc.f32) {
        build_lp_operator(c, (const double2 *)dc.g64.p, (const double *)dc.clinv.p, (float4 *)dc.lk12.p,
                          (float *)dc.claos.p);
        dc.f32 = true;
    }
}

void dirac_prepare(laph_ctx *c, const double *U, const laph_dirac *d, bool need_f32)
{
    c->dc.tgauge = false;
    prepare_cache(c, c->dc, U, gauge_fingerprint(c, U), U, d, need_f32);
}

void dirac_prepare_tgauge(laph_ctx *c, const double *U, const laph_dirac *d)
{
    DiracCache &dc = c->dct;
    dc.tgauge = true;
    const uint64_t fp = gauge_fingerprint(c, U);
    const size_t need = cache_unit_bytes(c->g, true, true);
    const void *held = dc.unit.p;
    cache_unit(c, dc, need);
    if (dc.unit.p != held || !dc.has_f32) {
        dc.valid = false;
        dc.f32 = false;
        cache_carve(c, dc, true, true);
    }
    const bool same_field = dc.valid && dc.U == U && dc.fp == fp;
    if (!same_field) {
        dc.valid = false;
        tgauge_fix(c, U, (double *)dc.gG.p, (double *)dc.gU.p);
    }
    prepare_cache(c, dc, U, fp, (const double *)dc.gU.p, d, true);
}

static void check_dirac(const laph_dirac *d)
{
    LAPH_CHECK(d && d->xi > 0 && std::isfinite(d->m0) && std::isfinite(d->c_sw) && std::isfinite(d->bc_t),
               LAPH_EINVAL, "invalid Dirac parameters");
}

extern "C" int laph_dirac_apply(laph_ctx_t c, const double *U, const laph_dirac *d, int op, const double *in,
                                double *out, int n)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(U && in && out && n > 0, LAPH_EINVAL, "null pointer or n <= 0");
    LAPH_CHECK(op == LAPH_OP_K || op == LAPH_OP_OMEGA || op == LAPH_OP_KDAG, LAPH_EINVAL, "bad op");
    check_dirac(d);
    dirac_prepare(c, U, d, false);
    long Vh = c->g.Vh;
    DiracCache &dc = c->dc;
    // fields in batches the FP64 hopping kernel addresses with 32-bit offsets
    const int B = std::min(n, max_block_rhs(c, LAPH_PREC_F64));
    LAPH_CHECK(B >= 1, LAPH_EINVAL, "lattice too large for the hopping kernel's 32-bit offsets");
    size_t bytes = (size_t)12 * Vh * B * 16;
    Vec xe{ctx_named(c, "app.xe", bytes)}, xo{ctx_named(c, "app.xo", bytes)};
    Vec oe{ctx_named(c, "app.oe", bytes)}, oo{ctx_named(c, "app.oo", bytes)};
    int gin = op == LAPH_OP_KDAG ? 5 : 0;
    int gout = op == LAPH_OP_KDAG ? 5 : (op == LAPH_OP_OMEGA ? 4 : 0);
    const size_t field = (size_t)c->g.V * 24;
    for (int f0 = 0; f0 < n; f0 += B) {
        const int nb = std::min(B, n - f0);
        Op64 hi{c, c->stream, Vh, nb, dc.g64.p, (const char *)dc.clinv.p, (const char *)dc.clov.p,
                -0.5 / dc.prm.xi, -0.5, dc.prm.bc_t, Vec{}};
        spinor_to_eo(c, in + f0 * field, nb, gin, (double2 *)xe.d, (double2 *)xo.d);
        apply_K(c, hi, xe, xo, oe, oo);
        spinor_from_eo(c, (const double2 *)oe.d, (const double2 *)oo.d, nb, gout, out + f0 * field);
    }
    LAPH_HIP(hipStreamSynchronize(c->stream));
    LAPH_API_END(c)
}

// ----------------------------------------------------------- workspace sizes
// Each function below sums the scratch buffers its entry point takes from the workspace
// (an upper bound where the path depends on the run: every branch is counted).
static size_t vec_bytes(long Vh, int R, int prec)
{
    const int sb = prec == LAPH_PREC_F64 ? 16 : prec == LAPH_PREC_F32 ? 8 : 4;
    size_t s = ws_align((size_t)12 * Vh * R * sb);
    if (prec == LAPH_PREC_F16) s += ws_align((size_t)Vh * R * 4);
    return s;
}

size_t dirac_cache_bytes(const Geom &g, bool tgauge) { return cache_unit_bytes(g, tgauge, true); }

size_t apply_scratch_bytes(laph_ctx *c, int n_fields)
{
    const int B = std::min(n_fields, max_block_rhs(c, LAPH_PREC_F64));
    return ws_align(8) + 4 * ws_align((size_t)12 * c->g.Vh * std::max(B, 1) * 16);
}

size_t hop_scratch_bytes(laph_ctx *c, const laph_hop *h, int R)
{
    const long Vh = c->g.Vh;
    size_t s = ws_align(8) + 6 * ws_align((size_t)12 * Vh * R * 16);
    if (h->precision != LAPH_PREC_F64) {
        s += 5 * vec_bytes(Vh, R, h->precision);
        const int S = h->sites_per_block > 0 ? h->sites_per_block : lds_tile_sites(c, h->precision, R);
        const int nq = h->mode == LAPH_HOP_INV_DOT ? 3 : 1;  // partial sums per field
        s += ws_align(sizeof(double) * nq * ((Vh + S - 1) / S) * R) + ws_align(sizeof(Scal) * R);
    }
    return s;
}

size_t tune_scratch_bytes(laph_ctx *c, int prec)
{
    const bool low = prec != LAPH_PREC_F64;
    size_t s = 0;
    for (int R : low ? std::vector<int>{4, 8, 16, 32} : std::vector<int>{1, 2, 4, 8, 16, 32})
        if (R <= max_block_rhs(c, prec)) s += 4 * vec_bytes(c->g.Vh, R, prec);  // names grow with R
    return s;
}

size_t solve_scratch_bytes(laph_ctx *c, int n_rhs, const laph_solver *sv)
{
    const long Vh = c->g.Vh, V = c->g.V;
    const int prec = sv->precision;
    const bool low = prec != LAPH_PREC_F64;
    const int xp = low ? LAPH_PREC_F32 : LAPH_PREC_F64;
    const bool fg = sv->solver == LAPH_SOLVER_FGMRES;
    laph_ptnet *net = (laph_ptnet *)sv->net;
    size_t s = ws_align(8);  // fingerprint
    int R = fg ? 1 : sv->block_rhs;
    // the solve tunes first when block_rhs = 0 finds no tuned block size: the tile it will
    // pick is not known yet, so the epilogue partials are sized for the smallest candidate
    const bool will_tune = R == 0 && low && !c->tuned_R.count(prec);
    if (R == 0) {
        if (!c->tuned_R.count(prec)) s += tune_scratch_bytes(c, prec);
        R = c->tuned_R.count(prec) ? c->tuned_R[prec] : 32;
    }
    R = std::max(1, std::min(R, max_block_rhs(c, prec)));
    int Rb = R;
    while (Rb / 2 >= n_rhs) Rb /= 2;  // the first (largest) batch
    // padding of a ragged tail batch
    const int tail = n_rhs % R;
    if (tail || n_rhs < R) {
        const int nreal = tail ? tail : n_rhs;
        int Rt = R;
        while (Rt / 2 >= nreal) Rt /= 2;
        if (nreal < Rt) s += 2 * ws_align((size_t)V * 24 * 8 * Rt);
    }
    const bool guess = net && !fg;
    if (low && guess) s += ws_align((size_t)V * 24 * 8 * Rb);  // rotated sources
    if (net) s += ptnet_scratch_bytes(c->g, net, guess ? Rb : 1, 3);
    // solve_batch
    s += ws_align(sizeof(Scal) * Rb) + ws_align(sizeof(double) * kMaxBlocks * Rb * 4);
    s += 10 * vec_bytes(Vh, Rb, LAPH_PREC_F64) + vec_bytes(Vh, Rb, prec);
    if (guess) s += 2 * ws_align(sizeof(float2) * 12 * V * Rb);
    if (sv->solver == LAPH_SOLVER_BICGSTAB && !low) s += 6 * vec_bytes(Vh, Rb, prec) + vec_bytes(Vh, Rb, xp);
    if (sv->solver == LAPH_SOLVER_BICGSTAB && low) {
        // r, r0, v, t and the ring of K (p, s) pairs; epilogue partials (three rows per RHS)
        const int K = sv->dir_buffers > 0 ? sv->dir_buffers : kDefaultDirs;
        s += (4 + 2 * K) * vec_bytes(Vh, Rb, prec) + vec_bytes(Vh, Rb, xp);
        const int S = will_tune ? std::max(1, 64 / Rb) : lds_tile_sites(c, prec, Rb);
        const long nb = std::max<long>((Vh + S - 1) / S, nblocks_for(Vh * Rb, kBS));
        s += ws_align(sizeof(double) * 3 * nb * Rb) + ws_align(sizeof(double) * 3 * kChunks * Rb);
    }
    if (fg) {
        const long n = 12 * Vh;
        const int m = sv->restart > 0 ? sv->restart : 24;
        long chunk = std::max<long>(kFgBS * 16, (n + 511) / 512);
        chunk = (chunk + kFgBS - 1) / kFgBS * kFgBS;
        const size_t nblk = (n + chunk - 1) / chunk;
        s += ws_align(sizeof(double2) * nblk * (m + 1)) + ws_align(sizeof(double2) * (m + 1)) +
             ws_align(sizeof(double2) * n * (m + 1)) + ws_align(sizeof(double2) * n * m) +
             ws_align(sizeof(double2) * n) + 2 * ws_align(sizeof(float2) * 12 * V);
    }
    // CG on the normal equations in the storage precision (the production form, and the
    // fallback of the other solvers)
    if (low) {
        const int K = sv->dir_buffers > 0 ? sv->dir_buffers : kDefaultDirs;
        s += (5 + (K - 1)) * vec_bytes(Vh, Rb, prec) + vec_bytes(Vh, Rb, xp);
        const int S = will_tune ? std::max(1, 64 / Rb) : lds_tile_sites(c, prec, Rb);
        s += ws_align(sizeof(double) * ((Vh + S - 1) / S) * Rb) + ws_align(sizeof(double) * kChunks * Rb);
    }
    // the last attempt: plain FP64 CG (the same names at FP64 size)
    s += 7 * vec_bytes(Vh, Rb, LAPH_PREC_F64);
    return s;
}

// One even-odd hopping launch of the solver's kernels on caller fields (see laph.h).
template <class SP>
static void hop_launch_lo(laph_ctx *c, const DiracCache &dc, const laph_hop *h, int R, Vec in, const Vec *x, Vec out,
                          Vec out2, Vec r, Vec y, const Scal *sc, double *partial)
{
    Op<SP, G32, C32> lo{c, c->stream, c->g.Vh, R, nullptr, nullptr, nullptr, -0.5 / dc.prm.xi, -0.5, dc.prm.bc_t,
                        Vec{}};
    lo.lk12 = (const float4 *)dc.lk12.p;
    lo.claos = (const float4 *)dc.claos.p;
    lo.tgauge = dc.tgauge ? 1 : 0;
    const int p = h->parity;
    MrArgs m = lo.mr_args(p, in, out, x, h->a, h->c, h->gamma5);
    int mode = M_PLAIN;
    switch (h->mode) {
    case LAPH_HOP_INV: mode = M_INV_AFTER; break;
    case LAPH_HOP_INV_DAG:
        mode = M_INV_AFTER_DAG;
        m.out2 = out2.d;
        m.out2_nrm = out2.n;
        m.partial = partial;
        break;
    case LAPH_HOP_PLAIN_CG:
        mode = M_PLAIN_CG;
        m.out = nullptr;
        m.out_nrm = nullptr;
        m.cg_r = r.d;
        m.cg_r_nrm = r.n;
        m.sc = sc;
        m.partial = partial;
        break;
    case LAPH_HOP_INV_DOT:
        mode = M_INV_AFTER_DOT;
        m.dot_y = y.d;
        m.dot_y_nrm = y.n;
        m.partial = partial;
        break;
    default: break;
    }
    launch_dslash_mr<SP>(c, mode, m, c->stream);
}

extern "C" int laph_hop_apply(laph_ctx_t c, const double *U, const laph_dirac *d, const laph_hop *h, const double *in,
                              const double *x, double *out, double *out2, const double *alpha, double *norm2, int n)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(U && h && in && out, LAPH_EINVAL, "null pointer");
    check_dirac(d);
    LAPH_CHECK(h->precision >= LAPH_PREC_F64 && h->precision <= LAPH_PREC_BF16, LAPH_EINVAL, "bad precision");
    LAPH_CHECK(h->mode >= LAPH_HOP_PLAIN && h->mode <= LAPH_HOP_INV_DOT, LAPH_EINVAL, "bad mode");
    LAPH_CHECK(h->parity == 0 || h->parity == 1, LAPH_EINVAL, "parity must be 0 or 1");
    LAPH_CHECK(h->walk == 0 || h->walk == 1, LAPH_EINVAL, "walk must be 0 or 1");
    LAPH_CHECK(h->sites_per_block >= 0, LAPH_EINVAL, "sites_per_block must be >= 0");
    LAPH_CHECK(n >= 1 && n <= 32 && (n & (n - 1)) == 0, LAPH_EINVAL, "n_fields must be a power of two <= 32");
    LAPH_CHECK(n <= max_block_rhs(c, h->precision), LAPH_EINVAL, "%d fields exceed the kernel's 32-bit offsets", n);
    const bool low = h->precision != LAPH_PREC_F64;
    const bool fused = h->mode == LAPH_HOP_INV_DAG || h->mode == LAPH_HOP_PLAIN_CG || h->mode == LAPH_HOP_INV_DOT;
    const bool dot = h->mode == LAPH_HOP_INV_DOT;
    LAPH_CHECK(low || !fused, LAPH_EINVAL, "fused epilogues exist for the low precisions only");
    LAPH_CHECK(!fused || x, LAPH_EINVAL, "the fused epilogues need the own-site operand x");
    LAPH_CHECK(h->mode != LAPH_HOP_INV_DAG || (out2 && h->c != 0), LAPH_EINVAL, "INV_DAG needs out2 and c != 0");
    LAPH_CHECK(h->mode != LAPH_HOP_PLAIN_CG || alpha, LAPH_EINVAL, "PLAIN_CG needs alpha");
    LAPH_CHECK(!dot || (out2 && norm2), LAPH_EINVAL, "INV_DOT needs the field y in out2 and norm2");
    if (h->temporal_gauge)
        dirac_prepare_tgauge(c, U, d);
    else
        dirac_prepare(c, U, d, low);
    const DiracCache &dc = h->temporal_gauge ? c->dct : c->dc;
    const double *G = h->temporal_gauge ? (const double *)dc.gG.p : nullptr;
    struct Reset {
        laph_ctx *c;
        ~Reset()
        {
            c->walk_mode = 0;
            c->tile_override = 0;
        }
    } reset{c};
    c->walk_mode = h->walk;
    c->tile_override = low ? h->sites_per_block : 0;

    const long Vh = c->g.Vh;
    const int R = n, p = h->parity;
    const size_t half64 = (size_t)12 * Vh * R * 16;
    Vec e64{ctx_named(c, "hop.e64", half64)}, o64{ctx_named(c, "hop.o64", half64)};
    Vec ie{ctx_named(c, "hop.ie", half64)}, io{ctx_named(c, "hop.io", half64)};
    Vec xh{ctx_named(c, "hop.xh", half64)};
    // the input lives on the other parity, x and r on the output parity
    spinor_to_eo(c, in, R, 0, (double2 *)ie.d, (double2 *)io.d, G);
    Vec in64 = p ? ie : io;
    if (x) {
        spinor_to_eo(c, x, R, 0, (double2 *)e64.d, (double2 *)o64.d, G);
        LAPH_HIP(hipMemcpyAsync(xh.d, p ? o64.d : e64.d, half64, hipMemcpyDeviceToDevice, c->stream));
    }
    Vec r64{ctx_named(c, "hop.r64", half64)};
    if (h->mode == LAPH_HOP_PLAIN_CG || dot) {
        // r (PLAIN_CG: the residual in out) or y (INV_DOT: the field in out2), parity p
        spinor_to_eo(c, dot ? out2 : out, R, 0, (double2 *)e64.d, (double2 *)o64.d, G);
        LAPH_HIP(hipMemcpyAsync(r64.d, p ? o64.d : e64.d, half64, hipMemcpyDeviceToDevice, c->stream));
    }
    const int nq = dot ? 3 : 1;  // partial sums per field
    std::vector<double> nrm((size_t)nq * R, 0.0);
    Vec res64 = p ? o64 : e64;   // result half in FP64
    Vec zero64 = p ? e64 : o64;  // the other parity of every output: zero
    if (!low) {
        Op64 hi{c, c->stream, Vh, R, dc.g64.p, (const char *)dc.clinv.p, (const char *)dc.clov.p, -0.5 / dc.prm.xi,
                -0.5, dc.prm.bc_t, Vec{}};
        DslashArgs a = hi.base(p);
        a.in = in64.d;
        a.x = x ? xh.d : nullptr;
        a.out = res64.d;
        a.clov = hi.cinv(p);
        a.a = h->a;
        a.c = h->c;
        a.g5d = h->gamma5;
        launch_dslash<S64, G64, C64>(c, h->mode == LAPH_HOP_INV ? M_INV_AFTER : M_PLAIN, a, c->stream);
    } else {
        const int sb = h->precision == LAPH_PREC_F32 ? 8 : 4;
        const bool nm = h->precision == LAPH_PREC_F16;
        auto lov = [&](const char *name) {
            Vec v{ctx_named(c, std::string("hop.") + name, (size_t)12 * Vh * R * sb)};
            if (nm) v.n = (float *)ctx_named(c, std::string("hop.") + name + ".n", (size_t)Vh * R * 4);
            return v;
        };
        Vec lin = lov("lin"), lx = lov("lx"), lout = lov("lout"), lout2 = lov("lout2"), lr = lov("lr");
        const long nl = Vh * R;
        Scal *sc = nullptr;
        double *part = nullptr;
        const long nblk = lds_dag_blocks(c, h->precision, R);
        if (fused) {
            part = (double *)ctx_named(c, "hop.part", sizeof(double) * nblk * R * nq);
            if (h->mode == LAPH_HOP_PLAIN_CG) {
                std::vector<Scal> hs(R);
                for (int q = 0; q < R; q++) {
                    hs[q] = Scal{};
                    hs[q].active = 1;
                    hs[q].alpha = make_double2(alpha[q], 0.0);
                }
                sc = (Scal *)ctx_named(c, "hop.scal", sizeof(Scal) * R);
                LAPH_HIP(hipMemcpyAsync(sc, hs.data(), sizeof(Scal) * R, hipMemcpyHostToDevice, c->stream));
            }
        }
        auto run = [&](auto tag) {
            using SP = decltype(tag);
            launch_el(c, k_store_lo<SP>, nl, in64, lin, Vh, R);
            if (x) launch_el(c, k_store_lo<SP>, nl, xh, lx, Vh, R);
            // INV_DOT with y the caller's x itself: the kernel's y = x form
            const bool y_is_x = dot && (const double *)out2 == x;
            if (h->mode == LAPH_HOP_PLAIN_CG || (dot && !y_is_x)) launch_el(c, k_store_lo<SP>, nl, r64, lr, Vh, R);
            hop_launch_lo<SP>(c, dc, h, R, lin, x ? &lx : nullptr, lout, lout2, lr, y_is_x ? lx : lr, sc, part);
            launch_el(c, k_load_lo<SP>, nl, h->mode == LAPH_HOP_PLAIN_CG ? lr : lout, res64, Vh, R);
            if (h->mode == LAPH_HOP_INV_DAG) launch_el(c, k_load_lo<SP>, nl, lout2, r64, Vh, R);
        };
        if (h->precision == LAPH_PREC_F32)
            run(S32{});
        else if (h->precision == LAPH_PREC_F16)
            run(S16{});
        else
            run(SB16{});
        if (fused) {
            std::vector<double> hp((size_t)nblk * R * nq);
            LAPH_HIP(hipMemcpyAsync(hp.data(), part, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, c->stream));
            LAPH_HIP(hipStreamSynchronize(c->stream));
            for (long b = 0; b < nblk; b++)  // block-major: [block][value][field]
                for (int q = 0; q < nq * R; q++) nrm[q] += hp[(size_t)b * nq * R + q];
        }
    }
    LAPH_HIP(hipMemsetAsync(zero64.d, 0, half64, c->stream));
    spinor_from_eo(c, (const double2 *)e64.d, (const double2 *)o64.d, R, 0, out, G);
    if (h->mode == LAPH_HOP_INV_DAG) {
        // out2 from r64 (its result half) and the zeroed half
        spinor_from_eo(c, p ? (const double2 *)zero64.d : (const double2 *)r64.d,
                       p ? (const double2 *)r64.d : (const double2 *)zero64.d, R, 0, out2, G);
    }
    LAPH_HIP(hipStreamSynchronize(c->stream));
    if (norm2 && dot) {
        // rows of the sums are value-major: Re <y, out> of every field, then Im, then |out|^2
        for (int q = 0; q < R; q++)
            for (int e = 0; e < 3; e++) norm2[3 * q + e] = nrm[(size_t)e * R + q];
    } else if (norm2) {
        for (int q = 0; q < R; q++) norm2[q] = nrm[q];
    }
    LAPH_API_END(c)
}

extern "C" int dirac_solve(laph_ctx_t c, const double *U, const laph_dirac *d, const double *eta, double *x,
                           int n_rhs, const laph_solver *sv, laph_solve_stats *stats)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(U && eta && x && sv && n_rhs > 0, LAPH_EINVAL, "null pointer or n_rhs <= 0");
    check_dirac(d);
    LAPH_CHECK(sv->tol > 0 && sv->maxiter > 0, LAPH_EINVAL, "tol and maxiter must be positive");
    LAPH_CHECK(sv->reliable_delta >= 0 && sv->reliable_delta < 1, LAPH_EINVAL, "reliable_delta must be in [0, 1)");
    LAPH_CHECK(sv->dir_buffers >= 0 && sv->dir_buffers <= kMaxDirs, LAPH_EINVAL, "dir_buffers must be in [0, 8]");
    LAPH_CHECK(sv->precision >= LAPH_PREC_F64 && sv->precision <= LAPH_PREC_BF16, LAPH_EINVAL, "bad precision");
    LAPH_CHECK(sv->solver == LAPH_SOLVER_BICGSTAB || sv->solver == LAPH_SOLVER_CGNR ||
                   sv->solver == LAPH_SOLVER_FGMRES,
               LAPH_EINVAL, "unknown solver kind");
    LAPH_CHECK(sv->block_rhs >= 0, LAPH_EINVAL, "block_rhs must be >= 0");
    int R = sv->block_rhs;
    bool low = sv->precision != LAPH_PREC_F64;
    // low-precision solves run in temporal gauge (the hop skips the unit time links); the
    // FP64 path keeps the caller's gauge
    const bool tg = low;
    if (tg)
        dirac_prepare_tgauge(c, U, d);
    else
        dirac_prepare(c, U, d, low);
    struct CurGuard {
        laph_ctx *c;
        ~CurGuard()
        {
            c->cur = &c->dc;
            c->tg_in = c->tg_out = nullptr;
        }
    } cur_guard{c};
    c->cur = tg ? &c->dct : &c->dc;
    const double *G = tg ? (const double *)c->dct.gG.p : nullptr;
    // eta' = G eta and x = G^dag x' inside the layout conversions of the solve; the network's
    // initial guess reads the rotated source itself, which is then formed beforehand
    const bool guess = sv->net && sv->solver != LAPH_SOLVER_FGMRES;
    c->tg_in = guess ? nullptr : G;
    c->tg_out = G;
    if (sv->solver == LAPH_SOLVER_FGMRES || sv->net) {
        laph_ptnet *net = (laph_ptnet *)sv->net;
        LAPH_CHECK(net && net->layers > 0, LAPH_EINVAL, "FGMRES needs a network");
        LAPH_CHECK(net->device == c->device, LAPH_EINVAL, "network and context on different devices");
        // the network is gauge equivariant: in temporal gauge it takes the rotated field
        ptnet_prepare(c, net, tg ? (const double *)c->dct.gU.p : U);
    }
    if (sv->solver == LAPH_SOLVER_FGMRES) {
        LAPH_CHECK(sv->restart >= 0 && sv->restart <= 256, LAPH_EINVAL, "restart must be in 0..256");
        R = 1;  // one right-hand side at a time
    }
    LAPH_CHECK(R <= 32 && (R & (R - 1)) == 0, LAPH_EINVAL, "block_rhs must be 0 or a power of two <= 32");
    if (R == 0) {
        if (!c->tuned_R.count(sv->precision)) tune_for(c, sv->precision);
        R = c->tuned_R[sv->precision];
    }
    // the hopping kernels address a block's spinors with 32-bit offsets: the block shrinks
    // to the largest power of two they reach on this lattice
    R = std::min(R, max_block_rhs(c, sv->precision));
    LAPH_CHECK(R >= 1, LAPH_EINVAL, "lattice too large for the hopping kernels' 32-bit offsets");
    long V = c->g.V;
    int first_err = LAPH_OK;
    for (int base = 0; base < n_rhs; base += R) {
        int nreal = std::min(R, n_rhs - base);
        int Rb = R;
        while (Rb / 2 >= nreal) Rb /= 2;  // smallest power of two holding the tail
        const double *eb = eta + (size_t)base * V * 24;
        double *xb = x + (size_t)base * V * 24;
        const double *src = eb;
        double *dst = xb;
        if (nreal < Rb) {
            // pad the batch with zero sources (inactive from the start)
            size_t fb = (size_t)V * 24 * sizeof(double);
            double *pe = (double *)ctx_named(c, "slv.pad_eta", fb * Rb);
            double *px = (double *)ctx_named(c, "slv.pad_x", fb * Rb);
            LAPH_HIP(hipMemsetAsync(pe, 0, fb * Rb, c->stream));
            LAPH_HIP(hipMemcpyAsync(pe, eb, fb * nreal, hipMemcpyDeviceToDevice, c->stream));
            src = pe;
            dst = px;
        }
        laph_solve_stats *st = stats ? stats + base : nullptr;
        if (tg && guess) {
            double *te = (double *)ctx_named(c, "slv.tg_eta", (size_t)V * 24 * sizeof(double) * Rb);
            tgauge_spinor(c, G, src, te, Rb, 0);
            src = te;
        }
        try {
            switch (sv->precision) {
            case LAPH_PREC_F64: solve_batch<S64, G64, C64, S64>(c, src, dst, Rb, nreal, sv, st); break;
            case LAPH_PREC_F32: solve_batch<S32, G32, C32, S32>(c, src, dst, Rb, nreal, sv, st); break;
            case LAPH_PREC_F16: solve_batch<S16, G32, C32, S32>(c, src, dst, Rb, nreal, sv, st); break;
            default: solve_batch<SB16, G32, C32, S32>(c, src, dst, Rb, nreal, sv, st); break;
            }
        } catch (const LaphError &e) {
            if (e.code != LAPH_ENOCONV) throw;
            if (first_err == LAPH_OK) first_err = e.code;
        }
        if (dst != xb) {
            size_t fb = (size_t)V * 24 * sizeof(double);
            LAPH_HIP(hipMemcpyAsync(xb, dst, fb * nreal, hipMemcpyDeviceToDevice, c->stream));
        }
    }
    LAPH_HIP(hipStreamSynchronize(c->stream));
    if (first_err != LAPH_OK) return first_err;
    LAPH_API_END(c)
}

extern "C" int laph_autotune(laph_ctx_t c, const double *U, const laph_dirac *d, int precision,
                             laph_tune_report *rep)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(U && rep, LAPH_EINVAL, "null pointer");
    check_dirac(d);
    LAPH_CHECK(precision >= LAPH_PREC_F64 && precision <= LAPH_PREC_BF16, LAPH_EINVAL, "bad precision");
    dirac_prepare(c, U, d, precision != LAPH_PREC_F64);
    std::vector<laph_tune_entry> e = tune_for(c, precision);
    memset(rep, 0, sizeof(*rep));
    rep->n = (int)std::min<size_t>(e.size(), LAPH_TUNE_MAX);
    for (int k = 0; k < rep->n; k++) rep->e[k] = e[k];
    rep->best_block_rhs = c->tuned_R[precision];
    rep->best_sites_per_block =
        precision == LAPH_PREC_F64 ? 0 : lds_tile_sites(c, precision, rep->best_block_rhs);
    LAPH_API_END(c)
}

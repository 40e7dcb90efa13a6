// laph_eigvecs: the N_v lowest eigenpairs of -Lap on every time slice by the
// Krylov-spectral restarted (thick-restart) Lanczos method of Sec. IV, batched over all
// slices so that one launch works on every slice at once.
//
//  * operator A = T_n(B), B = 1 + 2/(lamL - lamC)(Lap + lamC): the wanted low end of
//    -Lap becomes the top of A;
//  * full global reorthogonalisation by classical Gram-Schmidt; a pass is repeated while
//    it shrinks the vector by more than 1/kappa, kappa = sqrt(2), at most four repeats;
//  * Rayleigh-Ritz on the projected (real symmetric) matrix by parallel cyclic Jacobi,
//    one workgroup per slice;
//  * a Ritz pair with |A y - theta y| = beta_m |e_m^T s| < tol |A| is locked (kept in
//    the basis for orthogonalisation only); |A| is the largest |theta| seen;
//  * after a restart R_tot = N_v + (m - N_v)/2 vectors remain (locked + best Ritz
//    vectors) and the residual vector continues the Krylov sequence (this restart size
//    is our reading of the rule the paper takes from Wu and Simon; it bounds the kept
//    count by the converged count below and by m - locked - 12 above).
// Eigenvalues are Rayleigh quotients on -Lap; each eigenvector gets the phase that makes
// its first component with modulus >= 0.1 of the maximum real and positive.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "laplace.h"

namespace {

constexpr int GS_CH = 2048;  // rows per block in the Gram-Schmidt dot kernel

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

// partial[t][chunk][a] = sum_{rows in chunk} conj(Q[t][a][row]) w[t][row], a < cnt
__global__ __launch_bounds__(256) void k_gs_dots(const double2 *__restrict__ Q, long qslice, long n,
                                                 const double2 *__restrict__ w, int cnt, double2 *__restrict__ partial,
                                                 int nchunk, int pstride, const int *flags)
{
    int t = blockIdx.y;
    if (flags && !flags[t]) return;
    int ch = blockIdx.x;
    long row0 = (long)ch * GS_CH;
    int len = (int)min((long)GS_CH, n - row0);
    __shared__ double2 ws[GS_CH];
    const double2 *wt = w + t * n + row0;
    for (int r = threadIdx.x; r < len; r += blockDim.x) ws[r] = wt[r];
    __syncthreads();
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const double2 *Qt = Q + t * qslice + row0;
    for (int a = wave; a < cnt; a += nw) {
        const double2 *q = Qt + (long)a * n;
        double re = 0, im = 0;
        for (int r = lane; r < len; r += 64) {
            double2 u = q[r], v = ws[r];
            re += u.x * v.x + u.y * v.y;
            im += u.x * v.y - u.y * v.x;
        }
        for (int off = 32; off > 0; off >>= 1) {
            re += __shfl_down(re, off, 64);
            im += __shfl_down(im, off, 64);
        }
        if (lane == 0) partial[((long)t * nchunk + ch) * pstride + a] = make_double2(re, im);
    }
}

// coef[t][a] = sum over chunks; T[t][a][j] (+)= Re coef for a in [nlock[t], j]
__global__ void k_gs_fin(const double2 *__restrict__ partial, int nchunk, int pstride, int cnt,
                         double2 *__restrict__ coef, double *__restrict__ T, int m, int j, const int *__restrict__ nlock,
                         const int *flags, int accumulate)
{
    int t = blockIdx.x;
    if (flags && !flags[t]) return;
    for (int a = threadIdx.x; a < cnt; a += blockDim.x) {
        double2 s = make_double2(0, 0);
        for (int ch = 0; ch < nchunk; ch++) s = cadd(s, partial[((long)t * nchunk + ch) * pstride + a]);
        coef[(long)t * pstride + a] = s;
        if (j >= 0 && a >= nlock[t] && a <= j) {
            double *e = T + ((long)t * m + a) * m + j;
            *e = accumulate ? *e + s.x : s.x;
        }
    }
}

// w[t] -= sum_a Q[t][a] coef[t][a];  partial |w|^2 per block
__global__ __launch_bounds__(256) void k_gs_update(const double2 *__restrict__ Q, long qslice, long n,
                                                   double2 *__restrict__ w, int cnt, const double2 *__restrict__ coef,
                                                   int pstride, double *__restrict__ npart, const int *flags)
{
    int t = blockIdx.y;
    if (flags && !flags[t]) return;
    __shared__ double2 cs[256];
    __shared__ double red[256];
    long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double acc2 = 0;
    double2 v = make_double2(0, 0);
    if (row < n) v = w[t * n + row];
    for (int a0 = 0; a0 < cnt; a0 += 256) {
        int na = min(256, cnt - a0);
        __syncthreads();
        if ((int)threadIdx.x < na) cs[threadIdx.x] = coef[(long)t * pstride + a0 + threadIdx.x];
        __syncthreads();
        if (row < n) {
            const double2 *q = Q + t * qslice + (long)a0 * n + row;
            for (int a = 0; a < na; a++) v = csub(v, cmul(q[(long)a * n], cs[a]));
        }
    }
    if (row < n) {
        w[t * n + row] = v;
        acc2 = cnorm2(v);
    }
    red[threadIdx.x] = acc2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) npart[(long)t * gridDim.x + blockIdx.x] = red[0];
}

// partial |w|^2 (no update)
__global__ __launch_bounds__(256) void k_norm_slices(const double2 *__restrict__ w, long wslice, long n,
                                                     double *__restrict__ npart)
{
    int t = blockIdx.y;
    __shared__ double red[256];
    long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
    red[threadIdx.x] = row < n ? cnorm2(w[t * wslice + row]) : 0.0;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) npart[(long)t * gridDim.x + blockIdx.x] = red[0];
}

// norms: mode 0 -> nb = nrm (before the first pass); mode 1 -> after a pass: flag for
// another pass when nrm < nb / kappa (and passes remain), nb = nrm
__global__ void k_norm_fin(const double *__restrict__ npart, int nblk, int nt, double *nb, double *nrm,
                           int *flags, int mode, int last_pass)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    if (mode == 1 && flags && !flags[t]) return;
    double s = 0;
    for (int b = 0; b < nblk; b++) s += npart[(long)t * nblk + b];
    double v = sqrt(s);
    if (mode == 0) {
        nb[t] = v;
        nrm[t] = v;
        return;
    }
    const double kappa = 1.4142135623730951;
    bool again = (v < nb[t] / kappa) && !last_pass;
    nrm[t] = v;
    nb[t] = v;
    if (flags) flags[t] = again ? 1 : 0;
}

// q_{j+1} = w / |w|; T[j][j+1] = |w| (when j + 1 < m).  When |w| fell below 1e-10 of
// |A q_j| (an invariant subspace) a fresh Philox vector replaces w, T[j][j+1] = 0 and
// the slice is flagged for re-orthogonalisation (mode 0).  mode 1 normalises flagged
// slices only.
__global__ __launch_bounds__(256) void k_normalize(double2 *__restrict__ w, long n, double2 *__restrict__ qdst,
                                                   long qslice, const double *__restrict__ nrm,
                                                   const double *__restrict__ nb0, double *__restrict__ T, int m,
                                                   int j, int *bflag, int mode, uint32_t seed, double *beta_out)
{
    int t = blockIdx.y;
    long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (mode == 1 && !bflag[t]) return;
    double b = nrm[t];
    bool brk = (mode == 0) && !(b > 1e-10 * nb0[t]);
    if (brk) {
        if (row < n) {
            uint4 r = philox10(make_uint4((uint32_t)row, (uint32_t)t, (uint32_t)j, 0x42524bu), make_uint2(seed, 0x4C5A4E43u));
            w[t * n + row] = make_double2(r.x * 2.3283064365386963e-10 - 0.5, r.y * 2.3283064365386963e-10 - 0.5);
        }
        if (row == 0) {
            bflag[t] = 1;
            if (j + 1 < m) T[((long)t * m + j) * m + j + 1] = 0.0;
            if (beta_out) beta_out[t] = 0.0;
        }
        return;
    }
    if (row == 0) {
        if (mode == 0) {
            bflag[t] = 0;
            if (j + 1 < m) T[((long)t * m + j) * m + j + 1] = b;
            if (beta_out) beta_out[t] = b;
        }
    }
    if (row < n) qdst[t * qslice + row] = cscale(w[t * n + row], 1.0 / b);
}

__global__ __launch_bounds__(256) void k_random(double2 *__restrict__ q, long qslice, long n, uint32_t seed)
{
    int t = blockIdx.y;
    long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= n) return;
    uint4 r = philox10(make_uint4((uint32_t)row, (uint32_t)t, 0u, 0x53545254u), make_uint2(seed, 0x4C5A4E43u));
    q[t * qslice + row] = make_double2(r.x * 2.3283064365386963e-10 - 0.5, r.y * 2.3283064365386963e-10 - 0.5);
}

__global__ __launch_bounds__(256) void k_scale(double2 *__restrict__ q, long qslice, long n, const double *nrm)
{
    int t = blockIdx.y;
    long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (row < n) q[t * qslice + row] = cscale(q[t * qslice + row], 1.0 / nrm[t]);
}

// active block of T (rows/cols nlock..m-1), symmetrised from the upper triangle
__global__ void k_active(const double *__restrict__ T, double *__restrict__ M, int m, const int *__restrict__ nlock)
{
    int t = blockIdx.x;
    int l = nlock[t], na = m - l;
    for (int idx = threadIdx.x; idx < na * na; idx += blockDim.x) {
        int i = idx / na, k = idx % na;
        int gi = l + min(i, k), gk = l + max(i, k);
        M[((long)t * m + i) * m + k] = T[((long)t * m + gi) * m + gk];
    }
}

// parallel cyclic Jacobi on the na x na symmetric matrix M[t] (leading dimension m);
// Y[t] receives the eigenvectors (columns), theta[t] the eigenvalues sorted descending
// and perm[t] the column of Y that holds each sorted eigenvalue.
__global__ __launch_bounds__(256) void k_jacobi(double *__restrict__ Mall, double *__restrict__ Yall,
                                                double *__restrict__ theta, int *__restrict__ perm, int m,
                                                const int *__restrict__ nlock, int max_sweeps)
{
    int t = blockIdx.x;
    int na = m - nlock[t];
    double *A = Mall + (long)t * m * m;
    double *Y = Yall + (long)t * m * m;
    __shared__ double cs_c[96], cs_s[96];
    __shared__ int pp[96], qq[96];
    __shared__ double red[256];
    __shared__ int stop;
    for (int idx = threadIdx.x; idx < na * na; idx += blockDim.x) {
        int i = idx / na, k = idx % na;
        Y[(long)i * m + k] = (i == k) ? 1.0 : 0.0;
    }
    int nn = na + (na & 1);
    int half = nn / 2;
    __syncthreads();
    for (int sweep = 0; sweep < max_sweeps; sweep++) {
        // convergence: off-diagonal Frobenius norm against the whole
        double off = 0, tot = 0;
        for (int idx = threadIdx.x; idx < na * na; idx += blockDim.x) {
            int i = idx / na, k = idx % na;
            double v = A[(long)i * m + k];
            tot += v * v;
            if (i != k) off += v * v;
        }
        red[threadIdx.x] = off;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        double offs = red[0];
        __syncthreads();
        red[threadIdx.x] = tot;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        double tots = red[0];
        if (threadIdx.x == 0) stop = (offs <= 1e-30 * tots) ? 1 : 0;
        __syncthreads();
        if (stop) break;
        for (int round = 0; round < nn - 1; round++) {
            for (int k = threadIdx.x; k < half; k += blockDim.x) {
                int p, q;
                if (k == 0) {
                    p = nn - 1;
                    q = round;
                } else {
                    p = (round + k) % (nn - 1);
                    q = (round - k + nn - 1) % (nn - 1);
                }
                double c = 1, s = 0;
                if (p < na && q < na) {
                    double apq = A[(long)p * m + q];
                    if (fabs(apq) > 1e-300) {
                        double tau = (A[(long)q * m + q] - A[(long)p * m + p]) / (2 * apq);
                        double tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1 + tau * tau));
                        c = 1 / sqrt(1 + tt * tt);
                        s = tt * c;
                    }
                }
                pp[k] = p;
                qq[k] = q;
                cs_c[k] = c;
                cs_s[k] = s;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int idx = threadIdx.x; idx < half * na; idx += blockDim.x) {
                int k = idx / na, col = idx % na;
                int p = pp[k], q = qq[k];
                if (p >= na || q >= na) continue;
                double c = cs_c[k], s = cs_s[k];
                double a = A[(long)p * m + col], b = A[(long)q * m + col];
                A[(long)p * m + col] = c * a - s * b;
                A[(long)q * m + col] = s * a + c * b;
            }
            __syncthreads();
            // columns: A <- A J, Y <- Y J
            for (int idx = threadIdx.x; idx < half * na; idx += blockDim.x) {
                int k = idx / na, row = idx % na;
                int p = pp[k], q = qq[k];
                if (p >= na || q >= na) continue;
                double c = cs_c[k], s = cs_s[k];
                double a = A[(long)row * m + p], b = A[(long)row * m + q];
                A[(long)row * m + p] = c * a - s * b;
                A[(long)row * m + q] = s * a + c * b;
                a = Y[(long)row * m + p];
                b = Y[(long)row * m + q];
                Y[(long)row * m + p] = c * a - s * b;
                Y[(long)row * m + q] = s * a + c * b;
            }
            __syncthreads();
        }
    }
    // sort descending (selection of ranks: rank of i = #{k: d_k > d_i or (== and k < i)})
    for (int i = threadIdx.x; i < na; i += blockDim.x) {
        double di = A[(long)i * m + i];
        int rank = 0;
        for (int k = 0; k < na; k++) {
            double dk = A[(long)k * m + k];
            rank += (dk > di) || (dk == di && k < i);
        }
        theta[(long)t * m + rank] = di;
        perm[(long)t * m + rank] = i;
    }
}

// ylast[t][i] = Y[t][na-1][perm[t][i]]
__global__ void k_ylast(const double *__restrict__ Y, const int *__restrict__ perm, const int *__restrict__ nlock,
                        int m, double *__restrict__ ylast)
{
    int t = blockIdx.x;
    int na = m - nlock[t];
    for (int i = threadIdx.x; i < na; i += blockDim.x)
        ylast[(long)t * m + i] = Y[((long)t * m + (na - 1)) * m + perm[(long)t * m + i]];
}

// Qtmp[t][c] = sum_{a < na} Q[t][nlock + a] Y[t][a][ycol[t][c]], c < ncols[t]
constexpr int ROT_C = 16;
__global__ __launch_bounds__(256) void k_rotate(const double2 *__restrict__ Q, long qslice, long n,
                                                const double *__restrict__ Y, const int *__restrict__ ycol,
                                                const int *__restrict__ nlock, const int *__restrict__ ncols, int m,
                                                double2 *__restrict__ Qt, long tslice)
{
    int t = blockIdx.z;
    int c0 = blockIdx.y * ROT_C;
    int nc = min(ROT_C, ncols[t] - c0);
    if (nc <= 0) return;
    int l = nlock[t], na = m - l;
    __shared__ double yc[160][ROT_C];
    for (int idx = threadIdx.x; idx < na * ROT_C; idx += blockDim.x) {
        int a = idx / ROT_C, cc = idx % ROT_C;
        yc[a][cc] = cc < nc ? Y[((long)t * m + a) * m + ycol[(long)t * m + c0 + cc]] : 0.0;
    }
    __syncthreads();
    long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= n) return;
    double2 acc[ROT_C];
#pragma unroll
    for (int cc = 0; cc < ROT_C; cc++) acc[cc] = make_double2(0, 0);
    const double2 *q = Q + t * qslice + (long)l * n + row;
    for (int a = 0; a < na; a++) {
        double2 v = q[(long)a * n];
#pragma unroll
        for (int cc = 0; cc < ROT_C; cc++) {
            acc[cc].x += v.x * yc[a][cc];
            acc[cc].y += v.y * yc[a][cc];
        }
    }
    for (int cc = 0; cc < nc; cc++) Qt[t * tslice + (long)(c0 + cc) * n + row] = acc[cc];
}

// Q[t][nlock_old + c] = Qtmp[t][c] for c < ncols[t];  Q[t][rtot] = Q[t][m] (residual)
__global__ __launch_bounds__(256) void k_copyback(double2 *__restrict__ Q, long qslice, long n,
                                                  const double2 *__restrict__ Qt, long tslice,
                                                  const int *__restrict__ nlock_old, const int *__restrict__ ncols,
                                                  int m, int rtot)
{
    int t = blockIdx.y;
    long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= n) return;
    int l = nlock_old[t];
    for (int c = 0; c < ncols[t]; c++) Q[t * qslice + (long)(l + c) * n + row] = Qt[t * tslice + (long)c * n + row];
    Q[t * qslice + (long)rtot * n + row] = Q[t * qslice + (long)m * n + row];
}

// T[t] = 0 except T[p][p] = diag[t][p] for p in [lo[t], hi)
__global__ void k_set_T(double *__restrict__ T, const double *__restrict__ diag, const int *__restrict__ lo, int hi,
                        int m)
{
    int t = blockIdx.x;
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        int i = idx / m, k = idx % m;
        double v = 0;
        if (i == k && i >= lo[t] && i < hi) v = diag[(long)t * m + i];
        T[(long)t * m * m + idx] = v;
    }
}

// per-slice <a_t, b_t> partials (a, b with their own slice strides)
__global__ __launch_bounds__(256) void k_dot_slices(const double2 *__restrict__ a, long as, const double2 *__restrict__ b,
                                                    long bs, long n, double *__restrict__ part)
{
    int t = blockIdx.y;
    __shared__ double r0[256], r1[256];
    long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double re = 0, im = 0;
    if (row < n) {
        double2 u = a[t * as + row], v = b[t * bs + row];
        re = u.x * v.x + u.y * v.y;
        im = u.x * v.y - u.y * v.x;
    }
    r0[threadIdx.x] = re;
    r1[threadIdx.x] = im;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            r0[threadIdx.x] += r0[threadIdx.x + s];
            r1[threadIdx.x] += r1[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[((long)t * gridDim.x + blockIdx.x) * 2] = r0[0];
        part[((long)t * gridDim.x + blockIdx.x) * 2 + 1] = r1[0];
    }
}

// y = y + lam_t q (per slice), partial |y|^2
__global__ __launch_bounds__(256) void k_resid_slices(double2 *__restrict__ y, long n, const double2 *__restrict__ q,
                                                      long qs, const double *__restrict__ lam, double *__restrict__ part)
{
    int t = blockIdx.y;
    __shared__ double red[256];
    long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0;
    if (row < n) {
        double2 v = cadd(y[t * n + row], cscale(q[t * qs + row], lam[t]));
        acc = cnorm2(v);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(long)t * gridDim.x + blockIdx.x] = red[0];
}

// evecs[t][p] = phase * Q[t][src[t][p]] with the phase convention; one block per (p, t)
__global__ __launch_bounds__(256) void k_phase_out(const double2 *__restrict__ Q, long qslice, long n,
                                                   const int *__restrict__ src, int nv, double2 *__restrict__ out)
{
    int p = blockIdx.x, t = blockIdx.y;
    const double2 *v = Q + t * qslice + (long)src[t * nv + p] * n;
    __shared__ double red[256];
    __shared__ long ired[256];
    double mx = 0;
    for (long r = threadIdx.x; r < n; r += blockDim.x) mx = fmax(mx, cnorm2(v[r]));
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    double thr = 0.01 * red[0];  // |v_i| >= 0.1 max|v|  <=>  |v_i|^2 >= 0.01 max|v|^2
    long first = n;
    for (long r = threadIdx.x; r < n; r += blockDim.x)
        if (cnorm2(v[r]) >= thr) {
            first = r;
            break;
        }
    ired[threadIdx.x] = first;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) ired[threadIdx.x] = min(ired[threadIdx.x], ired[threadIdx.x + s]);
        __syncthreads();
    }
    double2 vi = v[ired[0]];
    double a = sqrt(cnorm2(vi));
    double2 ph = make_double2(vi.x / a, -vi.y / a);
    double2 *o = out + ((long)t * nv + p) * n;
    for (long r = threadIdx.x; r < n; r += blockDim.x) {
        double2 z = cmul(v[r], ph);
        if (r == ired[0]) z = make_double2(a, 0.0);
        o[r] = z;
    }
}

// w[t] = v[t * vs + off ...]
__global__ __launch_bounds__(256) void k_gather(const double2 *__restrict__ v, long vs, long off, long n,
                                                double2 *__restrict__ w)
{
    int t = blockIdx.y;
    long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (row < n) w[t * n + row] = v[t * vs + off + row];
}

struct Bufs {
    double2 *Q, *Qt, *w, *w0, *w1, *coef, *part;
    double *T, *M, *Y, *theta, *ylast, *diag, *nb, *nrm, *npart, *beta, *lam, *dpart;
    int *flags, *bflag, *nlock, *nlock_old, *ncols, *ycol, *perm, *src;
};

}  // namespace

// scratch of laph_eigvecs (the buffers below, in the same order)
size_t eig_scratch_bytes(const Geom &g, int m, int nv)
{
    const size_t nt = g.nt, n = 3 * g.V3, V = g.V;
    const size_t nchunk = (n + GS_CH - 1) / GS_CH, rb = (n + 255) / 256, ps = m + 1;
    size_t s = 0;
    for (size_t b : {V * 36 * 16, V * 36 * 16 /* stout.tmp */, 27 * V * 16, nt * (m + 1) * n * 16, nt * m * n * 16,
                     nt * n * 16, nt * n * 16, nt * n * 16, nt * ps * 16, nt * nchunk * ps * 16, nt * m * m * 8,
                     nt * m * m * 8, nt * m * m * 8, nt * m * 8, nt * m * 8, nt * m * 8, nt * 8, nt * 8, nt * 8,
                     nt * rb * 8, nt * 8, nt * 8, nt * rb * 16, nt * 4, nt * 4, nt * 4, nt * 4, nt * 4, nt * m * 4,
                     nt * m * 4, nt * (size_t)nv * 4})
        s += ws_align(b);
    return s;
}

extern "C" int laph_eigvecs(laph_ctx_t c, const double *U, const laph_stout *stout, const laph_lanczos *lz, int nv,
                            double *evals, double *evecs, laph_eig_stats *stats)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(U && stout && lz && evals && evecs && nv > 0, LAPH_EINVAL, "bad arguments");
    const int nt = c->g.nt;
    const long n = 3 * c->g.V3;
    const int m = lz->krylov_dim;
    LAPH_CHECK(m <= 160 && m > nv + 12 && m <= n, LAPH_EINVAL, "krylov_dim must satisfy nv + 12 < m <= min(160, 3 Ns^3)");
    LAPH_CHECK(lz->cheb_order >= 1 && lz->lambda_L > lz->lambda_C && lz->tol > 0 && lz->max_restarts >= 0,
               LAPH_EINVAL, "bad Lanczos parameters");
    const int rtot = std::min(nv + (m - nv) / 2, m - 12);
    hipStream_t st = c->stream;

    // smeared links (SoA) for the Laplacian
    double *Us = (double *)ctx_named(c, "eig.Us", (size_t)c->g.V * 36 * 16);
    stout_smear_device(c, U, stout->rho, stout->nsteps, Us);
    double2 *us = (double2 *)ctx_named(c, "lap.us", (size_t)27 * c->g.V * 16);
    smeared_links_to_soa(c, Us, us);

    const long qslice = (long)(m + 1) * n;
    const int nchunk = (int)((n + GS_CH - 1) / GS_CH);
    const int pstride = m + 1;
    const unsigned rb = nblocks_for(n, 256);
    Bufs b;
    b.Q = (double2 *)ctx_named(c, "eig.Q", (size_t)nt * qslice * 16);
    b.Qt = (double2 *)ctx_named(c, "eig.Qt", (size_t)nt * m * n * 16);
    b.w = (double2 *)ctx_named(c, "eig.w", (size_t)nt * n * 16);
    b.w0 = (double2 *)ctx_named(c, "eig.w0", (size_t)nt * n * 16);
    b.w1 = (double2 *)ctx_named(c, "eig.w1", (size_t)nt * n * 16);
    b.coef = (double2 *)ctx_named(c, "eig.coef", (size_t)nt * pstride * 16);
    b.part = (double2 *)ctx_named(c, "eig.part", (size_t)nt * nchunk * pstride * 16);
    b.T = (double *)ctx_named(c, "eig.T", (size_t)nt * m * m * 8);
    b.M = (double *)ctx_named(c, "eig.M", (size_t)nt * m * m * 8);
    b.Y = (double *)ctx_named(c, "eig.Y", (size_t)nt * m * m * 8);
    b.theta = (double *)ctx_named(c, "eig.theta", (size_t)nt * m * 8);
    b.ylast = (double *)ctx_named(c, "eig.ylast", (size_t)nt * m * 8);
    b.diag = (double *)ctx_named(c, "eig.diag", (size_t)nt * m * 8);
    b.nb = (double *)ctx_named(c, "eig.nb", (size_t)nt * 8);
    b.nrm = (double *)ctx_named(c, "eig.nrm", (size_t)nt * 8);
    double *nb0 = (double *)ctx_named(c, "eig.nb0", (size_t)nt * 8);
    b.npart = (double *)ctx_named(c, "eig.npart", (size_t)nt * rb * 8);
    b.beta = (double *)ctx_named(c, "eig.beta", (size_t)nt * 8);
    b.lam = (double *)ctx_named(c, "eig.lam", (size_t)nt * 8);
    b.dpart = (double *)ctx_named(c, "eig.dpart", (size_t)nt * rb * 16);
    b.flags = (int *)ctx_named(c, "eig.flags", (size_t)nt * 4);
    b.bflag = (int *)ctx_named(c, "eig.bflag", (size_t)nt * 4);
    b.nlock = (int *)ctx_named(c, "eig.nlock", (size_t)nt * 4);
    b.nlock_old = (int *)ctx_named(c, "eig.nlock_old", (size_t)nt * 4);
    b.ncols = (int *)ctx_named(c, "eig.ncols", (size_t)nt * 4);
    b.ycol = (int *)ctx_named(c, "eig.ycol", (size_t)nt * m * 4);
    b.perm = (int *)ctx_named(c, "eig.perm", (size_t)nt * m * 4);
    b.src = (int *)ctx_named(c, "eig.src", (size_t)nt * nv * 4);

    std::vector<int> h_nlock(nt, 0), h_ncols(nt, 0), h_ycol((size_t)nt * m, 0), h_src((size_t)nt * nv);
    std::vector<double> h_theta((size_t)nt * m), h_ylast((size_t)nt * m), h_beta(nt), h_diag((size_t)nt * m, 0.0);
    std::vector<int> h_perm((size_t)nt * m);
    std::vector<double> Anorm(nt, 0.0);
    LAPH_HIP(hipMemcpyAsync(b.nlock, h_nlock.data(), nt * 4, hipMemcpyHostToDevice, st));
    LAPH_HIP(hipMemsetAsync(b.T, 0, (size_t)nt * m * m * 8, st));
    LAPH_HIP(hipMemsetAsync(b.bflag, 0, (size_t)nt * 4, st));

    dim3 g2(rb, nt);
    // start vector: Philox draws, normalised
    hipLaunchKernelGGL(k_random, g2, dim3(256), 0, st, b.Q, qslice, n, lz->seed);
    hipLaunchKernelGGL(k_norm_slices, g2, dim3(256), 0, st, (const double2 *)b.Q, qslice, n, b.npart);
    hipLaunchKernelGGL(k_norm_fin, dim3(nblocks_for(nt, 64)), dim3(64), 0, st, (const double *)b.npart, (int)rb, nt,
                       b.nb, b.nrm, (int *)nullptr, 0, 0);
    hipLaunchKernelGGL(k_scale, g2, dim3(256), 0, st, b.Q, qslice, n, (const double *)b.nrm);
    LAPH_HIP(hipGetLastError());

    auto gs_pass = [&](int cnt, int j, const int *flags, int accumulate, int pass, bool last) {
        hipLaunchKernelGGL(k_gs_dots, dim3(nchunk, nt), dim3(256), 0, st, (const double2 *)b.Q, qslice, n,
                           (const double2 *)b.w, cnt, b.part, nchunk, pstride, flags);
        hipLaunchKernelGGL(k_gs_fin, dim3(nt), dim3(256), 0, st, (const double2 *)b.part, nchunk, pstride, cnt, b.coef,
                           b.T, m, j, (const int *)b.nlock, flags, accumulate);
        hipLaunchKernelGGL(k_gs_update, g2, dim3(256), 0, st, (const double2 *)b.Q, qslice, n, b.w, cnt,
                           (const double2 *)b.coef, pstride, b.npart, flags);
        hipLaunchKernelGGL(k_norm_fin, dim3(nblocks_for(nt, 64)), dim3(64), 0, st, (const double *)b.npart, (int)rb,
                           nt, b.nb, b.nrm, b.flags, 1, last ? 1 : 0);
        LAPH_HIP(hipGetLastError());
        (void)pass;
    };

    int j0 = 0, restarts = 0, matvecs = 0;
    std::vector<int> last_lold(nt, 0);
    bool converged = false;
    for (;; restarts++) {
        for (int j = j0; j < m; j++) {
            // w = A q_j
            cheb_apply(c, us, b.Q + (long)j * n, qslice, b.w, n, b.w0, b.w1, n, lz->lambda_L, lz->lambda_C,
                       lz->cheb_order, nullptr);
            matvecs++;
            hipLaunchKernelGGL(k_norm_slices, g2, dim3(256), 0, st, (const double2 *)b.w, n, n, b.npart);
            hipLaunchKernelGGL(k_norm_fin, dim3(nblocks_for(nt, 64)), dim3(64), 0, st, (const double *)b.npart,
                               (int)rb, nt, nb0, b.nrm, (int *)nullptr, 0, 0);
            LAPH_HIP(hipMemcpyAsync(b.nb, nb0, nt * 8, hipMemcpyDeviceToDevice, st));
            // first pass on every slice (sets flags), then up to four flagged repeats
            LAPH_HIP(hipMemsetAsync(b.flags, 0xff, nt * 4, st));  // all set: first pass everywhere
            gs_pass(j + 1, j, nullptr, 0, 0, false);
            for (int pass = 1; pass <= 4; pass++) gs_pass(j + 1, j, b.flags, 1, pass, pass == 4);
            // normalise into q_{j+1} (or the residual slot m)
            hipLaunchKernelGGL(k_normalize, g2, dim3(256), 0, st, b.w, n, b.Q + (long)(j + 1) * n, qslice,
                               (const double *)b.nrm, (const double *)nb0, b.T, m, j, b.bflag, 0,
                               lz->seed + 7919u * (uint32_t)restarts + 104729u * (uint32_t)j,
                               j == m - 1 ? b.beta : (double *)nullptr);
            // invariant-subspace replacement: orthogonalise the fresh vector twice, normalise
            for (int pass = 0; pass < 2; pass++) {
                hipLaunchKernelGGL(k_gs_dots, dim3(nchunk, nt), dim3(256), 0, st, (const double2 *)b.Q, qslice, n,
                                   (const double2 *)b.w, j + 1, b.part, nchunk, pstride, (const int *)b.bflag);
                hipLaunchKernelGGL(k_gs_fin, dim3(nt), dim3(256), 0, st, (const double2 *)b.part, nchunk, pstride,
                                   j + 1, b.coef, b.T, m, -1, (const int *)b.nlock, (const int *)b.bflag, 0);
                hipLaunchKernelGGL(k_gs_update, g2, dim3(256), 0, st, (const double2 *)b.Q, qslice, n, b.w, j + 1,
                                   (const double2 *)b.coef, pstride, b.npart, (const int *)b.bflag);
            }
            hipLaunchKernelGGL(k_norm_fin, dim3(nblocks_for(nt, 64)), dim3(64), 0, st, (const double *)b.npart,
                               (int)rb, nt, b.lam, b.lam, (int *)nullptr, 0, 0);
            hipLaunchKernelGGL(k_normalize, g2, dim3(256), 0, st, b.w, n, b.Q + (long)(j + 1) * n, qslice,
                               (const double *)b.lam, (const double *)nb0, b.T, m, j, b.bflag, 1, 0u,
                               (double *)nullptr);
            LAPH_HIP(hipGetLastError());
        }
        // Rayleigh-Ritz on the active block
        hipLaunchKernelGGL(k_active, dim3(nt), dim3(256), 0, st, (const double *)b.T, b.M, m, (const int *)b.nlock);
        hipLaunchKernelGGL(k_jacobi, dim3(nt), dim3(256), 0, st, b.M, b.Y, b.theta, b.perm, m, (const int *)b.nlock, 40);
        hipLaunchKernelGGL(k_ylast, dim3(nt), dim3(256), 0, st, (const double *)b.Y, (const int *)b.perm,
                           (const int *)b.nlock, m, b.ylast);
        LAPH_HIP(hipGetLastError());
        LAPH_HIP(hipMemcpyAsync(h_theta.data(), b.theta, h_theta.size() * 8, hipMemcpyDeviceToHost, st));
        LAPH_HIP(hipMemcpyAsync(h_ylast.data(), b.ylast, h_ylast.size() * 8, hipMemcpyDeviceToHost, st));
        LAPH_HIP(hipMemcpyAsync(h_perm.data(), b.perm, h_perm.size() * 4, hipMemcpyDeviceToHost, st));
        LAPH_HIP(hipMemcpyAsync(h_beta.data(), b.beta, nt * 8, hipMemcpyDeviceToHost, st));
        LAPH_HIP(hipStreamSynchronize(st));
        // lock / keep decisions per slice
        std::vector<int> nlock_new(nt);
        last_lold = h_nlock;
        bool all_done = true;
        for (int t = 0; t < nt; t++) {
            int l = h_nlock[t], na = m - l;
            const double *th = &h_theta[(size_t)t * m];
            const double *yl = &h_ylast[(size_t)t * m];
            for (int i = 0; i < na; i++) Anorm[t] = std::max(Anorm[t], std::fabs(th[i]));
            int want = nv - l;
            std::vector<int> lock, keep;
            std::vector<char> used(na, 0);
            for (int i = 0; i < want && i < na; i++) {
                double res = std::fabs(h_beta[t] * yl[i]);
                if (res < lz->tol * Anorm[t]) {
                    lock.push_back(i);
                    used[i] = 1;
                }
            }
            int ln = l + (int)lock.size();
            int nkeep = rtot - ln;
            for (int i = 0; i < na && (int)keep.size() < nkeep; i++)
                if (!used[i]) keep.push_back(i);
            h_ncols[t] = (int)(lock.size() + keep.size());
            int cc = 0;
            for (int i : lock) h_ycol[(size_t)t * m + cc++] = h_perm[(size_t)t * m + i];
            for (int i : keep) h_ycol[(size_t)t * m + cc++] = h_perm[(size_t)t * m + i];
            for (int k = 0; k < (int)keep.size(); k++) h_diag[(size_t)t * m + ln + k] = th[keep[k]];
            nlock_new[t] = ln;
            if (ln < nv) all_done = false;
        }
        bool stop = all_done || restarts >= lz->max_restarts;
        converged = all_done;
        // rotate the active block onto the selected Ritz vectors
        LAPH_HIP(hipMemcpyAsync(b.nlock_old, h_nlock.data(), nt * 4, hipMemcpyHostToDevice, st));
        LAPH_HIP(hipMemcpyAsync(b.ncols, h_ncols.data(), nt * 4, hipMemcpyHostToDevice, st));
        LAPH_HIP(hipMemcpyAsync(b.ycol, h_ycol.data(), h_ycol.size() * 4, hipMemcpyHostToDevice, st));
        int maxc = *std::max_element(h_ncols.begin(), h_ncols.end());
        hipLaunchKernelGGL(k_rotate, dim3(rb, (maxc + ROT_C - 1) / ROT_C, nt), dim3(256), 0, st, (const double2 *)b.Q,
                           qslice, n, (const double *)b.Y, (const int *)b.ycol, (const int *)b.nlock_old,
                           (const int *)b.ncols, m, b.Qt, (long)m * n);
        hipLaunchKernelGGL(k_copyback, g2, dim3(256), 0, st, b.Q, qslice, n, (const double2 *)b.Qt, (long)m * n,
                           (const int *)b.nlock_old, (const int *)b.ncols, m, rtot);
        LAPH_HIP(hipGetLastError());
        h_nlock = nlock_new;
        LAPH_HIP(hipMemcpyAsync(b.nlock, h_nlock.data(), nt * 4, hipMemcpyHostToDevice, st));
        if (stop) break;
        LAPH_HIP(hipMemcpyAsync(b.diag, h_diag.data(), h_diag.size() * 8, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_set_T, dim3(nt), dim3(256), 0, st, b.T, (const double *)b.diag, (const int *)b.nlock,
                           rtot, m);
        LAPH_HIP(hipGetLastError());
        j0 = rtot;
    }

    // Rayleigh quotients on -Lap and residuals for the first nv basis vectors
    std::vector<double> lam((size_t)nt * nv), res((size_t)nt * nv);
    std::vector<double> hp((size_t)nt * rb * 2);
    for (int p = 0; p < nv; p++) {
        const double2 *q = b.Q + (long)p * n;
        lap_fused(c, us, q, qslice, nullptr, 0, b.w, n, 1.0, 0.0, 0.0, nullptr);
        hipLaunchKernelGGL(k_dot_slices, g2, dim3(256), 0, st, q, qslice, (const double2 *)b.w, n, n, b.dpart);
        LAPH_HIP(hipMemcpyAsync(hp.data(), b.dpart, (size_t)nt * rb * 16, hipMemcpyDeviceToHost, st));
        LAPH_HIP(hipStreamSynchronize(st));
        std::vector<double> lt(nt);
        for (int t = 0; t < nt; t++) {
            double s = 0;
            for (unsigned k = 0; k < rb; k++) s += hp[((size_t)t * rb + k) * 2];
            lt[t] = -s;  // <q, Lap q> = -lambda
            lam[(size_t)t * nv + p] = -s;
        }
        LAPH_HIP(hipMemcpyAsync(b.lam, lt.data(), nt * 8, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_resid_slices, g2, dim3(256), 0, st, b.w, n, q, qslice, (const double *)b.lam, b.npart);
        LAPH_HIP(hipMemcpyAsync(hp.data(), b.npart, (size_t)nt * rb * 8, hipMemcpyDeviceToHost, st));
        LAPH_HIP(hipStreamSynchronize(st));
        for (int t = 0; t < nt; t++) {
            double s = 0;
            for (unsigned k = 0; k < rb; k++) s += hp[(size_t)t * rb + k];
            res[(size_t)t * nv + p] = std::sqrt(s);
        }
    }
    // ascending order per slice, phase convention, canonical output
    double maxres = 0;
    for (int t = 0; t < nt; t++) {
        std::vector<int> idx(nv);
        std::iota(idx.begin(), idx.end(), 0);
        std::stable_sort(idx.begin(), idx.end(),
                         [&](int a, int bb) { return lam[(size_t)t * nv + a] < lam[(size_t)t * nv + bb]; });
        for (int p = 0; p < nv; p++) {
            h_src[(size_t)t * nv + p] = idx[p];
            evals[(size_t)t * nv + p] = lam[(size_t)t * nv + idx[p]];
            maxres = std::max(maxres, res[(size_t)t * nv + idx[p]]);
        }
    }
    LAPH_HIP(hipMemcpyAsync(b.src, h_src.data(), h_src.size() * 4, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_phase_out, dim3(nv, nt), dim3(256), 0, st, (const double2 *)b.Q, qslice, n,
                       (const int *)b.src, nv, (double2 *)evecs);
    LAPH_HIP(hipGetLastError());
    if (stats) {
        stats->restarts = restarts;
        stats->matvecs = matvecs;
        stats->max_residual = maxres;
        // orthonormality of the output: max |<v_a, v_p> - delta_ap| over slices
        double mo = 0;
        std::vector<double2> hc((size_t)nt * pstride);
        for (int p = 0; p < nv; p++) {
            hipLaunchKernelGGL(k_gather, g2, dim3(256), 0, st, (const double2 *)evecs, (long)nv * n, (long)p * n, n, b.w);
            hipLaunchKernelGGL(k_gs_dots, dim3(nchunk, nt), dim3(256), 0, st, (const double2 *)evecs, (long)nv * n, n,
                               (const double2 *)b.w, nv, b.part, nchunk, pstride, (const int *)nullptr);
            hipLaunchKernelGGL(k_gs_fin, dim3(nt), dim3(256), 0, st, (const double2 *)b.part, nchunk, pstride, nv,
                               b.coef, b.T, m, -1, (const int *)b.nlock, (const int *)nullptr, 0);
            LAPH_HIP(hipMemcpyAsync(hc.data(), b.coef, hc.size() * 16, hipMemcpyDeviceToHost, st));
            LAPH_HIP(hipStreamSynchronize(st));
            for (int t = 0; t < nt; t++)
                for (int a2 = 0; a2 < nv; a2++) {
                    double2 v = hc[(size_t)t * pstride + a2];
                    double d = std::sqrt((v.x - (a2 == p ? 1.0 : 0.0)) * (v.x - (a2 == p ? 1.0 : 0.0)) + v.y * v.y);
                    mo = std::max(mo, d);
                }
        }
        stats->max_orth = mo;
        // gap estimate: the first Ritz value of A below the wanted ones, mapped back to -Lap
        double gap = 1e300;
        double cc = 2.0 / (lz->lambda_L - lz->lambda_C);
        for (int t = 0; t < nt; t++) {
            double th = h_theta[(size_t)t * m + (nv - last_lold[t])];
            double lam_next = lz->lambda_C;
            if (th > 1.0) lam_next = lz->lambda_C - (std::cosh(std::acosh(th) / lz->cheb_order) - 1.0) / cc;
            gap = std::min(gap, lam_next - evals[(size_t)t * nv + nv - 1]);
        }
        stats->min_gap = gap;
    }
    LAPH_HIP(hipStreamSynchronize(st));
    if (!converged) laph_fail(LAPH_EEIG, "eigensolver: not all %d pairs converged in %d restarts", nv, restarts);
    LAPH_API_END(c)
}

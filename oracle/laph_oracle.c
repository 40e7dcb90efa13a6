/*
 * laph_oracle.c -- plain, slow, FP64 CPU oracle for the stochastic-LapH hot path
 * of Morningstar et al., "Improved stochastic estimation of quark propagation with
 * Laplacian Heaviside smearing in lattice QCD" (arXiv:1104.3870).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or calls
 * this file; only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no code, header, table or helper with the GPU path.
 *
 * Every routine is written as the obvious loop over sites, spins and colours, in
 * double complex, with no blocking, no fusion and no even-odd tricks.  Each function
 * names the passage of the paper it follows.  Where the paper is silent the frozen
 * conventions are used (gamma basis, clover normalisation, anisotropy weights, noise
 * generator), each stated at the routine that uses it.
 *
 * Index conventions (canonical layouts, identical to the C-ABI of the product):
 *   site   s = x + Ns*(y + Ns*(z + Ns*t))
 *   links  U[((s*4 + mu)*3 + a)*3 + b],   mu = 0,1,2 (space), 3 (time)
 *   spinor psi[(s*4 + alpha)*3 + c]
 *   colour field (one per site, Laplacian) v[s*3 + c]
 *   eigenvectors evecs[((t*Nv + n)*Ns^3 + xyz)*3 + c]
 *   noise rho[(t*4 + alpha)*Nv + n]
 *   coefficients coef[(t*4 + alpha)*Nv + n]
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------ geometry */

static long or_site(int ns, int x, int y, int z, int t)
{
    return x + (long)ns * (y + (long)ns * (z + (long)ns * t));
}

static void or_coords(int ns, long s, int c[4])
{
    c[0] = (int)(s % ns); s /= ns;
    c[1] = (int)(s % ns); s /= ns;
    c[2] = (int)(s % ns); s /= ns;
    c[3] = (int)s;
}

/* neighbour of site s one step (step = +1 or -1) along direction mu, periodic */
static long or_neighbor(int ns, int nt, long s, int mu, int step)
{
    int c[4];
    or_coords(ns, s, c);
    int L = (mu == 3) ? nt : ns;
    c[mu] = (c[mu] + step + L) % L;
    return or_site(ns, c[0], c[1], c[2], c[3]);
}

/* ------------------------------------------------------- 3x3 colour matrices */

static void m3_mul(const cplx *a, const cplx *b, cplx *out)
{
    cplx r[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cplx acc = 0;
            for (int k = 0; k < 3; k++) acc += a[i * 3 + k] * b[k * 3 + j];
            r[i * 3 + j] = acc;
        }
    memcpy(out, r, sizeof(r));
}

static void m3_dag(const cplx *a, cplx *out)
{
    cplx r[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) r[i * 3 + j] = conj(a[j * 3 + i]);
    memcpy(out, r, sizeof(r));
}

static const cplx *or_link(const cplx *U, long s, int mu) { return U + (s * 4 + mu) * 9; }

/* ------------------------------------------------------------- stout smearing
 * Sec. II: spatial links are stout smeared (Morningstar & Peardon, PRD 69, 054501),
 * with spatial staples only; temporal links are not smeared.  One step:
 *   C_k(x) = rho * sum_{j != k, j spatial} [ U_j(x) U_k(x+j) U_j(x+k)^dag
 *                                           + U_j(x-j)^dag U_k(x-j) U_j(x-j+k) ]
 *   Om = C_k U_k^dag,  Q = (i/2)(Om^dag - Om) - (i/6) Tr(Om^dag - Om)
 *   U_k'(x) = exp(iQ) U_k(x)
 * exp is evaluated by its Taylor series with scaling and squaring (not by the
 * Cayley-Hamilton closed form the GPU path uses).
 */
static void m3_exp(const cplx *X, cplx *out)
{
    double nrm = 0;
    for (int i = 0; i < 9; i++) nrm += creal(X[i] * conj(X[i]));
    nrm = sqrt(nrm);
    int sq = 0;
    while (nrm > 0.25) { nrm *= 0.5; sq++; }
    double sc = ldexp(1.0, -sq);
    cplx Y[9], term[9], acc[9];
    for (int i = 0; i < 9; i++) Y[i] = X[i] * sc;
    for (int i = 0; i < 9; i++) { acc[i] = (i % 4 == 0) ? 1.0 : 0.0; term[i] = acc[i]; }
    for (int n = 1; n <= 24; n++) {
        m3_mul(term, Y, term);
        for (int i = 0; i < 9; i++) { term[i] /= (double)n; acc[i] += term[i]; }
    }
    for (int k = 0; k < sq; k++) m3_mul(acc, acc, acc);
    memcpy(out, acc, sizeof(acc));
}

void or_stout_spatial(const cplx *Uin, cplx *Uout, int ns, int nt, double rho, int nsteps)
{
    long V = (long)ns * ns * ns * nt;
    cplx *cur = (cplx *)malloc(sizeof(cplx) * V * 36);
    cplx *nxt = (cplx *)malloc(sizeof(cplx) * V * 36);
    memcpy(cur, Uin, sizeof(cplx) * V * 36);
    for (int step = 0; step < nsteps; step++) {
        memcpy(nxt, cur, sizeof(cplx) * V * 36);
#pragma omp parallel for schedule(static)
        for (long s = 0; s < V; s++) {
            for (int k = 0; k < 3; k++) {
                cplx C[9] = {0}, t1[9], t2[9];
                for (int j = 0; j < 3; j++) {
                    if (j == k) continue;
                    long sj = or_neighbor(ns, nt, s, j, +1);
                    long sk = or_neighbor(ns, nt, s, k, +1);
                    /* upper staple U_j(x) U_k(x+j) U_j(x+k)^dag */
                    m3_mul(or_link(cur, s, j), or_link(cur, sj, k), t1);
                    m3_dag(or_link(cur, sk, j), t2);
                    m3_mul(t1, t2, t1);
                    for (int i = 0; i < 9; i++) C[i] += t1[i];
                    /* lower staple U_j(x-j)^dag U_k(x-j) U_j(x-j+k) */
                    long smj = or_neighbor(ns, nt, s, j, -1);
                    long smjk = or_neighbor(ns, nt, smj, k, +1);
                    m3_dag(or_link(cur, smj, j), t1);
                    m3_mul(t1, or_link(cur, smj, k), t1);
                    m3_mul(t1, or_link(cur, smjk, j), t1);
                    for (int i = 0; i < 9; i++) C[i] += t1[i];
                }
                for (int i = 0; i < 9; i++) C[i] *= rho;
                cplx Ud[9], Om[9], Omd[9], Q[9], X[9], E[9];
                m3_dag(or_link(cur, s, k), Ud);
                m3_mul(C, Ud, Om);
                m3_dag(Om, Omd);
                cplx tr = 0;
                for (int i = 0; i < 3; i++) tr += Omd[i * 4] - Om[i * 4];
                for (int i = 0; i < 9; i++) Q[i] = 0.5 * I * (Omd[i] - Om[i]);
                for (int i = 0; i < 3; i++) Q[i * 4] -= (I / 6.0) * tr;
                for (int i = 0; i < 9; i++) X[i] = I * Q[i];
                m3_exp(X, E);
                m3_mul(E, or_link(cur, s, k), nxt + (s * 4 + k) * 9);
            }
        }
        cplx *tmp = cur; cur = nxt; nxt = tmp;
    }
    memcpy(Uout, cur, sizeof(cplx) * V * 36);
    free(cur);
    free(nxt);
}

/* average spatial plaquette Re Tr / 3 (a diagnostic for the smearing pins) */
double or_plaquette_spatial(const cplx *U, int ns, int nt)
{
    long V = (long)ns * ns * ns * nt;
    double acc = 0;
    for (long s = 0; s < V; s++)
        for (int mu = 0; mu < 3; mu++)
            for (int nu = mu + 1; nu < 3; nu++) {
                cplx a[9], b[9];
                long smu = or_neighbor(ns, nt, s, mu, +1), snu = or_neighbor(ns, nt, s, nu, +1);
                m3_mul(or_link(U, s, mu), or_link(U, smu, nu), a);
                m3_dag(or_link(U, snu, mu), b);
                m3_mul(a, b, a);
                m3_dag(or_link(U, s, nu), b);
                m3_mul(a, b, a);
                acc += creal(a[0] + a[4] + a[8]) / 3.0;
            }
    return acc / (3.0 * V);
}

/* --------------------------------------------------- gauge-covariant Laplacian
 * Sec. II, Laplacian definition:
 *   (Lap v)(x) = sum_{k=1..3} [ U_k(x) v(x+k) + U_k(x-k)^dag v(x-k) - 2 v(x) ]
 * applied on every time slice (it is block diagonal in time).  Uses only the
 * spatial links of the (smeared) field.  v, out: [V][3].
 */
void or_laplacian(const cplx *U, const cplx *v, cplx *out, int ns, int nt)
{
    long V = (long)ns * ns * ns * nt;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        cplx acc[3];
        for (int a = 0; a < 3; a++) acc[a] = -6.0 * v[s * 3 + a];
        for (int k = 0; k < 3; k++) {
            long sp = or_neighbor(ns, nt, s, k, +1);
            long sm = or_neighbor(ns, nt, s, k, -1);
            const cplx *Uf = or_link(U, s, k);
            const cplx *Ub = or_link(U, sm, k);
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) {
                    acc[a] += Uf[a * 3 + b] * v[sp * 3 + b];
                    acc[a] += conj(Ub[b * 3 + a]) * v[sm * 3 + b];
                }
        }
        for (int a = 0; a < 3; a++) out[s * 3 + a] = acc[a];
    }
}

/* The same Laplacian restricted to one time slice t; v3, out3: [Ns^3][3]. */
void or_laplacian_slice(const cplx *U, const cplx *v3, cplx *out3, int ns, int nt, int t)
{
    long V3 = (long)ns * ns * ns;
#pragma omp parallel for schedule(static)
    for (long r = 0; r < V3; r++) {
        long s = r + V3 * t;
        cplx acc[3];
        for (int a = 0; a < 3; a++) acc[a] = -6.0 * v3[r * 3 + a];
        for (int k = 0; k < 3; k++) {
            long sp = or_neighbor(ns, nt, s, k, +1) - V3 * t;
            long sm = or_neighbor(ns, nt, s, k, -1) - V3 * t;
            const cplx *Uf = or_link(U, s, k);
            const cplx *Ub = or_link(U, sm + V3 * t, k);
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) {
                    acc[a] += Uf[a * 3 + b] * v3[sp * 3 + b];
                    acc[a] += conj(Ub[b * 3 + a]) * v3[sm * 3 + b];
                }
        }
        for (int a = 0; a < 3; a++) out3[r * 3 + a] = acc[a];
    }
}

/* ------------------------------------------------------ Chebyshev transform
 * Sec. IV (Chebyshev acceleration):  B = 1 + 2/(lamL - lamC) (Lap + lamC),
 * A = T_n(B) with T_0 = 1, T_1 = x, T_n = 2x T_{n-1} - T_{n-2}.
 * out = T_order(B) v on every time slice.
 */
void or_chebyshev(const cplx *U, const cplx *v, cplx *out, int ns, int nt,
                  double lamL, double lamC, int order)
{
    long n = (long)ns * ns * ns * nt * 3;
    double c = 2.0 / (lamL - lamC);
    cplx *tm2 = (cplx *)malloc(sizeof(cplx) * n);
    cplx *tm1 = (cplx *)malloc(sizeof(cplx) * n);
    cplx *lap = (cplx *)malloc(sizeof(cplx) * n);
    memcpy(tm2, v, sizeof(cplx) * n);                 /* T_0 v */
    if (order == 0) { memcpy(out, v, sizeof(cplx) * n); goto done; }
    or_laplacian(U, v, lap, ns, nt);
    for (long i = 0; i < n; i++) tm1[i] = v[i] + c * (lap[i] + lamC * v[i]); /* T_1 v = B v */
    for (int k = 2; k <= order; k++) {
        or_laplacian(U, tm1, lap, ns, nt);
        for (long i = 0; i < n; i++) {
            cplx Bt = tm1[i] + c * (lap[i] + lamC * tm1[i]);
            cplx tk = 2.0 * Bt - tm2[i];
            tm2[i] = tm1[i];
            tm1[i] = tk;
        }
    }
    memcpy(out, tm1, sizeof(cplx) * n);
done:
    free(tm2); free(tm1); free(lap);
}

/* ---------------------------------------------------------- Philox4x32-10
 * Counter-based generator of Salmon, Moraes, Dror and Shaw (SC'11), written from
 * its published definition: ten rounds of
 *   (c0,c1,c2,c3) -> (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0))
 * with the key bumped by the Weyl constants between rounds.
 */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* --------------------------------------------------------------- Z4 noise
 * Sec. II (noise in the LapH subspace) and Sec. IV (Z4 noise identified by a
 * 16-bit noise id s and a 16-bit configuration id k, combined into one 32-bit m).
 * Frozen reading: m = (k << 16) | s; element (t, alpha, n) takes word 0 of
 * Philox4x32-10 with counter (n, alpha, t, 0) and key (m, 0x4C415048), and the
 * value i^(word0 mod 4) in {1, i, -1, -i}.   rho: [Nt][4][Nv].
 */
void or_z4_noise(unsigned s, unsigned k, int nt, int nv, cplx *rho)
{
    const cplx z4[4] = {1.0, I, -1.0, -I};
    uint32_t key[2] = {((uint32_t)(k & 0xFFFFu) << 16) | (uint32_t)(s & 0xFFFFu), 0x4C415048u};
    for (int t = 0; t < nt; t++)
        for (int a = 0; a < 4; a++)
            for (int n = 0; n < nv; n++) {
                uint32_t ctr[4] = {(uint32_t)n, (uint32_t)a, (uint32_t)t, 0u}, w[4];
                or_philox4x32_10(ctr, key, w);
                rho[((long)t * 4 + a) * nv + n] = z4[w[0] & 3u];
            }
}

/* ---------------------------------------------------------------- dilution
 * Sec. II, table of the four dilution schemes.  type: 0 none ("1"), 1 full ("F"),
 * 2 block-J ("BJ"), 3 interlace-J ("IJ").  N is the dimension of the diluted index.
 */
int or_dilution_count(int type, int J, int N)
{
    switch (type) {
    case 0: return 1;
    case 1: return N;
    case 2: case 3: return J;
    }
    return -1;
}

int or_dilution_member(int type, int J, int N, int i, int b)
{
    switch (type) {
    case 0: return b == 0;
    case 1: return i == b;
    case 2: return (int)(((long)J * i) / N) == b;
    case 3: return (i % J) == b;
    }
    return 0;
}

/* ------------------------------------------------------------------- source
 * Sec. II (quark line in the LapH subspace) and Sec. IV: the right-hand side is
 * eta = V_s P^(b) rho with P^(b) = P^(bT) (x) P^(bS) (x) P^(bL).
 * scheme[6] = {typeT, JT, typeS, JS, typeL, JL}; b = (bT*nS + bS)*nL + bL where
 * nX is the number of projectors of that kind.
 *   eta(x,t,c,alpha) = sum_{n in L(bL)} V_{t,n}(x,c) rho(t,alpha,n)  for t in T(bT),
 *                      alpha in S(bS); zero elsewhere.
 */
int or_source(const cplx *evecs, const cplx *rho, int ns, int nt, int nv,
              const int scheme[6], long b, cplx *eta)
{
    long V3 = (long)ns * ns * ns;
    int nT = or_dilution_count(scheme[0], scheme[1], nt);
    int nS = or_dilution_count(scheme[2], scheme[3], 4);
    int nL = or_dilution_count(scheme[4], scheme[5], nv);
    if (b < 0 || b >= (long)nT * nS * nL) return -1;
    int bL = (int)(b % nL), bS = (int)((b / nL) % nS), bT = (int)(b / ((long)nL * nS));
    memset(eta, 0, sizeof(cplx) * V3 * nt * 12);
    for (int t = 0; t < nt; t++) {
        if (!or_dilution_member(scheme[0], scheme[1], nt, t, bT)) continue;
        for (int a = 0; a < 4; a++) {
            if (!or_dilution_member(scheme[2], scheme[3], 4, a, bS)) continue;
            for (int n = 0; n < nv; n++) {
                if (!or_dilution_member(scheme[4], scheme[5], nv, n, bL)) continue;
                cplx r = rho[((long)t * 4 + a) * nv + n];
                const cplx *vec = evecs + ((long)t * nv + n) * V3 * 3;
                for (long xyz = 0; xyz < V3; xyz++)
                    for (int c = 0; c < 3; c++)
                        eta[((xyz + V3 * t) * 4 + a) * 3 + c] += vec[xyz * 3 + c] * r;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------ sink projection
 * Sec. IV (quark propagation coefficients V_s^dag Omega^-1 V_s P^(b) rho):
 *   coef(t,alpha,n) = sum_{x,c} conj(V_{t,n}(x,c)) X(x,t,c,alpha).
 */
void or_sink_project(const cplx *evecs, const cplx *X, int ns, int nt, int nv, cplx *coef)
{
    long V3 = (long)ns * ns * ns;
#pragma omp parallel for collapse(2) schedule(static)
    for (int t = 0; t < nt; t++)
        for (int n = 0; n < nv; n++) {
            const cplx *vec = evecs + ((long)t * nv + n) * V3 * 3;
            for (int a = 0; a < 4; a++) {
                cplx acc = 0;
                for (long xyz = 0; xyz < V3; xyz++)
                    for (int c = 0; c < 3; c++)
                        acc += conj(vec[xyz * 3 + c]) * X[((xyz + V3 * t) * 4 + a) * 3 + c];
                coef[((long)t * 4 + a) * nv + n] = acc;
            }
        }
}

/* ---------------------------------------------------------- baryon function
 * Sec. III.A (Eq. baryonfunc) for three full-lattice spinor fields:
 *   B(t) = sum_{alpha,beta,gamma} c_{alpha beta gamma} sum_x exp(-i p.x)
 *          sum_{a,b,c} eps_abc f1(x,t,a,alpha) f2(x,t,b,beta) f3(x,t,c,gamma),
 * c a 4x4x4 spin tensor c[(alpha*4 + beta)*4 + gamma], p = 2 pi k / Ns.
 */
void or_baryon_function(const cplx *f1, const cplx *f2, const cplx *f3, int ns, int nt, const cplx *c64,
                        const int *k, cplx *out)
{
    static const int perm[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}, {0, 2, 1}, {2, 1, 0}, {1, 0, 2}};
    static const double sgn[6] = {1, 1, 1, -1, -1, -1};
    long V3 = (long)ns * ns * ns;
    const double tw = 2.0 * acos(-1.0) / ns;
    for (int t = 0; t < nt; t++) {
        cplx acc = 0;
        for (long xyz = 0; xyz < V3; xyz++) {
            int c[4];
            or_coords(ns, xyz, c);
            cplx e = cexp(-I * tw * (k[0] * c[0] + k[1] * c[1] + k[2] * c[2]));
            long s = xyz + V3 * t;
            for (int al = 0; al < 4; al++)
                for (int be = 0; be < 4; be++)
                    for (int ga = 0; ga < 4; ga++) {
                        cplx g = c64[(al * 4 + be) * 4 + ga];
                        if (g == 0) continue;
                        cplx sum = 0;
                        for (int q = 0; q < 6; q++)
                            sum += sgn[q] * f1[(s * 4 + al) * 3 + perm[q][0]] * f2[(s * 4 + be) * 3 + perm[q][1]] *
                                   f3[(s * 4 + ga) * 3 + perm[q][2]];
                        acc += g * e * sum;
                    }
        }
        out[t] = acc;
    }
}

/* ------------------------------------------------------ covariant displacement
 * Sec. II (quark lines D^(j) S Omega^-1 S D^(k)dag): a displacement of type j moves a field
 * by `len` links along spatial direction dir (0, 1, 2 = x, y, z) with sign +1 or -1, in a
 * gauge-covariant way:
 *   (D v)(x) = U_dir(x) U_dir(x+e) ... U_dir(x+(len-1)e) v(x+len e)                 (+)
 *   (D v)(x) = U_dir(x-e)^dag U_dir(x-2e)^dag ... U_dir(x-len e)^dag v(x-len e)       (-)
 * on colour fields v[s*3 + c] over the whole lattice (each time slice separately; the
 * links are the caller's, e.g. the stout-smeared ones of the LapH subspace).
 */
void or_displace(const cplx *U, int ns, int nt, int dir, int sign, int len, const cplx *v, cplx *out)
{
    long V = (long)ns * ns * ns * nt;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        /* walk to the far end, then apply the links back towards s */
        long far = s;
        for (int k = 0; k < len; k++) far = or_neighbor(ns, nt, far, dir, sign);
        cplx w[3] = {v[far * 3], v[far * 3 + 1], v[far * 3 + 2]};
        long cur = far;
        for (int k = 0; k < len; k++) {
            long prev = or_neighbor(ns, nt, cur, dir, -sign); /* one step back towards s */
            cplx L[9];
            if (sign > 0)
                memcpy(L, or_link(U, prev, dir), sizeof(L)); /* U_dir(prev) w(prev + e) */
            else
                m3_dag(or_link(U, cur, dir), L);             /* U_dir(cur)^dag w(cur), cur = prev - e */
            cplx r[3];
            for (int a = 0; a < 3; a++) r[a] = L[a * 3] * w[0] + L[a * 3 + 1] * w[1] + L[a * 3 + 2] * w[2];
            memcpy(w, r, sizeof(w));
            cur = prev;
        }
        memcpy(out + s * 3, w, sizeof(w));
    }
}

/* -------------------------------------------------------- momentum overlaps
 * The momentum projection of the meson function (Sec. III.B, Eq. mesonfunc) between two
 * sets of colour fields on every slice:
 *   O[t][n][m] = sum_{x in slice t} exp(-i p.x) sum_c conj(a_n(x,c)) b_m(x,c),
 * p = 2 pi k / Ns; a, b in the eigenvector layout [Nt][n][Ns^3][3].
 */
void or_mom_overlap(const cplx *a, const cplx *b, int ns, int nt, int na, int nb, const int *k, cplx *out)
{
    long V3 = (long)ns * ns * ns;
    const double tw = 2.0 * acos(-1.0) / ns;
#pragma omp parallel for collapse(2) schedule(static)
    for (int t = 0; t < nt; t++)
        for (int n = 0; n < na; n++)
            for (int m = 0; m < nb; m++) {
                const cplx *va = a + ((long)t * na + n) * V3 * 3;
                const cplx *vb = b + ((long)t * nb + m) * V3 * 3;
                cplx acc = 0;
                for (long xyz = 0; xyz < V3; xyz++) {
                    int c[4];
                    or_coords(ns, xyz, c);
                    cplx e = cexp(-I * tw * (k[0] * c[0] + k[1] * c[1] + k[2] * c[2]));
                    cplx sum = 0;
                    for (int cc = 0; cc < 3; cc++) sum += conj(va[xyz * 3 + cc]) * vb[xyz * 3 + cc];
                    acc += e * sum;
                }
                out[((long)t * na + n) * nb + m] = acc;
            }
}

/* ---------------------------------------------------------- meson function
 * Sec. III.B (Eq. mesonfunc): for two full-lattice spinor fields f1 (its complex
 * conjugate enters) and f2,
 *   M(t) = sum_{alpha,beta} c_{alpha beta} sum_x exp(-i p.(x + (d1 + d2)/2))
 *          sum_a conj(f1(x,t,a,alpha)) f2(x,t,a,beta),
 * c a 4x4 spin matrix (row-major), p = 2 pi k / Ns with k an integer triple, d1 and d2
 * the spatial displacement vectors of the two fields in lattice units.
 */
void or_meson_function(const cplx *f1, const cplx *f2, int ns, int nt, const cplx *c16, const int *k,
                       const int *d1, const int *d2, cplx *out)
{
    long V3 = (long)ns * ns * ns;
    const double tw = 2.0 * acos(-1.0) / ns;
    for (int t = 0; t < nt; t++) {
        cplx acc = 0;
        for (long xyz = 0; xyz < V3; xyz++) {
            int c[4];
            or_coords(ns, xyz, c);
            double ph = 0;
            for (int i = 0; i < 3; i++) ph += tw * k[i] * (c[i] + 0.5 * (d1[i] + d2[i]));
            cplx e = cexp(-I * ph);
            long s = xyz + V3 * t;
            for (int al = 0; al < 4; al++)
                for (int be = 0; be < 4; be++) {
                    cplx g = c16[al * 4 + be];
                    if (g == 0) continue;
                    cplx sum = 0;
                    for (int a = 0; a < 3; a++) sum += conj(f1[(s * 4 + al) * 3 + a]) * f2[(s * 4 + be) * 3 + a];
                    acc += g * e * sum;
                }
        }
        out[t] = acc;
    }
}

/* ----------------------------------------------------- Dirac gamma matrices
 * The paper does not print its Dirac matrix (it names an improved anisotropic
 * clover action and Omega = gamma_4 K).  Frozen reading: Hermitian Euclidean
 * chiral basis, gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_4 = [[0,1],[1,0]].
 * gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 is computed from these, not typed.
 */
static cplx or_gam[5][4][4];
static int or_gam_ready = 0;

static void or_gamma_init(void)
{
    if (or_gam_ready) return;
    memset(or_gam, 0, sizeof(or_gam));
    cplx sig[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    for (int k = 0; k < 3; k++)
        for (int i = 0; i < 2; i++)
            for (int j = 0; j < 2; j++) {
                or_gam[k][i][2 + j] = -I * sig[k][i][j];
                or_gam[k][2 + i][j] = I * sig[k][i][j];
            }
    for (int i = 0; i < 2; i++) { or_gam[3][i][2 + i] = 1; or_gam[3][2 + i][i] = 1; }
    cplx t1[4][4], t2[4][4];
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            cplx a = 0;
            for (int k = 0; k < 4; k++) a += or_gam[0][i][k] * or_gam[1][k][j];
            t1[i][j] = a;
        }
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            cplx a = 0;
            for (int k = 0; k < 4; k++) a += t1[i][k] * or_gam[2][k][j];
            t2[i][j] = a;
        }
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            cplx a = 0;
            for (int k = 0; k < 4; k++) a += t2[i][k] * or_gam[3][k][j];
            or_gam[4][i][j] = a;
        }
    or_gam_ready = 1;
}

/* copy of gamma_mu (mu = 0..3 for gamma_1..gamma_4, 4 for gamma_5) */
void or_gamma(int mu, cplx *out16)
{
    or_gamma_init();
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) out16[i * 4 + j] = or_gam[mu][i][j];
}

/* -------------------------------------------------------------- clover term
 * Frozen reading of the anisotropic clover term (the paper only names the action):
 *   A(x) = (m0 + 1 + 3/xi) - 1/2 [ c_t sum_k sigma_k4 F_k4 + c_s sum_{k<l} sigma_kl F_kl ]
 *   sigma_mn = (i/2)[gamma_m, gamma_n],  c_s = c_sw/xi,  c_t = c_sw (1 + 1/xi)/2,
 *   F_mn = traceless part of (Q_mn - Q_mn^dag)/(8i), Q_mn the sum of the four plaquette
 *   leaves in the (m,n) plane that touch x.
 * A: [V][12][12] with row index alpha*3 + a.
 */
static void or_field_strength(const cplx *U, int ns, int nt, long s, int mu, int nu, cplx *F)
{
    cplx Q[9] = {0}, a[9], b[9];
    long xp_mu = or_neighbor(ns, nt, s, mu, +1), xp_nu = or_neighbor(ns, nt, s, nu, +1);
    long xm_mu = or_neighbor(ns, nt, s, mu, -1), xm_nu = or_neighbor(ns, nt, s, nu, -1);
    long xm_mu_p_nu = or_neighbor(ns, nt, xm_mu, nu, +1);
    long xm_mu_m_nu = or_neighbor(ns, nt, xm_mu, nu, -1);
    long xm_nu_p_mu = or_neighbor(ns, nt, xm_nu, mu, +1);
    /* leaf 1: U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag */
    m3_mul(or_link(U, s, mu), or_link(U, xp_mu, nu), a);
    m3_dag(or_link(U, xp_nu, mu), b); m3_mul(a, b, a);
    m3_dag(or_link(U, s, nu), b); m3_mul(a, b, a);
    for (int i = 0; i < 9; i++) Q[i] += a[i];
    /* leaf 2: U_nu(x) U_mu(x-mu+nu)^dag U_nu(x-mu)^dag U_mu(x-mu) */
    m3_dag(or_link(U, xm_mu_p_nu, mu), b); m3_mul(or_link(U, s, nu), b, a);
    m3_dag(or_link(U, xm_mu, nu), b); m3_mul(a, b, a);
    m3_mul(a, or_link(U, xm_mu, mu), a);
    for (int i = 0; i < 9; i++) Q[i] += a[i];
    /* leaf 3: U_mu(x-mu)^dag U_nu(x-mu-nu)^dag U_mu(x-mu-nu) U_nu(x-nu) */
    m3_dag(or_link(U, xm_mu, mu), a);
    m3_dag(or_link(U, xm_mu_m_nu, nu), b); m3_mul(a, b, a);
    m3_mul(a, or_link(U, xm_mu_m_nu, mu), a);
    m3_mul(a, or_link(U, xm_nu, nu), a);
    for (int i = 0; i < 9; i++) Q[i] += a[i];
    /* leaf 4: U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^dag */
    m3_dag(or_link(U, xm_nu, nu), a);
    m3_mul(a, or_link(U, xm_nu, mu), a);
    m3_mul(a, or_link(U, xm_nu_p_mu, nu), a);
    m3_dag(or_link(U, s, mu), b); m3_mul(a, b, a);
    for (int i = 0; i < 9; i++) Q[i] += a[i];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) F[i * 3 + j] = (Q[i * 3 + j] - conj(Q[j * 3 + i])) / (8.0 * I);
    cplx tr = (F[0] + F[4] + F[8]) / 3.0;
    for (int i = 0; i < 3; i++) F[i * 4] -= tr;
}

void or_clover(const cplx *U, int ns, int nt, double m0, double xi, double csw, cplx *A)
{
    or_gamma_init();
    long V = (long)ns * ns * ns * nt;
    double cs = csw / xi, ct = csw * (1.0 + 1.0 / xi) / 2.0;
    double diag = m0 + 1.0 + 3.0 / xi;
    /* sigma_mn for mu < nu */
    cplx sigma[4][4][4][4];
    for (int m = 0; m < 4; m++)
        for (int n = 0; n < 4; n++)
            for (int i = 0; i < 4; i++)
                for (int j = 0; j < 4; j++) {
                    cplx c = 0;
                    for (int k = 0; k < 4; k++)
                        c += or_gam[m][i][k] * or_gam[n][k][j] - or_gam[n][i][k] * or_gam[m][k][j];
                    sigma[m][n][i][j] = 0.5 * I * c;
                }
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        cplx *As = A + s * 144;
        memset(As, 0, sizeof(cplx) * 144);
        for (int i = 0; i < 12; i++) As[i * 12 + i] = diag;
        for (int m = 0; m < 4; m++)
            for (int n = m + 1; n < 4; n++) {
                cplx F[9];
                or_field_strength(U, ns, nt, s, m, n, F);
                double coef = (n == 3) ? ct : cs;
                for (int al = 0; al < 4; al++)
                    for (int be = 0; be < 4; be++)
                        for (int a = 0; a < 3; a++)
                            for (int b = 0; b < 3; b++)
                                As[(al * 3 + a) * 12 + be * 3 + b] -=
                                    0.5 * coef * sigma[m][n][al][be] * F[a * 3 + b];
            }
    }
}

/* --------------------------------------------------------------- Dirac matrix
 * K = A + H with the frozen anisotropic Wilson hopping term
 *   (H psi)(x) = -1/2 sum_mu w_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                                 + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
 * w_4 = 1, w_k = 1/xi; fermions antiperiodic in time (bc_t = -1 multiplies every hop
 * that crosses the t = Nt-1 <-> 0 boundary), periodic in space.
 * dagger = 1 applies K^dag (A is Hermitian; the hop adjoint flips gamma_mu's sign).
 * Omega = gamma_4 K (Sec. II, quark line definition).
 */
void or_dirac(const cplx *U, const cplx *A, int ns, int nt, double xi, double bc_t,
              int dagger, const cplx *psi, cplx *out)
{
    or_gamma_init();
    long V = (long)ns * ns * ns * nt;
    double sgn = dagger ? -1.0 : 1.0;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        int c[4];
        or_coords(ns, s, c);
        cplx acc[12];
        const cplx *As = A + s * 144;
        for (int i = 0; i < 12; i++) {
            cplx v = 0;
            for (int j = 0; j < 12; j++) v += (dagger ? conj(As[j * 12 + i]) : As[i * 12 + j]) * psi[s * 12 + j];
            acc[i] = v;
        }
        for (int mu = 0; mu < 4; mu++) {
            double w = (mu == 3) ? 1.0 : 1.0 / xi;
            long sp = or_neighbor(ns, nt, s, mu, +1);
            long sm = or_neighbor(ns, nt, s, mu, -1);
            double bf = (mu == 3 && c[3] == nt - 1) ? bc_t : 1.0;
            double bb = (mu == 3 && c[3] == 0) ? bc_t : 1.0;
            const cplx *Uf = or_link(U, s, mu);
            const cplx *Ub = or_link(U, sm, mu);
            cplx uf[12], ub[12];
            for (int al = 0; al < 4; al++)
                for (int a = 0; a < 3; a++) {
                    cplx f = 0, g = 0;
                    for (int b = 0; b < 3; b++) {
                        f += Uf[a * 3 + b] * psi[sp * 12 + al * 3 + b];
                        g += conj(Ub[b * 3 + a]) * psi[sm * 12 + al * 3 + b];
                    }
                    uf[al * 3 + a] = f * bf;
                    ub[al * 3 + a] = g * bb;
                }
            for (int al = 0; al < 4; al++)
                for (int a = 0; a < 3; a++) {
                    cplx v = 0;
                    for (int be = 0; be < 4; be++) {
                        double id = (al == be) ? 1.0 : 0.0;
                        v += (id - sgn * or_gam[mu][al][be]) * uf[be * 3 + a];
                        v += (id + sgn * or_gam[mu][al][be]) * ub[be * 3 + a];
                    }
                    acc[al * 3 + a] += -0.5 * w * v;
                }
        }
        for (int i = 0; i < 12; i++) out[s * 12 + i] = acc[i];
    }
}

static void or_gamma4_apply(long V, const cplx *in, cplx *out)
{
    for (long s = 0; s < V; s++)
        for (int al = 0; al < 4; al++)
            for (int a = 0; a < 3; a++) {
                cplx v = 0;
                for (int be = 0; be < 4; be++) v += or_gam[3][al][be] * in[s * 12 + be * 3 + a];
                out[s * 12 + al * 3 + a] = v;
            }
}

/* Omega psi = gamma_4 K psi   (dagger = 1:  Omega^dag psi = K^dag gamma_4 psi) */
void or_omega(const cplx *U, const cplx *A, int ns, int nt, double xi, double bc_t,
              int dagger, const cplx *psi, cplx *out)
{
    or_gamma_init();
    long V = (long)ns * ns * ns * nt;
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * V * 12);
    if (!dagger) {
        or_dirac(U, A, ns, nt, xi, bc_t, 0, psi, tmp);
        or_gamma4_apply(V, tmp, out);
    } else {
        or_gamma4_apply(V, psi, tmp);
        or_dirac(U, A, ns, nt, xi, bc_t, 1, tmp, out);
    }
    free(tmp);
}

/* dense matrix of Omega (or K when omega == 0) by application to unit vectors;
 * Mt: [N][N] holding the TRANSPOSE (column j of the operator is row j of Mt),
 * N = 12 V.  Only for tiny lattices.  */
void or_dense_operator(const cplx *U, const cplx *A, int ns, int nt, double xi, double bc_t,
                       int omega, cplx *Mt)
{
    long V = (long)ns * ns * ns * nt, N = 12 * V;
    cplx *e = (cplx *)calloc(N, sizeof(cplx));
    cplx *col = (cplx *)malloc(sizeof(cplx) * N);
    for (long j = 0; j < N; j++) {
        e[j] = 1.0;
        if (omega) or_omega(U, A, ns, nt, xi, bc_t, 0, e, col);
        else or_dirac(U, A, ns, nt, xi, bc_t, 0, e, col);
        memcpy(Mt + j * N, col, sizeof(cplx) * N);
        e[j] = 0.0;
    }
    free(e);
    free(col);
}

/* ----------------------------------------------------------------- the solve
 * Sec. IV: Omega x = y is solved; the paper's fallback is conjugate gradient on
 * Omega^dag Omega x = Omega^dag y, which is what the oracle uses (no even-odd
 * preconditioning).  The iteration stops when the true residual |y - Omega x|/|y|,
 * tracked by its own recurrence and confirmed by a direct evaluation, is below tol.
 * Returns the number of iterations (negative if maxiter was reached).
 */
static double or_norm2(long n, const cplx *a)
{
    double s = 0;
    for (long i = 0; i < n; i++) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
}

int or_cgnr(const cplx *U, const cplx *A, int ns, int nt, double xi, double bc_t,
            const cplx *y, cplx *x, double tol, int maxiter, double *true_resid)
{
    long V = (long)ns * ns * ns * nt, n = 12 * V;
    cplx *r = (cplx *)malloc(sizeof(cplx) * n);   /* normal-equation residual */
    cplx *p = (cplx *)malloc(sizeof(cplx) * n);
    cplx *q = (cplx *)malloc(sizeof(cplx) * n);
    cplx *res = (cplx *)malloc(sizeof(cplx) * n); /* y - Omega x */
    double ynorm = sqrt(or_norm2(n, y));
    int it = 0, converged = 0;
    memset(x, 0, sizeof(cplx) * n);
    if (ynorm == 0) { *true_resid = 0; goto out; }
    memcpy(res, y, sizeof(cplx) * n);
    or_omega(U, A, ns, nt, xi, bc_t, 1, res, r);
    memcpy(p, r, sizeof(cplx) * n);
    double rr = or_norm2(n, r);
    for (int pass = 0; pass < 4 && !converged; pass++) {
        while (it < maxiter) {
            or_omega(U, A, ns, nt, xi, bc_t, 0, p, q);
            double qq = or_norm2(n, q);
            double alpha = rr / qq;
            for (long i = 0; i < n; i++) { x[i] += alpha * p[i]; res[i] -= alpha * q[i]; }
            it++;
            if (sqrt(or_norm2(n, res)) <= tol * ynorm) break;
            or_omega(U, A, ns, nt, xi, bc_t, 1, q, q);
            for (long i = 0; i < n; i++) r[i] -= alpha * q[i];
            double rr_new = or_norm2(n, r);
            double beta = rr_new / rr;
            rr = rr_new;
            for (long i = 0; i < n; i++) p[i] = r[i] + beta * p[i];
        }
        /* confirm with a direct evaluation; restart from it if the recurrence drifted */
        or_omega(U, A, ns, nt, xi, bc_t, 0, x, q);
        for (long i = 0; i < n; i++) res[i] = y[i] - q[i];
        double tr = sqrt(or_norm2(n, res)) / ynorm;
        *true_resid = tr;
        if (tr <= tol) { converged = 1; break; }
        if (it >= maxiter) break;
        or_omega(U, A, ns, nt, xi, bc_t, 1, res, r);
        memcpy(p, r, sizeof(cplx) * n);
        rr = or_norm2(n, r);
    }
out:
    free(r); free(p); free(q); free(res);
    return converged ? it : -it;
}

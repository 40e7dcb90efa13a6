// Storage policies and the even-odd Wilson-clover hopping kernel.
//
// One lane computes one output site of one right-hand side; lanes of a wave take
// consecutive right-hand sides of a site first (layout [12][Vh][R]) so a link or clover
// element is fetched once per site and broadcast to the R lanes that need it.
//
// Hopping term (frozen reading of the anisotropic Wilson operator):
//   (D psi)(x) = sum_mu w_mu [(1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu)]
// with w_4 = -1/2 and w_k = -1/(2 xi), times bc_t on hops across the time boundary.
// In the chiral basis each (1 -+ g_mu) has rank two: the kernel forms the two-spinor
// h = P psi, multiplies only h by the link and rebuilds the lower spin pair from it.
#pragma once

#include "laph_impl.h"

// --------------------------------------------------------------- storage policies
// Element index of component k (alpha*3 + c) of right-hand side r at site i:
//   FP64 vectors keep one plane per component ([12][Vh][R], fully coalesced for R = 1);
//   lower precisions store each site-RHS spinor contiguously ([Vh][R][12]) so that a
//   lane fetches it with a few 16-byte loads.
struct S64 {
    using E = double2;
    using A = double;
    static constexpr bool kNorm = false;
    static constexpr bool kAoS = false;
    static constexpr int bytes = 16;
    __host__ __device__ static long idx(int k, long i, int r, long Vh, int R) { return ((long)k * Vh + i) * R + r; }
    __device__ static Cx<double> ld(const E *p, long i, float) { E v = p[i]; return {v.x, v.y}; }
    __device__ static void st(E *p, long i, Cx<double> v, float) { p[i] = make_double2(v.re, v.im); }
};
struct S32 {
    static constexpr bool kAoS = true;
    // chunked records (spinor_io.h): 2 complex per 16-byte chunk, 6 chunks
    __host__ __device__ static long idx(int k, long i, int r, long Vh, int R) { return ((i * 6 + k / 2) * R + r) * 2 + k % 2; }
    using E = float2;
    using A = float;
    static constexpr bool kNorm = false;
    static constexpr int bytes = 8;
    __device__ static Cx<float> ld(const E *p, long i, float) { E v = p[i]; return {v.x, v.y}; }
    __device__ static void st(E *p, long i, Cx<float> v, float) { p[i] = make_float2(v.re, v.im); }
};
// FP16 with one FP32 scale per site and right-hand side (value = half * scale)
struct S16 {
    static constexpr bool kAoS = true;
    // chunked records (spinor_io.h): 4 complex per 16-byte chunk, 3 chunks
    __host__ __device__ static long idx(int k, long i, int r, long Vh, int R) { return ((i * 3 + k / 4) * R + r) * 4 + k % 4; }
    using E = __half2;
    using A = float;
    static constexpr bool kNorm = true;
    static constexpr int bytes = 4;
    __device__ static Cx<float> ld(const E *p, long i, float s)
    {
        float2 f = __half22float2(p[i]);
        return {f.x * s, f.y * s};
    }
    __device__ static void st(E *p, long i, Cx<float> v, float inv)
    {
        p[i] = __floats2half2_rn(v.re * inv, v.im * inv);
    }
};
// BF16 (8-bit mantissa, FP32 range; no scale needed): (re, im) packed low/high
struct SB16 {
    static constexpr bool kAoS = true;
    // chunked records (spinor_io.h): 4 complex per 16-byte chunk, 3 chunks
    __host__ __device__ static long idx(int k, long i, int r, long Vh, int R) { return ((i * 3 + k / 4) * R + r) * 4 + k % 4; }
    using E = uint32_t;
    using A = float;
    static constexpr bool kNorm = false;
    static constexpr int bytes = 4;
    __device__ static float b2f(uint32_t h) { return __uint_as_float(h << 16); }
    __device__ static uint32_t f2b(float f)
    {
        uint32_t u = __float_as_uint(f);
        u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
        return u >> 16;
    }
    __device__ static Cx<float> ld(const E *p, long i, float)
    {
        uint32_t v = p[i];
        return {b2f(v & 0xFFFFu), b2f(v >> 16)};
    }
    __device__ static void st(E *p, long i, Cx<float> v, float) { p[i] = f2b(v.re) | (f2b(v.im) << 16); }
};

struct G64 {
    using E = double2;
    static constexpr int bytes = 16;
    template <typename A>
    __device__ static Cx<A> ld(const E *p, long i) { E v = p[i]; return {(A)v.x, (A)v.y}; }
};
struct G32 {
    using E = float2;
    static constexpr int bytes = 8;
    template <typename A>
    __device__ static Cx<A> ld(const E *p, long i) { E v = p[i]; return {(A)v.x, (A)v.y}; }
};
struct C64 {
    using E = double;
    static constexpr int bytes = 8;
};
struct C32 {
    using E = float;
    static constexpr int bytes = 4;
};

// epilogue modes
enum {
    M_PLAIN = 0,      // out = c D psi [+ a x]
    M_INV_AFTER = 1,  // out = a x + c A^-1 D psi
    M_INV_OF_SUM = 2, // out = A^-1 (a x + c D psi)
    M_CLOV_ADD = 3,   // out = A x + c D psi
    M_INV_AFTER_DAG = 4, // as M_INV_AFTER, and also out2 = A^-1 gamma_5 out and per-block
                         // partial sums of |out|^2 (multi-RHS low-precision kernel only)
    M_PLAIN_CG = 5,      // as M_PLAIN with out consumed by a CG update instead of stored
                         // (multi-RHS low-precision kernel only)
    M_INV_AFTER_DOT = 6  // as M_INV_AFTER, and also per-block partial sums of <y, out> and
                         // |out|^2 for a second own-site field y (BiCGStab; multi-RHS
                         // low-precision kernel only)
};

struct DslashArgs {
    void *out;
    const void *in;
    const void *x;  // same parity as out (may be null for M_PLAIN / M_INV_AFTER)
    float *out_nrm;
    const float *in_nrm;
    const float *x_nrm;
    const void *gauge;
    const void *clov;  // packed clover block set (A or A^-1) of the output parity
    int ns, nt;
    long Vh;
    int R;
    int par;        // output parity
    double a, c;    // epilogue coefficients
    double wt, ws;  // hop weights (time, space), including the -1/2
    double bct;     // sign on hops across the time boundary
    int g5d;        // 1: gamma_5 applied to D psi before the epilogue
    int wby, wbz;   // site walk: tiles of Ns x wby x wbz sites through all time slices (set
                    // by the launcher; 0: checkerboard order)
};

// launcher (dslash.hip); SPI = storage of in/out/x
template <class SP, class GP, class CP>
void launch_dslash(laph_ctx *c, int mode, const DslashArgs &a, hipStream_t st);

// local clover application out = [gamma_5] A x [gamma_5-free], x and out same parity
template <class SP, class CP>
void launch_clover_apply(laph_ctx *c, const void *clov, const void *x, const float *x_nrm, void *out,
                         float *out_nrm, long Vh, int R, int g5_in, hipStream_t st);

double dslash_bytes(long Vh, int R, int gbytes, int cbytes, int sbytes, bool has_norm, int mode, bool has_x);

// Internal definitions of the MI355X stochastic-LapH library (not part of the ABI).
//
// Device layouts (all "SoA over the per-site components", sites of one parity
// contiguous so that consecutive lanes of a wave touch consecutive addresses):
//   even-odd links   : T g[((mu*2 + par)*9 + a*3 + b)*Vh + i]          (T = double2/float2)
//   half spinor (R)  : S s[(k*Vh + i)*R + r],  k = alpha*3 + c          (R right-hand sides)
//   clover / inverse : double c[(par*72 + blk*36 + e)*Vh + i]  two Hermitian 6x6 chiral
//                      blocks per site packed as 6 real diagonals then the 15 complex
//                      entries below the diagonal, row-major.
//   smeared links    : double2 u[(k*9 + a*3 + b)*V + s]  (full lattice, k = 0,1,2)
// Checkerboard index of a site is lex/2 with lex = x + Ns(y + Ns(z + Ns t)); parity
// (x+y+z+t) & 1, even = 0.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/laph.h"

// ---------------------------------------------------------------- error handling
struct LaphError {
    int code;
};

#define LAPH_HIP(call)                                                                       \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) {                                                              \
            laph_fail(LAPH_EHIP, "%s:%d %s: %s", __FILE__, __LINE__, #call,                   \
                      hipGetErrorString(e_));                                                \
        }                                                                                    \
    } while (0)

#define LAPH_CHECK(cond, code, ...)                                                          \
    do {                                                                                     \
        if (!(cond)) laph_fail(code, __VA_ARGS__);                                           \
    } while (0)

[[noreturn]] void laph_fail(int code, const char *fmt, ...);

// -------------------------------------------------------------- complex helpers
__host__ __device__ inline double2 cmake(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cconjmul(double2 a, double2 b)  // conj(a) * b
{
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__host__ __device__ inline double2 cdiv(double2 a, double2 b)
{
    double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__host__ __device__ inline double cnorm2(double2 a) { return a.x * a.x + a.y * a.y; }

// Generic complex over a real type (float or double) for templated kernels.
template <typename R>
struct Cx {
    R re, im;
};
template <typename R>
__device__ __forceinline__ Cx<R> operator+(Cx<R> a, Cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> operator-(Cx<R> a, Cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> operator*(Cx<R> a, Cx<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ Cx<R> operator*(R s, Cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> conjmul(Cx<R> a, Cx<R> b)  // conj(a) * b
{
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename R>
__device__ __forceinline__ Cx<R> timesI(Cx<R> a) { return {-a.im, a.re}; }
template <typename R>
__device__ __forceinline__ Cx<R> timesMinusI(Cx<R> a) { return {a.im, -a.re}; }
template <typename R>
__device__ __forceinline__ Cx<R> cneg(Cx<R> a) { return {-a.re, -a.im}; }

// ---------------------------------------------------------------- geometry
struct Geom {
    int ns, nt;
    long V, Vh, V3;
};

__device__ __forceinline__ void cb_coords(long i, int par, int ns, int &x, int &y, int &z, int &t)
{
    int nsh = ns >> 1;
    long r = i / nsh;
    int xh = (int)(i - r * nsh);
    y = (int)(r % ns);
    r /= ns;
    z = (int)(r % ns);
    t = (int)(r / ns);
    x = 2 * xh + ((y + z + t + par) & 1);
}

__device__ __forceinline__ long lex_index(int x, int y, int z, int t, int ns)
{
    return x + (long)ns * (y + (long)ns * (z + (long)ns * t));
}

// XCD-aware block index: the hardware deals consecutive workgroups round-robin over the
// 8 XCDs; remap so that each XCD works on one contiguous range of the grid and the
// neighbour re-reads of a stencil stay in that XCD's L2.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nblocks)
{
    const unsigned nx = 8;
    unsigned per = nblocks / nx;
    if (b >= per * nx) return b;  // ragged tail keeps its index
    return (b % nx) * per + b / nx;
}

// ---------------------------------------------------------------- buffers
// Every device buffer of the library is a piece of the caller's workspace
// (laph_set_workspace): named scratch buffers of one call are taken from its bottom and
// released when the call returns; the cached operators of a gauge field live at its top
// until another field, a workspace change or a lack of room evicts them.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// ---------------------------------------------------------------- gauge caches
struct DiracCache {
    const double *U = nullptr;  // caller pointer the cache was built from
    uint64_t fp = 0;            // fingerprint of that field's contents
    laph_dirac prm{};
    bool valid = false;
    DevBuf unit;    // the cache's piece of the workspace, carved into the fields below
    DevBuf g64;     // even-odd links FP64 (double2)
    DevBuf clov;    // clover FP64 packed
    DevBuf clinv;   // clover inverse FP64 packed
    DevBuf lk12;    // reconstruct-12 FP32 links, per-site AoS (low-precision operator)
    DevBuf claos;   // FP32 clover inverse, per-site AoS (low-precision operator)
    bool has_f32 = false;  // the unit holds lk12 / claos
    bool f32 = false;      // lk12 / claos are current
    // temporal gauge (the solver's cache): the operator is built from U' = G U G^dag with
    // unit time links except on the last slice; gU holds U', gG the rotations G(x)
    bool tgauge = false;
    DevBuf gU, gG;
};

struct laph_ctx {
    Geom g;
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;
    DiracCache dc;   // operator of the caller's field (apply entry points)
    DiracCache dct;  // the same operator in temporal gauge (low-precision solves)
    DiracCache *cur = &dc;  // the cache the running solve uses
    // temporal-gauge rotations the running solve folds into its layout conversions: G on
    // the source (null where the source is rotated beforehand) and G^dag on the solution
    const double *tg_in = nullptr, *tg_out = nullptr;
    std::map<std::string, DevBuf> bufs;  // named scratch buffers of the running call
    // caller workspace: scratch [0, ws_lo), the cache unit [ws_bytes - ws_hi, ws_bytes).
    // At most one cached operator is held; the running call pins the one it prepared, and
    // an unpinned one is evicted when scratch needs its room.
    char *ws = nullptr;
    size_t ws_bytes = 0, ws_lo = 0, ws_hi = 0;
    DiracCache *ws_unit = nullptr;
    bool ws_pinned = false;
    // device address of the fixed scratch array of sink_project_noalloc on this device
    void *sink_scratch = nullptr;
    // autotuning: LDS tile (sites per block) per (precision, R) and the chosen R per
    // precision (0: not tuned)
    std::map<std::pair<int, int>, int> lds_tile;
    std::map<int, int> tuned_R;
    // launch overrides of the multi-RHS hopping kernel, set only for the duration of a
    // laph_hop_apply call: walk_mode 1 visits sites in checkerboard order instead of the
    // tiled walk, tile_override > 0 fixes the sites per block
    int walk_mode = 0;
    int tile_override = 0;
    hipStream_t cap_stream = nullptr;  // capture stream for HIP graphs (default priority)
    // pinned two-slot readback of the per-RHS Krylov scalars and the events marking each
    // slot's copy (the CG loop reads the previous iteration's slot without draining the queue)
    void *pin = nullptr;
    size_t pin_bytes = 0;
    hipEvent_t pin_ev[2] = {nullptr, nullptr};
    // timing
    struct TimeAcc {
        double ms = 0, bytes = 0;
        long launches = 0;
    };
    bool timing = false;
    std::map<std::string, TimeAcc> tacc;  // per kernel variant
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;  // recorded, not yet read
    std::vector<double> pending_bytes;
    std::vector<const char *> pending_label;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> event_pool;
};

// named scratch buffer of the running call (grow-only within the call; released when the
// call returns); LAPH_ENOMEM when the workspace has no room
void *ctx_named(laph_ctx *c, const std::string &name, size_t bytes);
// release every scratch buffer (end of an ABI call)
void scratch_reset(laph_ctx *c);
// give cache dc a unit of at least `bytes` at the top of the workspace (the other cache is
// evicted) and pin it for the running call; the unit's contents are undefined afterwards
// when it moved
void cache_unit(laph_ctx *c, DiracCache &dc, size_t bytes);
// drop the cache unit (its fields become invalid)
void cache_release_all(laph_ctx *c);
// bytes of a Dirac cache unit (FP64 operator; with f32 the low-precision operator; with
// tgauge also U' and G) and the layout of its fields
size_t cache_unit_bytes(const Geom &g, bool tgauge, bool f32);
void cache_carve(laph_ctx *c, DiracCache &dc, bool tgauge, bool f32);
// 64-bit fingerprint of a gauge field's contents (device pass over all links)
uint64_t gauge_fingerprint(laph_ctx *c, const double *U);
inline size_t ws_align(size_t n) { return (n + 255) & ~size_t(255); }


// ---------------------------------------------------------------- internal API
// source.hip: look up the device address of sink_project_noalloc's scratch array (once per
// device, with the context's device current)
void sink_scratch_init(laph_ctx *c);
// layout.hip
void links_to_eo(laph_ctx *c, const double *U, double2 *g64);
void eo64_to_eo32(laph_ctx *c, const double2 *g64, float2 *g32, long n);
// gam: 0 none, 4 multiply by gamma_4, 5 multiply by gamma_5 (applied per site)
// G (may be null): site-local colour rotations [V][3][3] applied to the field on the way in
// (to_eo) or their adjoints on the way out (from_eo)
void spinor_to_eo(laph_ctx *c, const double *psi, int nrhs, int gam, double2 *even, double2 *odd,
                  const double *G = nullptr);
void spinor_from_eo(laph_ctx *c, const double2 *even, const double2 *odd, int nrhs, int gam, double *psi,
                    const double *G = nullptr);
void smeared_links_to_soa(laph_ctx *c, const double *U, double2 *us);

// clover.hip
void clover_build(laph_ctx *c, const double *U, const laph_dirac *d, double *clov, double *clinv);
void clover_to_f32(laph_ctx *c, const double *cl, float *cl32);

// dirac setup shared by the solver and the apply entry point
void dirac_prepare(laph_ctx *c, const double *U, const laph_dirac *d, bool need_f32);
// the solver's temporal-gauge cache c->dct (FP64 and low-precision operator of U')
void dirac_prepare_tgauge(laph_ctx *c, const double *U, const laph_dirac *d);

// tgauge.hip: G (double2 [V][3][3]) and U' = G U G^dag (ABI layout) of the field U;
// out = G in (dag: G^dag in) for nrhs canonical spinor fields (in == out allowed)
void tgauge_fix(laph_ctx *c, const double *U, double *G, double *Up);
void tgauge_spinor(laph_ctx *c, const double *G, const double *in, double *out, int nrhs, int dag);

// stout.hip
void stout_smear_device(laph_ctx *c, const double *U, double rho, int nsteps, double *out);

// timing
void timing_begin(laph_ctx *c, hipEvent_t *a, hipEvent_t *b);
void timing_end(laph_ctx *c, hipEvent_t a, hipEvent_t b, double bytes, const char *label);
void timing_collect(laph_ctx *c);
// stable name "kernel<prec,mode,R>" for timing_end (mode: M_* of dslash.h)
const char *timing_label(const char *kernel, const char *prec, int mode, int R);

// launch helper
inline unsigned nblocks_for(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

struct ScratchScope {
    laph_ctx *c;
    ~ScratchScope() { scratch_reset(c); }
};

#define LAPH_API_BEGIN(ctx)                                                                  \
    try {                                                                                    \
        if (!(ctx)) return LAPH_EINVAL;                                                      \
        ScratchScope scratch_scope_{ctx};                                                    \
        LAPH_HIP(hipSetDevice((ctx)->device));

#define LAPH_API_END(ctx)                                                                    \
    }                                                                                        \
    catch (const LaphError &e_) {                                                            \
        return e_.code;                                                                      \
    }                                                                                        \
    catch (...) {                                                                            \
        return LAPH_EHIP;                                                                    \
    }                                                                                        \
    return LAPH_OK;

extern thread_local laph_ctx *g_current_ctx;  // context of the running API call (errors)

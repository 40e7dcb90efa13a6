/*
 * laph.h -- C ABI of the MI355X stochastic-LapH hot path.
 *
 * The calls follow the statement of the problem in Morningstar et al. (arXiv:1104.3870):
 * the LapH subspace V_s of the stout-smeared 3D covariant Laplacian (Sec. II, Eq. smearA
 * and the definition of V_s; eigensolver of Sec. IV), Z4 noise rho diluted by projectors
 * P^(b) in that subspace (Sec. II, dilution schemes; Sec. IV, Z4 noise), the solve of
 * Omega x = V_s P^(b) rho with Omega = gamma_4 K (Sec. II, Sec. IV), and the quark
 * propagation coefficients V_s^dag x (Sec. IV).
 *
 * Conventions shared by every call (frozen readings where the paper is silent):
 *  - lattice Ns^3 x Nt, Ns and Nt even; site s = x + Ns*(y + Ns*(z + Ns*t));
 *  - complex numbers are interleaved (re, im) doubles;
 *  - gauge links    U[((s*4 + mu)*3 + a)*3 + b], mu = 0,1,2 space, 3 time;
 *  - spinor fields  psi[(s*4 + alpha)*3 + c]; n fields are stored back to back;
 *  - colour fields  v[s*3 + c];
 *  - eigenvectors   evecs[((t*Nv + n)*Ns^3 + xyz)*3 + c];
 *  - coefficients   coef[((r*Nt + t)*4 + alpha)*Nv + n];
 *  - noise          rho[(t*4 + alpha)*Nv + n].
 *  - gamma matrices: Hermitian chiral basis, gamma_k = [[0,-i sigma_k],[i sigma_k,0]],
 *    gamma_4 = [[0,1],[1,0]], gamma_5 = diag(1,1,-1,-1).
 *
 * Ownership: the caller owns every pointer and the library never frees caller memory.
 * Field arguments are DEVICE pointers unless stated otherwise; statistics structs and
 * eigenvalues are host memory.  The library allocates no device memory: its scratch and
 * the operator it derives from a gauge field live in a workspace the caller provides
 * (laph_set_workspace, sized by laph_workspace_bytes).  The derived operator is cached for
 * the last gauge field seen, keyed by the field's address and a fingerprint of its
 * contents, so a field changed in place or a new field at a freed one's address is
 * noticed; laph_forget_gauge() drops the cache.  The library keeps one small pinned host
 * buffer per context for the solver's scalar readback.
 * Every call enqueues work on the context's HIP stream; calls that return statistics
 * synchronise that stream.  One context per stream; contexts share nothing.
 *
 * Errors: every call returns an int status (LAPH_OK on success); no C++ exception
 * crosses the ABI.  laph_strerror() names a status, laph_last_error() gives detail.
 */
#ifndef LAPH_H
#define LAPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define LAPH_API __attribute__((visibility("default")))
#else
#define LAPH_API
#endif

enum {
    LAPH_OK = 0,
    LAPH_EINVAL = 1,  /* bad argument: null pointer, odd extent, out-of-range index */
    LAPH_EDIVIDE = 2, /* a dilution N/J that is not an integer (Sec. II) */
    LAPH_ENOCONV = 3, /* true residual above tol after every fallback; x holds the best iterate */
    LAPH_EEIG = 4,    /* eigensolver reached max_restarts before all N_v pairs converged */
    LAPH_EHIP = 5,    /* HIP runtime error */
    LAPH_ENOMEM = 6   /* the workspace (laph_set_workspace) is too small for the call */
};

typedef struct laph_ctx *laph_ctx_t;

typedef struct {
    int ns; /* spatial extent (even) */
    int nt; /* temporal extent (even) */
} laph_geom;

/* ------------------------------------------------------------------ context */

/* Create a context for one lattice geometry; hip_stream is a hipStream_t (NULL: the
 * null stream).  The device is the one current when this is called. */
LAPH_API int laph_create(laph_ctx_t *ctx, const laph_geom *geom, void *hip_stream);
LAPH_API int laph_destroy(laph_ctx_t ctx);
LAPH_API const char *laph_strerror(int status);
LAPH_API const char *laph_last_error(laph_ctx_t ctx);
/* Drop every cached field derived from a gauge field. */
LAPH_API int laph_forget_gauge(laph_ctx_t ctx);
/* Workspace bytes in use: the cached operator plus the running call's scratch. */
LAPH_API size_t laph_device_bytes(laph_ctx_t ctx);

/* -------------------------------------------------- stout smearing (Sec. II)
 * Spatial stout smearing (Morningstar & Peardon 2004) with spatial staples only; time
 * links are copied unchanged.  U_out may not alias U. */
typedef struct {
    double rho; /* staple weight */
    int nsteps;
} laph_stout;

LAPH_API int laph_stout_smear(laph_ctx_t ctx, const double *U, const laph_stout *stout, double *U_out);

/* ------------------------------------------------ Laplacian (Sec. II, Sec. IV)
 * out = Lap v on every time slice, (Lap v)(x) = sum_k [U_k(x) v(x+k) + U_k(x-k)^dag
 * v(x-k) - 2 v(x)], with U the (smeared) links given.  v, out: colour fields [V][3]. */
LAPH_API int laph_laplacian_apply(laph_ctx_t ctx, const double *U, const double *v, double *out);

/* out = T_order(B) v with B = 1 + 2/(lambda_L - lambda_C) (Lap + lambda_C)  (Sec. IV,
 * Chebyshev acceleration). */
LAPH_API int laph_chebyshev_apply(laph_ctx_t ctx, const double *U, double lambda_L, double lambda_C,
                         int order, const double *v, double *out);

/* --------------------------------------------------------- LapH eigenvectors
 * The N_v lowest eigenpairs of -Lap on every time slice of the stout-smeared field
 * (Sec. II, definition of V_s) by the Krylov-spectral restarted Lanczos method with
 * Chebyshev acceleration, full reorthogonalisation with the kappa = sqrt(2) rule (at
 * most four extra passes), locking of converged pairs and the convergence test
 * |A x - lambda x| < tol |A| (Sec. IV).  Eigenvalues are the Rayleigh quotients on
 * -Lap, ascending per slice; each eigenvector is multiplied by the phase that makes its
 * first component (storage order) of modulus >= 0.1 of the largest real and positive
 * (the paper asks for a convention without stating it).  U is the UNSMEARED field; the
 * call smears it.  evals: HOST [Nt][Nv]; evecs: device [Nt][Nv][Ns^3][3]. */
typedef struct {
    int krylov_dim;     /* m, at most 160 */
    int cheb_order;     /* n of T_n */
    double lambda_L;    /* upper bound of the spectrum of -Lap */
    double lambda_C;    /* cut-off above the wanted part */
    double tol;         /* convergence tolerance relative to |A| */
    int max_restarts;
    uint32_t seed;      /* start vectors are Philox draws from this seed */
} laph_lanczos;

typedef struct {
    int restarts;        /* restarts used */
    int matvecs;         /* applications of A = T_n(B) per slice */
    double max_residual; /* max over pairs of |(-Lap) v - lambda v| */
    double max_orth;     /* max over slices of |V^dag V - 1| (elementwise) */
    double min_gap;      /* min over slices of (next Ritz value) - lambda_{Nv}, estimate */
} laph_eig_stats;

LAPH_API int laph_eigvecs(laph_ctx_t ctx, const double *U, const laph_stout *stout,
                 const laph_lanczos *lanczos, int nv, double *evals, double *evecs,
                 laph_eig_stats *stats);

/* ------------------------------------------------- noise and dilution (Sec. II)
 * Dilution projector families (Sec. II): none "1", full "F", block-J "BJ" (b = J i / N),
 * interlace-J "IJ" (b = i mod J), applied to time (N = Nt), spin (N = 4) and LapH
 * index (N = Nv).  The projector index is b = (b_T * n_S + b_S) * n_L + b_L. */
enum { LAPH_DIL_NONE = 0, LAPH_DIL_FULL = 1, LAPH_DIL_BLOCK = 2, LAPH_DIL_INTERLACE = 3 };

typedef struct {
    int type[3]; /* time, spin, LapH */
    int J[3];    /* J for block / interlace, ignored otherwise */
} laph_dilution;

/* Parse "TI16,SF,LI8" or "(TF, SF, LB4)"; LAPH_EDIVIDE when N/J is not an integer.
 * Host-only; needs no context. */
LAPH_API int laph_parse_dilution(const char *text, int nt, int nv, laph_dilution *out);
/* number of projectors n_T * n_S * n_L, or -1 for an invalid scheme. Host-only. */
LAPH_API long laph_dilution_count(const laph_dilution *dil, int nt, int nv);

/* Z4 noise rho(t, alpha, n) = i^(w mod 4), w the first word of Philox4x32-10 with counter
 * (n, alpha, t, 0) and key ((k << 16) | s, 0x4C415048) (Sec. IV names the noise by a
 * 16-bit id s and a 16-bit configuration id k; the generator is our reading).
 * rho: device [Nt][4][Nv]. */
LAPH_API int laph_z4_noise(laph_ctx_t ctx, uint16_t noise_s, uint16_t config_k, int nv, double *rho);

/* element type of a field written by the library */
enum { LAPH_DTYPE_C128 = 0, LAPH_DTYPE_C64 = 1 };

/* eta^[b] = V_s P^(b) rho for the n_src projector indices b_first .. b_first+n_src-1
 * (Sec. IV, right-hand side y = V_s P^[b] rho).  eta: device, n_src spinor fields of
 * complex128 (dtype LAPH_DTYPE_C128, what dirac_solve takes) or complex64
 * (LAPH_DTYPE_C64: the FP64 sums rounded once, for callers with their own solver);
 * another dtype gives LAPH_EINVAL. */
LAPH_API int make_diluted_source(laph_ctx_t ctx, const double *evecs, int nv, uint16_t noise_s,
                        uint16_t config_k, const laph_dilution *dil, int64_t b_first,
                        int n_src, void *eta, int dtype);

/* ------------------------------------------------------------- Dirac operator
 * K = A + H, the anisotropic Wilson-clover matrix (frozen reading; the paper names an
 * improved anisotropic clover action, Sec. V):
 *   (H psi)(x) = -1/2 sum_mu w_mu [(1-gamma_mu) U_mu(x) psi(x+mu) + (1+gamma_mu) U_mu(x-mu)^dag psi(x-mu)]
 *   w_4 = 1, w_k = 1/xi, every hop across t = Nt-1 <-> 0 multiplied by bc_t,
 *   A(x) = m0 + 1 + 3/xi - 1/2 [c_t sum_k sigma_k4 F_k4 + c_s sum_{k<l} sigma_kl F_kl],
 *   c_s = c_sw/xi, c_t = c_sw (1 + 1/xi)/2, F the traceless anti-Hermitian part of the
 *   four-leaf clover divided by 8i.  Omega = gamma_4 K (Sec. II). */
typedef struct {
    double m0;
    double xi;
    double c_sw;
    double bc_t; /* -1: antiperiodic fermions */
} laph_dirac;

enum { LAPH_OP_K = 0, LAPH_OP_OMEGA = 1, LAPH_OP_KDAG = 2 };

/* out = op(in) on n_fields spinor fields (full lattice, FP64). */
LAPH_API int laph_dirac_apply(laph_ctx_t ctx, const double *U, const laph_dirac *dirac, int op,
                     const double *in, double *out, int n_fields);

enum { LAPH_PREC_F64 = 0, LAPH_PREC_F32 = 1, LAPH_PREC_F16 = 2, LAPH_PREC_BF16 = 3 };

/* ---------------------------------------------- even-odd hopping kernels
 * One launch of the hopping kernels that the solver of Omega x = eta runs (Sec. II: K
 * split by site parity; Sec. IV: the even-odd preconditioned solve in mixed precision), on
 * caller fields, so that each kernel and its fused epilogue can be checked against a
 * reference in every storage precision.  With D_{p,1-p} the hopping term H of K from the
 * sites of parity 1-p to those of parity p (H as under laph_dirac_apply, its -1/2 and the
 * weights included), A_pp the clover term of parity p and g5 = gamma_5 when hop->gamma5
 * is set (else 1), the launch computes on the sites of the output parity p:
 *   LAPH_HOP_PLAIN:    out = c g5 D in + a x                (x may be NULL: no addend)
 *   LAPH_HOP_INV:      out = a x + c A_pp^-1 g5 D in        (x may be NULL)
 *   LAPH_HOP_INV_DAG:  as LAPH_HOP_INV (x required, c != 0), and also
 *                      out2 = A_pp^-1 gamma_5 out and norm2[r] = |out_r|^2,
 *                      both from out as stored in the storage precision
 *   LAPH_HOP_PLAIN_CG: r -= alpha_r (c g5 D in + a x) with r = out on entry (x required),
 *                      norm2[r] = |r_r|^2 after the update, from r as stored
 *   LAPH_HOP_INV_DOT:  as LAPH_HOP_INV (x required), and the two inner products of a
 *                      BiCGStab step (Sec. IV) from out as stored: out2 is an INPUT here,
 *                      a field y read on parity p, and norm2 (3 n_fields values) receives
 *                      per field Re <y_r, out_r>, Im <y_r, out_r>, |out_r|^2, with
 *                      <y, out> = sum conj(y) out (out2 == x: y is x, the kernel's
 *                      form that reuses the loaded x)
 * The input is read on the sites of parity 1-p, x and r on parity p; every output is
 * written on parity p and zero on parity 1-p.  Fields are converted to the storage
 * precision (FP16 records carry one FP32 scale per site and field), the kernel runs in
 * FP32 arithmetic with FP32 reconstruct-12 links and FP32 clover inverse (LAPH_PREC_F64:
 * the FP64 kernel, modes PLAIN and INV only), and the results come back as FP64.
 * temporal_gauge = 1 builds the operator from U' = G U G^dag with unit time links except
 * on the last slice (the low-precision solves' form, whose kernel skips the unit links),
 * applies G to the fields on the way in and G^dag on the way out: the result is the
 * operator of U either way.  walk = 1 visits the sites in checkerboard order instead of
 * the tiled walk; sites_per_block > 0 fixes the tile (S sites x n_fields lanes, S
 * n_fields <= 256).
 * in, x, out, out2: device, n_fields canonical spinor fields each; alpha, norm2: HOST
 * arrays of n_fields (norm2 may be NULL).  n_fields: a power of two <= 32 (one launch). */
enum { LAPH_HOP_PLAIN = 0, LAPH_HOP_INV = 1, LAPH_HOP_INV_DAG = 2, LAPH_HOP_PLAIN_CG = 3, LAPH_HOP_INV_DOT = 4 };

typedef struct {
    int precision;       /* LAPH_PREC_* of the fields the kernel reads and writes */
    int mode;            /* LAPH_HOP_* */
    int parity;          /* output parity p: 0 even, 1 odd ((x + y + z + t) mod 2) */
    int gamma5;          /* 1: gamma_5 applied to D in */
    int temporal_gauge;  /* 1: operator built in temporal gauge (see above) */
    int walk;            /* 0: tiled site walk where the lattice allows it; 1: checkerboard */
    int sites_per_block; /* low precisions: sites per thread block; 0: tuned or default */
    double a, c;         /* epilogue coefficients */
} laph_hop;

LAPH_API int laph_hop_apply(laph_ctx_t ctx, const double *U, const laph_dirac *dirac, const laph_hop *hop,
                            const double *in, const double *x, double *out, double *out2, const double *alpha,
                            double *norm2, int n_fields);

enum { LAPH_SOLVER_BICGSTAB = 0, LAPH_SOLVER_CGNR = 1, LAPH_SOLVER_FGMRES = 2 };

typedef struct {
    double tol;         /* true relative residual |eta - Omega x| / |eta| in FP64 */
    int maxiter;        /* Krylov iterations per right-hand side and attempt */
    int solver;         /* LAPH_SOLVER_*: BiCGStab on the even-odd system with CGNR fallback
                           (Sec. IV), CGNR only, or FGMRES with a learned preconditioner */
    int precision;      /* LAPH_PREC_*: storage precision of the inner Krylov vectors;
                           FP64 reliable updates are used for every lower precision */
    int reliable_every; /* most iterations between FP64 reliable updates (mixed precision) */
    int block_rhs;      /* right-hand sides iterated together (power of two <= 32); 0 = the
                           block size laph_autotune picks (run on first use) */
    int use_graph;      /* replay the Krylov iteration's hops and reductions from HIP graphs
                           (mixed-precision BiCGStab and CGNR; not with timing on) */
    const void *net;    /* learned network (laph_ptnet_t) or NULL: the right preconditioner of
                           LAPH_SOLVER_FGMRES; with the other solvers the initial guess
                           x0 = N(gamma_4 eta) on odd sites (N approximates K^-1) */
    int restart;        /* FGMRES restart length (0: 24) */
    double reliable_delta; /* mixed precision: FP64 reliable update once half of a block's
                              active right-hand sides have their iterated even-odd residual
                              below this fraction of its last FP64 value (0: 0.1) or below the
                              target (convergence candidates, confirmed by the FP64 residual),
                              or one non-candidate fell 100 times further, or every active one
                              is a candidate; at the latest every reliable_every iterations */
    int dir_buffers;    /* mixed-precision BiCGStab and CGNR: iterations whose solution steps
                           (alpha p + omega s, or alpha p) are kept owed in buffers before the
                           solution increment is read and written once for all of them
                           (1..8; 0: 8) */
} laph_solver;

typedef struct {
    int iters;          /* Krylov iterations of the successful attempt(s) */
    int status;         /* LAPH_OK or LAPH_ENOCONV */
    int fallback_used;  /* 1 if the CGNR fallback (or plain solver) was needed */
    double true_resid;  /* |eta - Omega x| / |eta| evaluated in FP64 after the solve */
} laph_solve_stats;

/* Solve Omega x = eta for n_rhs right-hand sides (Sec. IV).  eta, x: device, n_rhs
 * spinor fields each (FP64); stats: HOST array of n_rhs (may be NULL).
 * Up to three BiCGStab (or FGMRES) attempts (each restarted from the current x with a
 * tighter even-odd target when the FP64 true residual of the full system misses tol) are
 * followed by the CGNR fallback, which runs up to max(maxiter, 5000) iterations.
 * LAPH_SOLVER_FGMRES solves one right-hand side at a time (block_rhs is ignored) with an
 * FP64 basis and solver->net as right preconditioner; iters counts its iterations (one
 * network application and one even-odd operator each) plus any fallback iterations. */
LAPH_API int dirac_solve(laph_ctx_t ctx, const double *U, const laph_dirac *dirac, const double *eta,
                double *x, int n_rhs, const laph_solver *solver, laph_solve_stats *stats);

/* ------------------------------------------------- learned preconditioner
 * Not in the paper: a gauge-equivariant parallel-transport network N that approximates
 * K^-1 and serves as the right preconditioner of flexible GMRES on the even-odd system
 * (LAPH_SOLVER_FGMRES).  The answer is still judged by the FP64 true residual of
 * Omega x = eta, and a right-hand side the preconditioned solve does not finish falls back
 * to plain CGNR (fallback_used = 1).
 *
 * Layer l maps ch[l] spinor fields to ch[l+1] fields:
 *   out_c(x) = sum_{c', d} W_l[c][c'][d] (T_d phi_c')(x),  d = 0 (self), 1..4 (+mu), 5..8 (-mu),
 *   T_{+mu} phi(x) = U_mu(x) phi(x+mu),  T_{-mu} phi(x) = U_mu(x-mu)^dag phi(x-mu),
 * mu = x, y, z, t, hops across the time boundary multiplied by bc_t.  W_l[c][c'][d] is a
 * complex 4x4 matrix on spin; every layer is therefore gauge equivariant.  Kernels use
 * BF16 copies of the weights (round to nearest even) with FP32 arithmetic; the optimiser
 * keeps FP32 master weights.
 * Weight layout (get/set): layers in order, each [ch[l+1]][ch[l]][9][4][4] complex as
 * interleaved (re, im) doubles; n = sum_l ch[l] ch[l+1] 144 complex numbers.
 * Fields (in, out, gradients): canonical spinor fields, device, FP64. */
#define LAPH_PTNET_MAX_LAYERS 8
typedef struct laph_ptnet *laph_ptnet_t;

/* channels[0..layers]: first and last 1, each 1, 2 or 4.  Weights start as small seeded
 * Gaussian numbers plus 1/ch[l] times the identity on the self path.  The net lives on
 * the device of ctx and may be used with any context on that device. */
LAPH_API int laph_ptnet_create(laph_ctx_t ctx, int layers, const int *channels, uint64_t seed,
                               laph_ptnet_t *net);
LAPH_API int laph_ptnet_destroy(laph_ptnet_t net);
LAPH_API int laph_ptnet_num_weights(laph_ptnet_t net, size_t *n_complex);
/* FP32 master weights as doubles (host array of 2n); set also resets the optimiser. */
LAPH_API int laph_ptnet_get_weights(laph_ptnet_t net, double *w);
LAPH_API int laph_ptnet_set_weights(laph_ptnet_t net, const double *w);
/* out = N(in) for n_fields fields. */
LAPH_API int laph_ptnet_forward(laph_ctx_t ctx, laph_ptnet_t net, const double *U, double bc_t,
                                const double *in, double *out, int n_fields);
/* Backward pass of a real loss L given gout = dL/d(N(in))^*: writes dL/din^* to gin (device,
 * may be NULL) and dL/dW^* (host, 2n doubles, summed over the fields) to gw. */
LAPH_API int laph_ptnet_backward(laph_ctx_t ctx, laph_ptnet_t net, const double *U, double bc_t,
                                 const double *in, const double *gout, double *gin, double *gw,
                                 int n_fields);

typedef struct {
    double lr, beta1, beta2, eps; /* Adam */
    int loss_parity;              /* sites entering the loss: -1 all, 0 even, 1 odd */
} laph_adam;

/* One Adam step on L = sum_r |N(b_r) - x_r|^2 / |x_r|^2 over n_pairs (source, solution)
 * pairs (device fields); *loss (host, may be NULL) receives L / n_pairs before the step. */
LAPH_API int laph_ptnet_train_step(laph_ctx_t ctx, laph_ptnet_t net, const double *U, double bc_t,
                                   const double *b, const double *x, int n_pairs,
                                   const laph_adam *opt, double *loss);

/* ---------------------------------------------------------------- autotuning
 * Times the even-odd hopping kernel with its fused clover-inverse epilogue on the
 * prepared operator of (U, dirac) for every block size R (4..32 for the low precisions,
 * 1..32 for FP64) and, for the low precisions, every tile of S sites x R lanes
 * (S R = 64, 128, 256).  The context keeps the fastest tile per R and the R with the
 * lowest time per right-hand side; dirac_solve with block_rhs = 0 uses them. */
#define LAPH_TUNE_MAX 24
typedef struct {
    int block_rhs;
    int sites_per_block; /* 0 for FP64 */
    double ms_per_rhs;   /* per launch and right-hand side */
} laph_tune_entry;

typedef struct {
    int n;
    laph_tune_entry e[LAPH_TUNE_MAX];
    int best_block_rhs;
    int best_sites_per_block;
} laph_tune_report;

LAPH_API int laph_autotune(laph_ctx_t ctx, const double *U, const laph_dirac *dirac, int precision,
                           laph_tune_report *report);

/* ----------------------------------------------------------- sink projection
 * coef[r][t][alpha][n] = sum_{x,c} conj(V_{t,n}(x,c)) X_r(x,t,c,alpha): the quark
 * propagation coefficients V_s^dag Omega^-1 V_s P^[b] rho (Sec. IV).  X: device n_rhs
 * spinor fields; coef: device [n_rhs][Nt][4][Nv] complex. */
LAPH_API int sink_project(laph_ctx_t ctx, const double *evecs, int nv, const double *X, int n_rhs,
                 double *coef);

/* ------------------------------------------------ hadron functions (Sec. II, III.B)
 * Quark sources and sinks in LapH coordinates, with the trivial displacement: a quark
 * source varrho^[b] = V_s P^(b) rho (Eq. varrhodef) has the coefficients
 * V_s^dag varrho^[b] = P^(b) rho, and a LapH-smeared quark sink varphi^[b] = V_s V_s^dag X^[b]
 * (Eq. varphidef) has the coefficients sink_project(X^[b]).  Coefficient arrays are
 * device [n][Nt][4][Nv] complex (the layout of sink_project); spin matrices are HOST
 * row-major 4x4 complex (32 doubles).
 *
 * laph_quark_source: the coefficients of varrho^[b] for b = b_first .. b_first + n_src - 1
 * (noise as laph_z4_noise), or with bar = 1 those of varrho-bar = -gamma_5 gamma_4 varrho
 * of the gamma_5-Hermitian estimate (Eq. laphpropg5). */
LAPH_API int laph_quark_source(laph_ctx_t ctx, int nv, uint16_t noise_s, uint16_t config_k,
                               const laph_dilution *dil, int64_t b_first, int n_src, int bar, double *out);
/* out[r][t][alpha][n] = sum_beta S[alpha][beta] in[r][t][beta][n] for n fields (in == out
 * allowed): e.g. S = gamma_5 gamma_4 gives the coefficients of varphi-bar (Eq. laphpropg5). */
LAPH_API int laph_spin_apply(laph_ctx_t ctx, const double *S, const double *in, int n, int nv, double *out);
/* Meson functions at zero momentum (Sec. III.B, Eq. mesonfunc with trivial displacements)
 * for fields f1 = V_s a_i (entering complex conjugated) and f2 = V_s b_j:
 *   M[t][i][j] = sum_{alpha,beta} c_{alpha beta} sum_{x,colour} conj(f1_i) f2_j
 *              = sum_{alpha,beta} c_{alpha beta} sum_n conj(a_i[t][alpha][n]) b_j[t][beta][n]
 * (the sums over sites and colours reduce to the LapH index, V_s^dag V_s = 1 per slice).
 * out: device [Nt][n1][n2]; with diag = 1 (n1 == n2) only i = j: out [Nt][n1] (the
 * internal loops of same-time quark lines). */
LAPH_API int laph_meson_function(laph_ctx_t ctx, const double *c, const double *a, int n1, const double *b, int n2,
                                 int nv, int diag, double *out);
/* Meson correlator terms (Sec. III.B, Eq. mesoncorr) from meson functions, for every sink
 * slice t_F and the source slice t0, summed over the dilution indices:
 *   diag = 0: C[t_F] = - sum_{i,j} snk[t_F][i][j] conj(src[t0][i][j])  (snk, src [Nt][n1][n2])
 *   diag = 1: C[t_F] = (sum_i snk[t_F][i]) conj(sum_i src[t0][i])       (snk, src [Nt][n1])
 * (the connected term with snk = M(varphi-bar_1, varphi_2), src = M(varrho-bar_1, varrho_2);
 * the internal-line term of isoscalars with snk = M(varrho_1, varphi_1), src = M(varphi_2,
 * varrho_2)).  out: device [Nt] complex. */
LAPH_API int laph_meson_correlator(laph_ctx_t ctx, const double *snk, const double *src, int n1, int n2, int diag,
                                   int t0, double *out);

/* Covariant displacements (Sec. II, displacement types D^(j) of the quark lines
 * D^(j) S Omega^-1 S D^(k)dag; the paper's are typically 3 links along one spatial axis):
 *   (D v)(x) = U_d(x) U_d(x+e) ... U_d(x+(len-1)e) v(x+len e)             sign = +1
 *   (D v)(x) = U_d(x-e)^dag ... U_d(x-len e)^dag v(x-len e)                sign = -1
 * for n colour fields per time slice in the eigenvector layout v[((t*n + j)*Ns^3 + xyz)*3 + c]
 * (dir 0, 1, 2 = x, y, z; U in the ABI link layout, e.g. the stout-smeared field of the
 * LapH subspace).  out may not alias v. */
LAPH_API int laph_displace(laph_ctx_t ctx, const double *U, int dir, int sign, int length, const double *v, int n,
                           double *out);
/* Momentum overlaps of two sets of colour fields on every slice (the momentum projection
 * of Eq. mesonfunc): O[t][i][j] = sum_{x,c} exp(-2 pi i k.x / Ns) conj(a_i(x,c)) b_j(x,c),
 * k an integer triple (HOST int[3]); a [Nt][na][Ns^3][3], b [Nt][nb][Ns^3][3], out [Nt][na][nb].
 * With a = D^(j) V_s and b = D^(k) V_s the displaced, momentum-projected meson function
 * of fields D^(j) V_s a' and D^(k) V_s b' is exp(-i p.(d_j + d_k)/2) sum c conj(a') O b'. */
LAPH_API int laph_mom_overlap(laph_ctx_t ctx, const double *a, int na, const double *b, int nb, const int *k,
                              double *out);
/* out[r][t][beta][i] = sum_j O[t][i][j] b[r][t][beta][j] for n coefficient arrays b with nb
 * LapH vectors (O [Nt][na][nb] from laph_mom_overlap; out has na).  Followed by
 * laph_meson_function(c exp(-i p.(d_j + d_k)/2), a', ., out, ...) it gives the displaced,
 * momentum-projected meson function. */
LAPH_API int laph_overlap_apply(laph_ctx_t ctx, const double *O, int na, int nb, const double *b, int n,
                                double *out);

/* Baryon functions (Sec. III.A, Eq. baryonfunc) with the trivial displacement, from LapH
 * coefficients.  laph_baryon_tensor: the eigenvector tensor
 *   T[t][n1][n2][n3] = sum_x exp(-2 pi i k.x / Ns) eps_abc V_n1(x,a) V_n2(x,b) V_n3(x,c)
 * (totally antisymmetric), T: device [Nt][nv][nv][nv], k HOST int[3].
 * laph_baryon_function: for quark sinks varphi_k = V_s f_k (coefficients f1 [n1][Nt][4][nv],
 * f2, f3 as sink_project writes them) and a spin tensor c (HOST 4x4x4 complex,
 * c[(alpha*4 + beta)*4 + gamma]):
 *   B[t][i][j][k] = sum_{abg} c_abg sum_{n1 n2 n3} T[t][n1][n2][n3] f1_i[t][a][n1] f2_j[t][b][n2] f3_k[t][g][n3]
 * = the baryon function of Eq. baryonfunc for every dilution triple; out: device
 * [Nt][n1][n2][n3].  With quark sources (laph_quark_source coefficients) in place of the
 * sinks it gives the source functions.
 * laph_baryon_correlator: Eq. baryoncorr for three quark lines of one flavour from the sink
 * functions snk [Nt][n][n][n] and the source functions of the six noise orderings
 * src [6][Nt][n][n][n], in the order (1,2,3)+, (1,3,2)-, (2,1,3)-, (3,2,1)-, (2,3,1)+,
 * (3,1,2)+ with src[s][t][i][j][k] indexed by the dilution indices of the noises in that
 * order: C[t_F] = sum_{b1 b2 b3} snk[t_F][b1][b2][b3] conj(sum_s sign_s src[s][t0][b_s1][b_s2][b_s3]).
 * out: device [Nt] complex. */
LAPH_API int laph_baryon_tensor(laph_ctx_t ctx, const double *evecs, int nv, const int *k, double *T);
LAPH_API int laph_baryon_function(laph_ctx_t ctx, const double *T, int nv, const double *c, const double *f1, int n1,
                                  const double *f2, int n2, const double *f3, int n3, double *out);
LAPH_API int laph_baryon_correlator(laph_ctx_t ctx, const double *snk, const double *src, int n, int t0,
                                    double *out);

/* Sink projection for callers that cannot allocate or hand over a workspace (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation): the same
 * coefficients as sink_project (sums over site ranges may be grouped differently, so
 * results agree to FP64 rounding), with the partial sums in a fixed device array of
 * LAPH_SINK_NOALLOC_BYTES that each device holds from the first laph_create on it until
 * the process ends.  The call allocates nothing and needs no workspace.  Requires
 * n_rhs * Nt * 4 * nv * 16 <= LAPH_SINK_NOALLOC_BYTES (else LAPH_EINVAL, nothing
 * launched).  Every call on one device shares that array: calls that overlap on one GPU
 * (several streams or host threads) race; serialise them. */
#define LAPH_SINK_NOALLOC_BYTES (64u << 20)
LAPH_API int sink_project_noalloc(laph_ctx_t ctx, const double *evecs, int nv, const double *X, int n_rhs,
                                  double *coef);

/* ----------------------------------------------------------------- workspace
 * The library allocates no device memory.  Every call takes its device scratch, and the
 * context keeps the operator it derives from a gauge field (even-odd links, clover term
 * and inverse, their low-precision copies, the temporal-gauge field), in one workspace
 * the caller allocates and hands over with laph_set_workspace (a torch tensor, say, so
 * that PyTorch owns all device memory).  laph_workspace_bytes gives the bytes one entry
 * point needs on this context's lattice: with a workspace of at least that size the call
 * never fails for lack of room, whatever ran before (a cached operator the call does not
 * use is evicted when its room is needed; at most one is held).  A call without room
 * returns LAPH_ENOMEM and leaves its outputs undefined.  Scratch is released when a call
 * returns; the cached operator stays until another field, another set of Dirac parameters
 * or laph_set_workspace / laph_forget_gauge replaces it.  The workspace must stay valid
 * while work enqueued on the context's stream may use it.
 * Ops and the fields of laph_ws_params they read:
 *   LAPH_WS_STOUT, LAPH_WS_LAPLACIAN, LAPH_WS_CHEBYSHEV, LAPH_WS_NOISE: none (params may be NULL);
 *   LAPH_WS_EIGVECS: nv, krylov_dim;   LAPH_WS_SOURCE: nv;   LAPH_WS_SINK: nv, n (= n_rhs);
 *   LAPH_WS_DIRAC_APPLY: n (= n_fields);   LAPH_WS_HOP_APPLY: hop, n (= n_fields);
 *   LAPH_WS_SOLVE: solver, n (= n_rhs) (a learned network is taken from solver->net);
 *   LAPH_WS_AUTOTUNE: precision;   LAPH_WS_PTNET_FORWARD / _BACKWARD / _TRAIN: net, n
 *   (= n_fields or n_pairs);   LAPH_WS_MOM_OVERLAP, LAPH_WS_BARYON_TENSOR: none;
 *   LAPH_WS_BARYON_FUNCTION: nv, n, n2, n3 (the three dilution counts).  The other calls
 *   need no workspace.
 * Returns 0 for an unknown op or missing parameters. */
enum {
    LAPH_WS_STOUT = 0,
    LAPH_WS_LAPLACIAN = 1,
    LAPH_WS_CHEBYSHEV = 2,
    LAPH_WS_EIGVECS = 3,
    LAPH_WS_NOISE = 4,
    LAPH_WS_SOURCE = 5,
    LAPH_WS_DIRAC_APPLY = 6,
    LAPH_WS_HOP_APPLY = 7,
    LAPH_WS_SOLVE = 8,
    LAPH_WS_AUTOTUNE = 9,
    LAPH_WS_SINK = 10,
    LAPH_WS_PTNET_FORWARD = 11,
    LAPH_WS_PTNET_BACKWARD = 12,
    LAPH_WS_PTNET_TRAIN = 13,
    LAPH_WS_MOM_OVERLAP = 14,
    LAPH_WS_BARYON_TENSOR = 15,
    LAPH_WS_BARYON_FUNCTION = 16
};

typedef struct {
    int n;                     /* fields, right-hand sides, sources or training pairs of the call */
    int nv;                    /* LapH vectors per time slice */
    int krylov_dim;            /* eigensolver Krylov dimension m */
    int precision;             /* LAPH_PREC_* (autotuning) */
    const laph_solver *solver; /* solve parameters */
    const laph_hop *hop;       /* hopping-launch parameters */
    laph_ptnet_t net;          /* network */
    int n2, n3;                /* second and third field counts (baryon functions) */
} laph_ws_params;

LAPH_API size_t laph_workspace_bytes(laph_ctx_t ctx, int op, const void *params);
/* Hand the context its workspace: dev_ptr (256-byte aligned device memory on the
 * context's device, or NULL to release it) of `bytes` bytes.  Waits for the context's
 * stream and drops the cached operator. */
LAPH_API int laph_set_workspace(laph_ctx_t ctx, void *dev_ptr, size_t bytes);

/* ----------------------------------------------------------------- profiling
 * With timing on, the library brackets every even-odd hopping kernel launch and every
 * meson-function launch with HIP events on its stream and accumulates their durations
 * per kernel variant. */
#define LAPH_TIMING_KERNELS 8
typedef struct {
    char kernel[48];  /* kernel and variant, e.g. "dslash_lds<f16,inv>" */
    double ms;        /* summed duration of its launches */
    long launches;
    double bytes;     /* algorithmic bytes moved by those launches */
} laph_kernel_timing;

typedef struct {
    int n;  /* entries used, ordered by decreasing summed duration */
    laph_kernel_timing k[LAPH_TIMING_KERNELS];
} laph_timing;

LAPH_API int laph_set_timing(laph_ctx_t ctx, int enable);
LAPH_API int laph_get_timing(laph_ctx_t ctx, laph_timing *out, int reset);

#ifdef __cplusplus
}
#endif

#endif /* LAPH_H */

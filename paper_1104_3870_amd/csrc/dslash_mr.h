// Multi-right-hand-side low-precision hopping kernel (see dslash_mr.hip).
#pragma once

#include "cg_scal.h"
#include "dslash.h"

struct MrArgs {
    void *out;
    const void *in;
    const void *x;  // epilogue operand (same parity as out) or null
    float *out_nrm;
    const float *in_nrm;
    const float *x_nrm;
    const void *links;  // reconstruct-12 FP32 links: float4[(mu*2 + par) * Vh * 3 + i * 3 + k]
    const void *clov;   // per-site FP32 clover blocks of the output parity: float4[i * 18 + k]
    int ns, nt;
    long Vh;
    int R;
    int par;
    double a, c;
    double wt, ws, bct;
    int g5d;
    // M_INV_AFTER_DAG: second output A^-1 gamma_5 out (same parity and layout as out).
    // M_PLAIN_CG: out is not stored; for active right-hand sides cg_r -= alpha out (alpha
    // and the mask from sc[r]).  Both write partial[block * R + r] = sum over the block's
    // sites of |out_r|^2 (DAG) or |cg_r|^2 after the update (CG), from the stored values.
    void *out2;
    float *out2_nrm;
    double *partial;
    const Scal *sc;
    void *cg_r;
    float *cg_r_nrm;
    // M_INV_AFTER_DOT: the field y (same parity and layout as out); partial[(block * 3 + q)
    // * R + r] holds the block's sum of Re <y_r, out_r> (q = 0), Im (q = 1) and |out_r|^2
    // (q = 2), <y, out> = sum conj(y) out, from out as stored
    const void *dot_y;
    const float *dot_y_nrm;
    // order in which the LDS-staged kernel visits output sites: wby = 0 walks the
    // checkerboard index; otherwise spatial tiles of ns x wby x wbz sites are walked slice
    // by slice through all time slices, one tile after the other
    int wby, wbz;
    // multiply-high reciprocals of the kernel's index divisors (ns/2, ns, nt, wby,
    // ns/wby, ns/2 wby wbz): q = umulhi(n, m) is n / d for every n the kernel divides
    // (the launcher checks Vh d < 2^32); 0 stands for d = 1
    unsigned m_nsh, m_ns, m_nt, m_by, m_nty, m_A;
    // 1.0, passed at run time: a + (+-unit) b stays one mixed-precision FMA per component
    // for FP16 records instead of being folded into two conversions and an add
    float unit;
    // the links are in temporal gauge: every time-direction link except those leaving the
    // last slice is the unit matrix (applied without a product)
    int tgauge;
};

// mode: M_PLAIN (out = c D psi [+ a x]) or M_INV_AFTER (out = a x + c A^-1 D psi)
template <class SP>
void launch_dslash_mr(laph_ctx *c, int mode, const MrArgs &a, hipStream_t st);

// out = A x (gamma_5 applied to x first when g5_in); cl: per-site blocks of x's parity
template <class SP>
void launch_clover_mr(laph_ctx *c, const void *cl, const void *x, const float *x_nrm, void *out, float *out_nrm,
                      long Vh, int R, int g5_in, hipStream_t st);

// FP64 even-odd links / packed clover inverse -> the low-precision layouts above
void build_lp_operator(laph_ctx *c, const double2 *g64, const double *clinv64, float4 *links12, float *clinv_aos);

// algorithmic HBM bytes of one launch (y_is_x: the dot epilogue's y is the own-site x)
double dslash_mr_bytes(long Vh, int R, int sbytes, bool has_norm, int mode, bool has_x, bool y_is_x = false);

// sites per block of the LDS-staged hopping kernel for (precision, R); S R <= 256 lanes
int lds_tile_sites(laph_ctx *c, int prec, int R);
// largest power-of-two block R <= 32 whose records the kernel's 32-bit offsets reach on
// this lattice in this precision (0: none)
int lds_max_rhs(laph_ctx *c, int prec);
// number of partial sums per right-hand side the fused epilogues write
long lds_dag_blocks(laph_ctx *c, int prec, int R);
// whether launches walk the sites in tiles through time (else checkerboard order)
bool lds_walk_tiled(laph_ctx *c);

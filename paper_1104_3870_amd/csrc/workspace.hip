// laph_workspace_bytes: the workspace an entry point needs on this context's lattice.
#include "laph_impl.h"
#include "ptnet.h"

size_t eig_scratch_bytes(const Geom &g, int m, int nv);
size_t sink_scratch_bytes(const Geom &g, int nv, int n_rhs);
size_t source_scratch_bytes(const Geom &g, int nv);
size_t dirac_cache_bytes(const Geom &g, bool tgauge);
size_t apply_scratch_bytes(laph_ctx *c, int n_fields);
size_t hop_scratch_bytes(laph_ctx *c, const laph_hop *h, int R);
size_t tune_scratch_bytes(laph_ctx *c, int prec);
size_t solve_scratch_bytes(laph_ctx *c, int n_rhs, const laph_solver *sv);
size_t baryon_scratch_bytes(const Geom &g, int nv, int n1, int n2, int n3);

extern "C" size_t laph_workspace_bytes(laph_ctx_t c, int op, const void *params)
{
    if (!c) return 0;
    const laph_ws_params *p = (const laph_ws_params *)params;
    const Geom &g = c->g;
    const size_t field = (size_t)g.V * 36 * 16;
    try {
        switch (op) {
        case LAPH_WS_STOUT: return ws_align(field);
        case LAPH_WS_LAPLACIAN: return ws_align((size_t)27 * g.V * 16);
        case LAPH_WS_CHEBYSHEV: return ws_align((size_t)27 * g.V * 16) + 2 * ws_align((size_t)g.V * 3 * 16);
        case LAPH_WS_NOISE: return 256;
        case LAPH_WS_MOM_OVERLAP:
        case LAPH_WS_BARYON_TENSOR: return ws_align(sizeof(double2) * g.V3);
        case LAPH_WS_BARYON_FUNCTION:
            if (!p || p->nv <= 0 || p->n <= 0 || p->n2 <= 0 || p->n3 <= 0) return 0;
            return baryon_scratch_bytes(g, p->nv, p->n, p->n2, p->n3);
        case LAPH_WS_EIGVECS:
            if (!p || p->nv <= 0 || p->krylov_dim <= 0) return 0;
            return eig_scratch_bytes(g, p->krylov_dim, p->nv);
        case LAPH_WS_SOURCE:
            if (!p || p->nv <= 0) return 0;
            return source_scratch_bytes(g, p->nv);
        case LAPH_WS_SINK:
            if (!p || p->nv <= 0 || p->n <= 0) return 0;
            return sink_scratch_bytes(g, p->nv, p->n);
        case LAPH_WS_DIRAC_APPLY:
            if (!p || p->n <= 0) return 0;
            return dirac_cache_bytes(g, false) + apply_scratch_bytes(c, p->n);
        case LAPH_WS_HOP_APPLY:
            if (!p || !p->hop || p->n <= 0 || p->n > 32) return 0;
            return dirac_cache_bytes(g, p->hop->temporal_gauge != 0) + hop_scratch_bytes(c, p->hop, p->n);
        case LAPH_WS_AUTOTUNE:
            if (!p || p->precision < LAPH_PREC_F64 || p->precision > LAPH_PREC_BF16) return 0;
            return ws_align(8) + dirac_cache_bytes(g, false) + tune_scratch_bytes(c, p->precision);
        case LAPH_WS_SOLVE:
            if (!p || !p->solver || p->n <= 0) return 0;
            return dirac_cache_bytes(g, p->solver->precision != LAPH_PREC_F64) +
                   solve_scratch_bytes(c, p->n, p->solver);
        case LAPH_WS_PTNET_FORWARD:
        case LAPH_WS_PTNET_BACKWARD:
        case LAPH_WS_PTNET_TRAIN:
            if (!p || !p->net || p->n <= 0) return 0;
            return ptnet_scratch_bytes(g, p->net, p->n, op - LAPH_WS_PTNET_FORWARD);
        }
    } catch (...) {
        return 0;
    }
    return 0;
}

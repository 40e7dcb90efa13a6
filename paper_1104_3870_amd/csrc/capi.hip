// Context, errors, device buffers, timing and the host-only dilution helpers.
#include <algorithm>
#include <cctype>
#include <cstdarg>
#include <cstdlib>

#include "laph_impl.h"

thread_local laph_ctx *g_current_ctx = nullptr;

void laph_fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (g_current_ctx) g_current_ctx->err = buf;
    throw LaphError{code};
}

void *ctx_buf(laph_ctx *c, DevBuf &b, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (b.bytes >= bytes) return b.p;
    if (b.p) {
        LAPH_HIP(hipStreamSynchronize(c->stream));
        LAPH_HIP(hipFree(b.p));
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = (bytes + 4095) & ~size_t(4095);
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        laph_fail(LAPH_ENOMEM, "hipMalloc of %zu bytes failed: %s", want, hipGetErrorString(e));
    }
    b.bytes = want;
    return b.p;
}

void ctx_free(DevBuf &b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

static void free_dirac_cache(DiracCache &d)
{
    ctx_free(d.g64);
    ctx_free(d.g32);
    ctx_free(d.clov);
    ctx_free(d.clinv);
    ctx_free(d.clinv32);
    ctx_free(d.lk12);
    ctx_free(d.claos);
    ctx_free(d.gU);
    ctx_free(d.gG);
    d.valid = false;
    d.U = nullptr;
}

extern "C" int laph_create(laph_ctx_t *out, const laph_geom *geom, void *stream)
{
    if (!out || !geom) return LAPH_EINVAL;
    *out = nullptr;
    if (geom->ns < 2 || geom->nt < 2 || (geom->ns & 1) || (geom->nt & 1)) return LAPH_EINVAL;
    laph_ctx *c = new laph_ctx();
    c->g.ns = geom->ns;
    c->g.nt = geom->nt;
    c->g.V3 = (long)geom->ns * geom->ns * geom->ns;
    c->g.V = c->g.V3 * geom->nt;
    c->g.Vh = c->g.V / 2;
    c->stream = (hipStream_t)stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return LAPH_EHIP;
    }
    *out = c;
    return LAPH_OK;
}

extern "C" int laph_destroy(laph_ctx_t c)
{
    if (!c) return LAPH_EINVAL;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    free_dirac_cache(c->dc);
    free_dirac_cache(c->dct);
    for (auto &kv : c->bufs) ctx_free(kv.second);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->pin) (void)hipHostFree(c->pin);
    for (hipEvent_t e : c->pin_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &p : c->event_pool) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    for (auto &p : c->pending) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    delete c;
    return LAPH_OK;
}

extern "C" const char *laph_strerror(int s)
{
    switch (s) {
    case LAPH_OK: return "ok";
    case LAPH_EINVAL: return "invalid argument";
    case LAPH_EDIVIDE: return "dilution N/J is not an integer";
    case LAPH_ENOCONV: return "solver did not reach the requested true residual";
    case LAPH_EEIG: return "eigensolver did not converge within max_restarts";
    case LAPH_EHIP: return "HIP runtime error";
    case LAPH_ENOMEM: return "device allocation failed";
    }
    return "unknown status";
}

extern "C" const char *laph_last_error(laph_ctx_t c) { return c ? c->err.c_str() : ""; }

extern "C" int laph_forget_gauge(laph_ctx_t c)
{
    if (!c) return LAPH_EINVAL;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    free_dirac_cache(c->dc);
    free_dirac_cache(c->dct);
    return LAPH_OK;
}

extern "C" size_t laph_device_bytes(laph_ctx_t c)
{
    if (!c) return 0;
    size_t s = 0;
    for (const DiracCache *d : {&c->dc, &c->dct})
        s += d->g64.bytes + d->g32.bytes + d->clov.bytes + d->clinv.bytes + d->clinv32.bytes + d->lk12.bytes +
             d->claos.bytes + d->gU.bytes + d->gG.bytes;
    for (auto &kv : c->bufs) s += kv.second.bytes;
    return s;
}

// ----------------------------------------------------------------------- timing
void timing_begin(laph_ctx *c, hipEvent_t *a, hipEvent_t *b)
{
    if (!c->timing) {
        *a = *b = nullptr;
        return;
    }
    if (c->event_pool.empty()) {
        hipEvent_t e0, e1;
        LAPH_HIP(hipEventCreate(&e0));
        LAPH_HIP(hipEventCreate(&e1));
        c->event_pool.push_back({e0, e1});
    }
    auto p = c->event_pool.back();
    c->event_pool.pop_back();
    *a = p.first;
    *b = p.second;
    LAPH_HIP(hipEventRecord(*a, c->stream));
}

void timing_end(laph_ctx *c, hipEvent_t a, hipEvent_t b, double bytes, const char *label)
{
    if (!a) return;
    LAPH_HIP(hipEventRecord(b, c->stream));
    c->pending.push_back({a, b});
    c->pending_bytes.push_back(bytes);
    c->pending_label.push_back(label);
    if (c->pending.size() >= 512) timing_collect(c);
}

const char *timing_label(const char *kernel, const char *prec, int mode, int R)
{
    static std::map<std::string, std::string> names;
    static const char *modes[] = {"plain", "inv", "inv_of_sum", "clov_add", "inv_dag", "plain_cg"};
    char buf[96];
    snprintf(buf, sizeof(buf), "%s<%s,%s,R%d>", kernel, prec, (mode >= 0 && mode < 6) ? modes[mode] : "?", R);
    auto &v = names[buf];
    if (v.empty()) v = buf;
    return v.c_str();
}

void timing_collect(laph_ctx *c)
{
    if (c->pending.empty()) return;
    LAPH_HIP(hipEventSynchronize(c->pending.back().second));
    for (size_t k = 0; k < c->pending.size(); k++) {
        float ms = 0;
        LAPH_HIP(hipEventElapsedTime(&ms, c->pending[k].first, c->pending[k].second));
        auto &acc = c->tacc[c->pending_label[k]];
        acc.ms += ms;
        acc.launches += 1;
        acc.bytes += c->pending_bytes[k];
        c->event_pool.push_back(c->pending[k]);
    }
    c->pending.clear();
    c->pending_bytes.clear();
    c->pending_label.clear();
}

extern "C" int laph_set_timing(laph_ctx_t c, int enable)
{
    if (!c) return LAPH_EINVAL;
    g_current_ctx = c;
    try {
        timing_collect(c);
    } catch (const LaphError &e) {
        return e.code;
    }
    c->timing = enable != 0;
    return LAPH_OK;
}

extern "C" int laph_get_timing(laph_ctx_t c, laph_timing *out, int reset)
{
    if (!c || !out) return LAPH_EINVAL;
    g_current_ctx = c;
    try {
        LAPH_HIP(hipSetDevice(c->device));
        timing_collect(c);
    } catch (const LaphError &e) {
        return e.code;
    }
    std::vector<std::pair<std::string, laph_ctx::TimeAcc>> v(c->tacc.begin(), c->tacc.end());
    std::sort(v.begin(), v.end(), [](const auto &a, const auto &b) { return a.second.ms > b.second.ms; });
    memset(out, 0, sizeof(*out));
    out->n = (int)std::min<size_t>(v.size(), LAPH_TIMING_KERNELS);
    for (int k = 0; k < out->n; k++) {
        snprintf(out->k[k].kernel, sizeof(out->k[k].kernel), "%s", v[k].first.c_str());
        out->k[k].ms = v[k].second.ms;
        out->k[k].launches = v[k].second.launches;
        out->k[k].bytes = v[k].second.bytes;
    }
    if (reset) c->tacc.clear();
    return LAPH_OK;
}

// ------------------------------------------------------------ dilution (host)
// Sec. II: "1" (no dilution), "F" (full), "BJ" (block-J), "IJ" (interlace-J) for time,
// spin and LapH index; N/J must be an integer.
static int dil_count1(int type, int J, int N)
{
    switch (type) {
    case LAPH_DIL_NONE: return 1;
    case LAPH_DIL_FULL: return N;
    case LAPH_DIL_BLOCK:
    case LAPH_DIL_INTERLACE: return (J > 0 && N % J == 0) ? J : -1;
    }
    return -1;
}

extern "C" long laph_dilution_count(const laph_dilution *d, int nt, int nv)
{
    if (!d || nt <= 0 || nv <= 0) return -1;
    int N[3] = {nt, 4, nv};
    long n = 1;
    for (int k = 0; k < 3; k++) {
        int c = dil_count1(d->type[k], d->J[k], N[k]);
        if (c <= 0) return -1;
        n *= c;
    }
    return n;
}

extern "C" int laph_parse_dilution(const char *text, int nt, int nv, laph_dilution *out)
{
    if (!text || !out || nt <= 0 || nv <= 0) return LAPH_EINVAL;
    std::string s;
    for (const char *p = text; *p; p++)
        if (!isspace((unsigned char)*p) && *p != '(' && *p != ')') s += (char)toupper((unsigned char)*p);
    const char want[3] = {'T', 'S', 'L'};
    int N[3] = {nt, 4, nv};
    size_t pos = 0;
    for (int k = 0; k < 3; k++) {
        size_t end = s.find(',', pos);
        if (k < 2 && end == std::string::npos) return LAPH_EINVAL;
        if (k == 2) {
            if (end != std::string::npos) return LAPH_EINVAL;
            end = s.size();
        }
        std::string tok = s.substr(pos, end - pos);
        pos = end + 1;
        if (tok.size() < 2 || tok[0] != want[k]) return LAPH_EINVAL;
        std::string body = tok.substr(1);
        if (body == "1") {
            out->type[k] = LAPH_DIL_NONE;
            out->J[k] = 0;
        } else if (body == "F") {
            out->type[k] = LAPH_DIL_FULL;
            out->J[k] = 0;
        } else if ((body[0] == 'B' || body[0] == 'I') && body.size() > 1) {
            for (size_t q = 1; q < body.size(); q++)
                if (!isdigit((unsigned char)body[q])) return LAPH_EINVAL;
            long J = strtol(body.c_str() + 1, nullptr, 10);
            if (J <= 0 || J > N[k]) return (J > N[k]) ? LAPH_EDIVIDE : LAPH_EINVAL;
            if (N[k] % J != 0) return LAPH_EDIVIDE;
            out->type[k] = body[0] == 'B' ? LAPH_DIL_BLOCK : LAPH_DIL_INTERLACE;
            out->J[k] = (int)J;
        } else {
            return LAPH_EINVAL;
        }
    }
    return LAPH_OK;
}

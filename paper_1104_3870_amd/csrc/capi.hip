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

// ------------------------------------------------------------------ workspace
void *ctx_named(laph_ctx *c, const std::string &name, size_t bytes)
{
    DevBuf &b = c->bufs[name];
    if (bytes == 0) bytes = 256;
    if (b.bytes >= bytes) return b.p;
    // a grown buffer takes a new piece (the old one stays until the call returns)
    const size_t want = ws_align(bytes);
    if (c->ws && c->ws_lo + want + c->ws_hi > c->ws_bytes && c->ws_unit && !c->ws_pinned) cache_release_all(c);
    if (!c->ws || c->ws_lo + want + c->ws_hi > c->ws_bytes)
        laph_fail(LAPH_ENOMEM, "workspace of %zu bytes has no room for %zu more bytes (%s; scratch %zu, cached "
                  "operator %zu): size it with laph_workspace_bytes",
                  c->ws_bytes, want, name.c_str(), c->ws_lo, c->ws_hi);
    b.p = c->ws + c->ws_lo;
    b.bytes = want;
    c->ws_lo += want;
    return b.p;
}

void scratch_reset(laph_ctx *c)
{
    c->bufs.clear();
    c->ws_lo = 0;
    c->ws_pinned = false;
}

static void invalidate(DiracCache &d)
{
    d.valid = false;
    d.f32 = false;
    d.U = nullptr;
    d.fp = 0;
    d.unit = DevBuf{};
    d.g64 = d.clov = d.clinv = d.lk12 = d.claos = d.gU = d.gG = DevBuf{};
    d.has_f32 = false;
}

void cache_release_all(laph_ctx *c)
{
    if (c->ws_unit) invalidate(*c->ws_unit);
    c->ws_unit = nullptr;
    c->ws_hi = 0;
    c->ws_pinned = false;
}

void cache_unit(laph_ctx *c, DiracCache &dc, size_t bytes)
{
    bytes = ws_align(bytes);
    if (c->ws_unit == &dc && dc.unit.bytes >= bytes) {
        c->ws_pinned = true;
        return;
    }
    cache_release_all(c);
    if (!c->ws || c->ws_lo + bytes > c->ws_bytes)
        laph_fail(LAPH_ENOMEM, "workspace of %zu bytes has no room for a cached operator of %zu bytes: size it "
                  "with laph_workspace_bytes", c->ws_bytes, bytes);
    c->ws_hi = bytes;
    dc.unit.p = c->ws + (c->ws_bytes - bytes);
    dc.unit.bytes = bytes;
    c->ws_unit = &dc;
    c->ws_pinned = true;
}

// fields of a cache unit, in order
static void unit_layout(const Geom &g, bool tgauge, bool f32, size_t (&sz)[7])
{
    const long Vh = g.Vh, V = g.V;
    sz[0] = (size_t)72 * Vh * 16;                 // g64
    sz[1] = (size_t)144 * Vh * 8;                 // clov
    sz[2] = (size_t)144 * Vh * 8;                 // clinv
    sz[3] = f32 ? (size_t)8 * Vh * 3 * 16 : 0;    // lk12
    sz[4] = f32 ? (size_t)2 * Vh * 72 * 4 : 0;    // claos
    sz[5] = tgauge ? (size_t)V * 36 * 16 : 0;     // gU
    sz[6] = tgauge ? (size_t)V * 9 * 16 : 0;      // gG
}

size_t cache_unit_bytes(const Geom &g, bool tgauge, bool f32)
{
    size_t sz[7], s = 0;
    unit_layout(g, tgauge, f32, sz);
    for (size_t v : sz) s += ws_align(v);
    return s;
}

void cache_carve(laph_ctx *c, DiracCache &dc, bool tgauge, bool f32)
{
    size_t sz[7];
    unit_layout(c->g, tgauge, f32, sz);
    DevBuf *f[7] = {&dc.g64, &dc.clov, &dc.clinv, &dc.lk12, &dc.claos, &dc.gU, &dc.gG};
    char *p = (char *)dc.unit.p;
    for (int k = 0; k < 7; k++) {
        f[k]->p = sz[k] ? p : nullptr;
        f[k]->bytes = sz[k];
        p += ws_align(sz[k]);
    }
    dc.has_f32 = f32;
}

// sum over the field's 64-bit words of a mixed (word, index) hash, wrapping: equal for
// equal contents, different with overwhelming probability otherwise
__global__ void k_fingerprint(const unsigned long long *__restrict__ w, long n, unsigned long long *out)
{
    unsigned long long acc = 0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        unsigned long long z = w[i] + 0x9E3779B97F4A7C15ull * (unsigned long long)(i + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        acc += z ^ (z >> 31);
    }
    __shared__ unsigned long long red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(out, red[0]);
}

uint64_t gauge_fingerprint(laph_ctx *c, const double *U)
{
    unsigned long long *d = (unsigned long long *)ctx_named(c, "fp.sum", 8);
    LAPH_HIP(hipMemsetAsync(d, 0, 8, c->stream));
    const long n = c->g.V * 4 * 9 * 2;
    hipLaunchKernelGGL(k_fingerprint, dim3(1024), dim3(256), 0, c->stream, (const unsigned long long *)U, n, d);
    LAPH_HIP(hipGetLastError());
    unsigned long long h = 0;
    LAPH_HIP(hipMemcpyAsync(&h, d, 8, hipMemcpyDeviceToHost, c->stream));
    LAPH_HIP(hipStreamSynchronize(c->stream));
    return h;
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
    try {
        g_current_ctx = c;
        sink_scratch_init(c);
    } catch (const LaphError &e) {
        g_current_ctx = nullptr;
        delete c;
        return e.code;
    }
    g_current_ctx = nullptr;
    *out = c;
    return LAPH_OK;
}

extern "C" int laph_destroy(laph_ctx_t c)
{
    if (!c) return LAPH_EINVAL;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    cache_release_all(c);
    scratch_reset(c);
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
    case LAPH_ENOMEM: return "workspace too small";
    }
    return "unknown status";
}

extern "C" const char *laph_last_error(laph_ctx_t c) { return c ? c->err.c_str() : ""; }

extern "C" int laph_forget_gauge(laph_ctx_t c)
{
    if (!c) return LAPH_EINVAL;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    cache_release_all(c);
    return LAPH_OK;
}

extern "C" size_t laph_device_bytes(laph_ctx_t c)
{
    if (!c) return 0;
    return c->ws_hi + c->ws_lo;
}

extern "C" int laph_set_workspace(laph_ctx_t c, void *dev_ptr, size_t bytes)
{
    if (!c) return LAPH_EINVAL;
    if (!dev_ptr && bytes) return LAPH_EINVAL;
    if (((uintptr_t)dev_ptr & 255) != 0) return LAPH_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LAPH_EHIP;
    // nothing queued may still use the old workspace
    if (hipStreamSynchronize(c->stream) != hipSuccess) return LAPH_EHIP;
    cache_release_all(c);
    scratch_reset(c);
    c->ws = (char *)dev_ptr;
    c->ws_bytes = dev_ptr ? bytes & ~size_t(255) : 0;  // every piece stays 256-byte aligned
    return LAPH_OK;
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
    static const char *modes[] = {"plain", "inv", "inv_of_sum", "clov_add", "inv_dag", "plain_cg", "inv_dot"};
    char buf[96];
    snprintf(buf, sizeof(buf), "%s<%s,%s,R%d>", kernel, prec, (mode >= 0 && mode < 7) ? modes[mode] : "?", R);
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

// Gauge-equivariant parallel-transport network used as a learned preconditioner of the
// even-odd Dirac solve: layer forward, adjoint backward, weight gradients, Adam, and the
// C-ABI around them.
//
// A layer maps C_in FP32 spinor fields to C_out fields,
//   out_c(x) = sum_{c', d} W[c][c'][d] (T_d phi_c')(x),   d = 0 (self), 1..4 (+mu), 5..8 (-mu),
//   T_{+mu} phi(x) = U_mu(x) phi(x+mu),  T_{-mu} phi(x) = U_mu(x-mu)^dag phi(x-mu),
// with W[c][c'][d] a complex 4x4 spin matrix held in BF16 and every hop across the time
// boundary multiplied by the fermion boundary factor.  Spin-only weights and colour-only
// transports make each layer gauge equivariant.  One thread owns one site of one field:
// the nine transports of every input channel are formed in registers and mixed into the
// C_out accumulators with weights broadcast from LDS.
#include <cmath>
#include <random>

#include "ptnet.h"

namespace {

constexpr int kPtBS = 256;

__device__ __forceinline__ float bf_lo(uint32_t u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float bf_hi(uint32_t u) { return __uint_as_float(u & 0xffff0000u); }

// FP32 -> BF16 with round-to-nearest-even (finite inputs)
__host__ __device__ inline uint32_t f2bf(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__host__ __device__ inline uint32_t pack_bf(float re, float im) { return f2bf(re) | (f2bf(im) << 16); }

__device__ __forceinline__ void lex_coords(long s, int ns, int &x, int &y, int &z, int &t)
{
    x = (int)(s % ns);
    long q = s / ns;
    y = (int)(q % ns);
    q /= ns;
    z = (int)(q % ns);
    t = (int)(q / ns);
}

// Transport matrix of direction d at site (x,y,z,t): the neighbour whose field is
// transported and the 3x3 colour matrix (boundary factor folded in); d = 0 gives the
// identity.
__device__ __forceinline__ long pt_hop(const float2 *__restrict__ links, long s, int d, int x, int y, int z, int t,
                                       int ns, int nt, float bct, Cx<float> L[9])
{
    if (d == 0) {
#pragma unroll
        for (int k = 0; k < 9; k++) L[k] = Cx<float>{(k % 4 == 0) ? 1.f : 0.f, 0.f};
        return s;
    }
    const int mu = (d - 1) & 3;
    const int sg = d <= 4 ? 1 : -1;
    float ph = 1.f;
    int xx = x, yy = y, zz = z, tt = t;
    switch (mu) {
    case 0: xx = (x + sg + ns) % ns; break;
    case 1: yy = (y + sg + ns) % ns; break;
    case 2: zz = (z + sg + ns) % ns; break;
    default:
        tt = t + sg;
        if (tt == nt) {
            tt = 0;
            ph = bct;
        } else if (tt < 0) {
            tt = nt - 1;
            ph = bct;
        }
    }
    long nb = lex_index(xx, yy, zz, tt, ns);
    if (d <= 4) {
        const float2 *u = links + (s * 4 + mu) * 9;
#pragma unroll
        for (int k = 0; k < 9; k++) {
            float2 v = u[k];
            L[k] = Cx<float>{ph * v.x, ph * v.y};
        }
    } else {
        const float2 *u = links + (nb * 4 + mu) * 9;
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) {
                float2 v = u[b * 3 + a];
                L[a * 3 + b] = Cx<float>{ph * v.x, -ph * v.y};
            }
    }
    return nb;
}

__device__ __forceinline__ void ld12(const float2 *__restrict__ p, Cx<float> v[12])
{
    const float4 *q = (const float4 *)p;
#pragma unroll
    for (int k = 0; k < 6; k++) {
        float4 a = q[k];
        v[2 * k] = Cx<float>{a.x, a.y};
        v[2 * k + 1] = Cx<float>{a.z, a.w};
    }
}
__device__ __forceinline__ void st12(float2 *__restrict__ p, const Cx<float> v[12])
{
    float4 *q = (float4 *)p;
#pragma unroll
    for (int k = 0; k < 6; k++) q[k] = make_float4(v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im);
}

// tv = L phi (colour matrix on each spin component)
__device__ __forceinline__ void transport(const Cx<float> L[9], const Cx<float> phi[12], Cx<float> tv[12])
{
#pragma unroll
    for (int sp = 0; sp < 4; sp++)
#pragma unroll
        for (int a = 0; a < 3; a++)
            tv[sp * 3 + a] = L[a * 3] * phi[sp * 3] + L[a * 3 + 1] * phi[sp * 3 + 1] + L[a * 3 + 2] * phi[sp * 3 + 2];
}

// One layer: out[r][co][s] = sum_{ci,d} W[co][ci][d] (T_d in[r][ci])(s).  Weights: BF16 pairs
// [CO][cin][9][16], staged in LDS as FP32.
template <int CO>
__global__ __launch_bounds__(kPtBS) void k_pt_layer(const float2 *__restrict__ links, const float2 *__restrict__ in,
                                                     float2 *__restrict__ out, const uint32_t *__restrict__ w,
                                                     int cin, int ns, int nt, long V, float bct)
{
    extern __shared__ float2 sw[];
    const int nwl = CO * cin * 144;
    for (int i = threadIdx.x; i < nwl; i += blockDim.x) {
        uint32_t u = w[i];
        sw[i] = make_float2(bf_lo(u), bf_hi(u));
    }
    __syncthreads();
    long s = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= V) return;
    int x, y, z, t;
    lex_coords(s, ns, x, y, z, t);
    const float2 *inr = in + (size_t)r * cin * V * 12;
    Cx<float> acc[CO][12];
#pragma unroll
    for (int co = 0; co < CO; co++)
#pragma unroll
        for (int k = 0; k < 12; k++) acc[co][k] = Cx<float>{0.f, 0.f};
    for (int d = 0; d < 9; d++) {
        Cx<float> L[9];
        long nb = pt_hop(links, s, d, x, y, z, t, ns, nt, bct, L);
        for (int ci = 0; ci < cin; ci++) {
            Cx<float> phi[12], tv[12];
            ld12(inr + ((size_t)ci * V + nb) * 12, phi);
            transport(L, phi, tv);
            const float2 *wp = sw + (ci * 9 + d) * 16;
#pragma unroll
            for (int co = 0; co < CO; co++)
#pragma unroll
                for (int sa = 0; sa < 4; sa++)
#pragma unroll
                    for (int sb = 0; sb < 4; sb++) {
                        float2 wv = wp[co * cin * 144 + sa * 4 + sb];
                        Cx<float> wc{wv.x, wv.y};
#pragma unroll
                        for (int a = 0; a < 3; a++) acc[co][sa * 3 + a] = acc[co][sa * 3 + a] + wc * tv[sb * 3 + a];
                    }
        }
    }
#pragma unroll
    for (int co = 0; co < CO; co++) st12(out + ((size_t)(r * CO + co) * V + s) * 12, acc[co]);
}

// Partial weight gradients of one (ci, d) pair per blockIdx.y over a chunk of (field, site)
// items: p[co][sa][sb] = sum g[co](x)[sa][c] conj((T_d act[ci])(x)[sb][c]).
template <int CO>
__global__ __launch_bounds__(kPtBS) void k_pt_wgrad(const float2 *__restrict__ links, const float2 *__restrict__ act,
                                                     const float2 *__restrict__ g, float2 *__restrict__ gpart,
                                                     int cin, int ns, int nt, long V, int R, float bct, long chunk)
{
    const int ci = blockIdx.y / 9, d = blockIdx.y % 9;
    const long n = V * R;
    const long beg = blockIdx.x * chunk;
    const long end = beg + chunk < n ? beg + chunk : n;
    Cx<float> p[CO][16];
#pragma unroll
    for (int co = 0; co < CO; co++)
#pragma unroll
        for (int e = 0; e < 16; e++) p[co][e] = Cx<float>{0.f, 0.f};
    for (long it = beg + threadIdx.x; it < end; it += blockDim.x) {
        int r = (int)(it / V);
        long s = it - (long)r * V;
        int x, y, z, t;
        lex_coords(s, ns, x, y, z, t);
        Cx<float> L[9], phi[12], tv[12];
        long nb = pt_hop(links, s, d, x, y, z, t, ns, nt, bct, L);
        ld12(act + (((size_t)r * cin + ci) * V + nb) * 12, phi);
        transport(L, phi, tv);
#pragma unroll
        for (int co = 0; co < CO; co++) {
            Cx<float> gg[12];
            ld12(g + (((size_t)r * CO + co) * V + s) * 12, gg);
#pragma unroll
            for (int sa = 0; sa < 4; sa++)
#pragma unroll
                for (int sb = 0; sb < 4; sb++) {
                    Cx<float> acc = p[co][sa * 4 + sb];
#pragma unroll
                    for (int a = 0; a < 3; a++) acc = acc + gg[sa * 3 + a] * Cx<float>{tv[sb * 3 + a].re, -tv[sb * 3 + a].im};
                    p[co][sa * 4 + sb] = acc;
                }
        }
    }
    __shared__ float2 red[kPtBS / 64][CO * 16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int co = 0; co < CO; co++)
#pragma unroll
        for (int e = 0; e < 16; e++) {
            float re = p[co][e].re, im = p[co][e].im;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                re += __shfl_xor(re, off);
                im += __shfl_xor(im, off);
            }
            if (lane == 0) red[wv][co * 16 + e] = make_float2(re, im);
        }
    __syncthreads();
    const size_t nwl = (size_t)CO * cin * 144;
    for (int j = threadIdx.x; j < CO * 16; j += blockDim.x) {
        float2 sum = red[0][j];
        for (int q = 1; q < kPtBS / 64; q++) {
            sum.x += red[q][j].x;
            sum.y += red[q][j].y;
        }
        int co = j >> 4, e = j & 15;
        gpart[blockIdx.x * nwl + ((size_t)(co * cin + ci) * 9 + d) * 16 + e] = sum;
    }
}

__global__ void k_pt_sum_parts(const float2 *__restrict__ gpart, float2 *__restrict__ grad, int nblk, long nwl)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= nwl) return;
    float2 s = gpart[i];
    for (int b = 1; b < nblk; b++) {
        s.x += gpart[b * nwl + i].x;
        s.y += gpart[b * nwl + i].y;
    }
    grad[i] = s;
}

// Wa[ci][co][d'] = W[co][ci][rev(d')]^dag, rev swapping +mu and -mu: the layer whose action
// is the adjoint of the forward layer (T_d^dag = T_rev(d)).
__global__ void k_pt_adjoint(const uint32_t *__restrict__ w, uint32_t *__restrict__ wa, int cout, int cin)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cout * cin * 144) return;
    int e = i % 16, q = i / 16;
    int dp = q % 9;
    q /= 9;
    int co = q % cout, ci = q / cout;  // output layout [ci][co][9][16]
    int sa = e >> 2, sb = e & 3;
    int d = dp == 0 ? 0 : (dp <= 4 ? dp + 4 : dp - 4);
    uint32_t u = w[((co * cin + ci) * 9 + d) * 16 + sb * 4 + sa];
    wa[i] = u ^ 0x80000000u;  // conjugate: flip the sign of the imaginary BF16
}

__global__ void k_pt_adam(float2 *__restrict__ w, uint32_t *__restrict__ wbf, float2 *__restrict__ m1,
                          float2 *__restrict__ m2, const float2 *__restrict__ grad, long n, float lr, float b1,
                          float b2, float eps, float bc1, float bc2)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    // real-parameter gradient of a real loss: d/dRe W + i d/dIm W = 2 dL/dW^*
    float2 g = make_float2(2.f * grad[i].x, 2.f * grad[i].y);
    float2 m = m1[i], v = m2[i], x = w[i];
    m.x = b1 * m.x + (1.f - b1) * g.x;
    m.y = b1 * m.y + (1.f - b1) * g.y;
    v.x = b2 * v.x + (1.f - b2) * g.x * g.x;
    v.y = b2 * v.y + (1.f - b2) * g.y * g.y;
    x.x -= lr * (m.x / bc1) / (sqrtf(v.x / bc2) + eps);
    x.y -= lr * (m.y / bc1) / (sqrtf(v.y / bc2) + eps);
    m1[i] = m;
    m2[i] = v;
    w[i] = x;
    wbf[i] = pack_bf(x.x, x.y);
}

__global__ void k_pt_from64(const double2 *__restrict__ a, float2 *__restrict__ b, long n)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) b[i] = make_float2((float)a[i].x, (float)a[i].y);
}
__global__ void k_pt_to64(const float2 *__restrict__ a, double2 *__restrict__ b, long n)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) b[i] = make_double2(a[i].x, a[i].y);
}

__global__ void k_eo_to_net(const double2 *__restrict__ half, int par, float2 *__restrict__ full, int ns, long V,
                            long Vh)
{
    long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (tid >= V * 12) return;
    long s = tid / 12;
    int k = (int)(tid - s * 12);
    int x, y, z, t;
    lex_coords(s, ns, x, y, z, t);
    float2 v = make_float2(0.f, 0.f);
    if (((x + y + z + t) & 1) == par) {
        double2 h = half[(long)k * Vh + (s >> 1)];
        v = make_float2((float)h.x, (float)h.y);
    }
    full[tid] = v;
}

__global__ void k_net_to_eo(const float2 *__restrict__ full, int par, double2 *__restrict__ half, int ns, long Vh)
{
    long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (tid >= Vh * 12) return;
    int k = (int)(tid / Vh);
    long i = tid - (long)k * Vh;
    int x, y, z, t;
    cb_coords(i, par, ns, x, y, z, t);
    long s = lex_index(x, y, z, t, ns);
    float2 v = full[s * 12 + k];
    half[tid] = make_double2(v.x, v.y);
}

// per-block partial sums over the sites of one field (parity mask: -1 all, 0 even, 1 odd)
//   part_x2[r][b] = sum |x|^2,  with out != null also
//   part_l[r][b]  = sum |out - x|^2 and g = mask (out - x) * inv_x2[r]
__global__ void k_pt_loss(const float2 *__restrict__ out, const double2 *__restrict__ x, const double *__restrict__ inv_x2,
                          float2 *__restrict__ g, double *__restrict__ part, int ns, long V, int par, long chunk)
{
    const int r = blockIdx.y;
    const long beg = blockIdx.x * chunk;
    const long end = beg + chunk < V ? beg + chunk : V;
    double acc = 0;
    for (long s = beg + threadIdx.x; s < end; s += blockDim.x) {
        int xx, y, z, t;
        lex_coords(s, ns, xx, y, z, t);
        bool on = par < 0 || ((xx + y + z + t) & 1) == par;
        const double2 *xs = x + ((size_t)r * V + s) * 12;
        if (out) {
            const float2 *os = out + ((size_t)r * V + s) * 12;
            float2 *gs = g + ((size_t)r * V + s) * 12;
            double sc = inv_x2[r];
            for (int k = 0; k < 12; k++) {
                double dr = on ? (double)os[k].x - xs[k].x : 0.0;
                double di = on ? (double)os[k].y - xs[k].y : 0.0;
                acc += dr * dr + di * di;
                gs[k] = make_float2((float)(dr * sc), (float)(di * sc));
            }
        } else if (on) {
            for (int k = 0; k < 12; k++) acc += xs[k].x * xs[k].x + xs[k].y * xs[k].y;
        }
    }
    __shared__ double red[kPtBS];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kPtBS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)r * gridDim.x + blockIdx.x] = red[0];
}

template <int CO>
void launch_layer_t(laph_ctx *c, const float2 *links, const float2 *in, float2 *out, const uint32_t *w, int cin,
                    int nrhs, float bct)
{
    long V = c->g.V;
    size_t lds = (size_t)CO * cin * 144 * sizeof(float2);
    hipLaunchKernelGGL(k_pt_layer<CO>, dim3(nblocks_for(V, kPtBS), nrhs), dim3(kPtBS), lds, c->stream, links, in,
                       out, w, cin, c->g.ns, c->g.nt, V, bct);
    LAPH_HIP(hipGetLastError());
}

void launch_layer(laph_ctx *c, const float2 *links, const float2 *in, float2 *out, const uint32_t *w, int cin,
                  int cout, int nrhs, float bct)
{
    switch (cout) {
    case 1: launch_layer_t<1>(c, links, in, out, w, cin, nrhs, bct); break;
    case 2: launch_layer_t<2>(c, links, in, out, w, cin, nrhs, bct); break;
    case 4: launch_layer_t<4>(c, links, in, out, w, cin, nrhs, bct); break;
    default: laph_fail(LAPH_EINVAL, "unsupported channel count %d", cout);
    }
}

template <int CO>
void launch_wgrad_t(laph_ctx *c, laph_ptnet *net, const float2 *act, const float2 *g, int cin, int nrhs, float bct,
                    float2 *grad)
{
    long V = c->g.V;
    long n = V * nrhs;
    // a few thousand items per block keep the block reduction cheap; at most 256 blocks
    long chunk = std::max<long>(kPtBS * 8, (n + 255) / 256);
    chunk = (chunk + kPtBS - 1) / kPtBS * kPtBS;
    int nblk = (int)((n + chunk - 1) / chunk);
    long nwl = (long)CO * cin * 144;
    float2 *gpart = (float2 *)ctx_named(c, "net.gpart", sizeof(float2) * nwl * nblk);
    hipLaunchKernelGGL(k_pt_wgrad<CO>, dim3(nblk, cin * 9), dim3(kPtBS), 0, c->stream, net->links,
                       act, g, gpart, cin, c->g.ns, c->g.nt, V, nrhs, bct, chunk);
    LAPH_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_pt_sum_parts, dim3(nblocks_for(nwl, 256)), dim3(256), 0, c->stream, (const float2 *)gpart,
                       grad, nblk, nwl);
    LAPH_HIP(hipGetLastError());
}

void launch_wgrad(laph_ctx *c, laph_ptnet *net, const float2 *act, const float2 *g, int cin, int cout, int nrhs,
                  float bct, float2 *grad)
{
    switch (cout) {
    case 1: launch_wgrad_t<1>(c, net, act, g, cin, nrhs, bct, grad); break;
    case 2: launch_wgrad_t<2>(c, net, act, g, cin, nrhs, bct, grad); break;
    case 4: launch_wgrad_t<4>(c, net, act, g, cin, nrhs, bct, grad); break;
    default: laph_fail(LAPH_EINVAL, "unsupported channel count %d", cout);
    }
}

void check_net(laph_ctx *c, laph_ptnet *net)
{
    LAPH_CHECK(net && net->layers > 0, LAPH_EINVAL, "null or empty network");
    LAPH_CHECK(net->device == c->device, LAPH_EINVAL, "network lives on device %d, context on %d", net->device,
               c->device);
}

}  // namespace

// ---------------------------------------------------------------- internal API
void ptnet_prepare(laph_ctx *c, laph_ptnet *net, const double *U)
{
    // links rebuilt on every call: a caller may free a field and allocate the next one at
    // the same address, so the pointer does not identify the field
    long V = c->g.V;
    float2 *lk = (float2 *)ctx_named(c, "net.links", sizeof(float2) * V * 36);
    hipLaunchKernelGGL(k_pt_from64, dim3(nblocks_for(V * 36, 256)), dim3(256), 0, c->stream, (const double2 *)U, lk,
                       V * 36);
    LAPH_HIP(hipGetLastError());
    net->links = lk;
    net->wbf_h.resize(net->nw);
    for (size_t i = 0; i < net->nw; i++) net->wbf_h[i] = pack_bf(net->w32[2 * i], net->w32[2 * i + 1]);
    uint32_t *wbf = (uint32_t *)ctx_named(c, "net.wbf", sizeof(uint32_t) * net->nw);
    LAPH_HIP(hipMemcpyAsync(wbf, net->wbf_h.data(), sizeof(uint32_t) * net->nw, hipMemcpyHostToDevice, c->stream));
    net->wbf = wbf;
}

void ptnet_forward(laph_ctx *c, laph_ptnet *net, float bct, const float2 *in, float2 *out, int nrhs, int keep)
{
    size_t fb = sizeof(float2) * 12 * c->g.V * nrhs;  // one channel of the batch
    const float2 *cur = in;
    if (keep) {
        net->acts.assign(net->layers, nullptr);
        net->act0 = in;
    }
    for (int l = 0; l < net->layers; l++) {
        int ci = net->ch[l], co = net->ch[l + 1];
        float2 *dst;
        if (l == net->layers - 1)
            dst = out;
        else if (keep)
            dst = (float2 *)ctx_named(c, "net.act" + std::to_string(l + 1), fb * co);
        else
            dst = (float2 *)ctx_named(c, std::string("net.tmp") + ((l & 1) ? "1" : "0"), fb * net->cmax);
        if (keep && l + 1 < net->layers) net->acts[l + 1] = dst;
        launch_layer(c, net->links, cur, dst, net->wbf + net->woff[l], ci, co, nrhs, bct);
        cur = dst;
    }
}

void ptnet_backward(laph_ctx *c, laph_ptnet *net, float bct, const float2 *g, float2 *gin, int nrhs)
{
    size_t fb = sizeof(float2) * 12 * c->g.V * nrhs;
    net->grad = (float2 *)ctx_named(c, "net.grad", sizeof(float2) * net->nw);
    const float2 *cur = g;
    for (int l = net->layers - 1; l >= 0; l--) {
        int ci = net->ch[l], co = net->ch[l + 1];
        const float2 *act = l == 0 ? net->act0 : net->acts[l];
        launch_wgrad(c, net, act, cur, ci, co, nrhs, bct, net->grad + net->woff[l]);
        if (l == 0 && !gin) break;
        uint32_t *wa = (uint32_t *)ctx_named(c, "net.wadj", sizeof(uint32_t) * net->cmax * net->cmax * 144);
        hipLaunchKernelGGL(k_pt_adjoint, dim3(nblocks_for(co * ci * 144, 256)), dim3(256), 0, c->stream,
                           net->wbf + net->woff[l], wa, co, ci);
        LAPH_HIP(hipGetLastError());
        float2 *dst = l == 0 ? gin : (float2 *)ctx_named(c, std::string("net.tmp") + ((l & 1) ? "1" : "0"),
                                                          fb * net->cmax);
        launch_layer(c, net->links, cur, dst, wa, co, ci, nrhs, bct);
        cur = dst;
    }
}

void eo_to_net(laph_ctx *c, const double2 *half, int par, float2 *full)
{
    long n = c->g.V * 12;
    hipLaunchKernelGGL(k_eo_to_net, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, half, par, full, c->g.ns,
                       c->g.V, c->g.Vh);
    LAPH_HIP(hipGetLastError());
}

void net_to_eo(laph_ctx *c, const float2 *full, int par, double2 *half)
{
    long n = c->g.Vh * 12;
    hipLaunchKernelGGL(k_net_to_eo, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, full, par, half, c->g.ns,
                       c->g.Vh);
    LAPH_HIP(hipGetLastError());
}

// gamma_4 eta for R canonical FP64 fields -> net layout (one channel); gamma_4 swaps the
// upper and lower spin pairs (chiral basis)
__global__ void k_g4_to_net(const double2 *__restrict__ eta, float2 *__restrict__ out, long n)
{
    long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (tid >= n) return;
    long s = tid / 12;
    int k = (int)(tid - s * 12);
    double2 v = eta[s * 12 + ((k / 3) ^ 2) * 3 + k % 3];
    out[tid] = make_float2((float)v.x, (float)v.y);
}

// half[(k*Vh + i)*R + r] = full[r][site(i, par)][k]
__global__ void k_net_to_eo_batch(const float2 *__restrict__ full, double2 *__restrict__ half, int par, int ns,
                                  long V, long Vh, int R)
{
    long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (tid >= 12 * Vh * R) return;
    int k = (int)(tid / (Vh * R));
    long rem = tid - (long)k * Vh * R;
    long i = rem / R;
    int r = (int)(rem - i * R);
    int x, y, z, t;
    cb_coords(i, par, ns, x, y, z, t);
    float2 v = full[((long)r * V + lex_index(x, y, z, t, ns)) * 12 + k];
    half[tid] = make_double2(v.x, v.y);
}

void ptnet_initial_guess(laph_ctx *c, laph_ptnet *net, float bct, const double *eta, int R, double2 *xo)
{
    long V = c->g.V, n = V * 12 * R;
    float2 *a = (float2 *)ctx_named(c, "net.x0in", sizeof(float2) * n);
    float2 *b = (float2 *)ctx_named(c, "net.x0out", sizeof(float2) * n);
    hipLaunchKernelGGL(k_g4_to_net, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, (const double2 *)eta, a, n);
    LAPH_HIP(hipGetLastError());
    ptnet_forward(c, net, bct, a, b, R, 0);
    long m = 12 * c->g.Vh * R;
    hipLaunchKernelGGL(k_net_to_eo_batch, dim3(nblocks_for(m, 256)), dim3(256), 0, c->stream, (const float2 *)b, xo,
                       1, c->g.ns, V, c->g.Vh, R);
    LAPH_HIP(hipGetLastError());
}

// scratch of the network calls: what = 0 forward, 1 backward (with input gradient), 2 one
// training step, 3 the solver's use (links, weights and a forward pass on nrhs fields)
size_t ptnet_scratch_bytes(const Geom &g, const laph_ptnet *net, int nrhs, int what)
{
    const size_t V = g.V, fb = sizeof(float2) * 12 * V * nrhs, nw = net->nw;
    size_t s = ws_align(sizeof(float2) * V * 36) + ws_align(4 * nw);            // links, wbf
    s += 2 * ws_align(fb * net->cmax);                                            // tmp0, tmp1
    if (what == 3) return s;
    s += 2 * ws_align(fb);                                                         // in, out
    if (what == 0) return s;
    for (int l = 1; l < net->layers; l++) s += ws_align(fb * net->ch[l]);          // kept activations
    s += ws_align(sizeof(float2) * nw) + ws_align(4 * (size_t)net->cmax * net->cmax * 144);  // grad, wadj
    const long n = (long)V * nrhs;
    long chunk = std::max<long>(kPtBS * 8, (n + 255) / 256);
    chunk = (chunk + kPtBS - 1) / kPtBS * kPtBS;
    const size_t nblk = (n + chunk - 1) / chunk;
    for (int l = 0; l < net->layers; l++)  // the per-layer partial gradients (grow-only name)
        s += ws_align(sizeof(float2) * net->ch[l] * net->ch[l + 1] * 144 * nblk);
    s += ws_align(fb);  // g
    if (what == 1) return s + ws_align(fb);  // gin
    const size_t pb = (V + 16 * kPtBS - 1) / (16 * kPtBS);
    s += ws_align(sizeof(double) * pb * nrhs) + ws_align(sizeof(double) * nrhs);  // loss partials, 1/|x|^2
    s += 3 * ws_align(sizeof(float2) * nw) + ws_align(4 * nw);                     // w32, m1, m2, new BF16
    return s;
}

// ---------------------------------------------------------------------- C-ABI
static void set_master(laph_ptnet *net, const std::vector<float> &w)
{
    net->w32 = w;
    net->m1.assign(2 * net->nw, 0.0f);
    net->m2.assign(2 * net->nw, 0.0f);
    net->step = 0;
}

extern "C" int laph_ptnet_create(laph_ctx_t c, int layers, const int *channels, uint64_t seed, laph_ptnet_t *out)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    LAPH_CHECK(out && channels && layers >= 1 && layers <= LAPH_PTNET_MAX_LAYERS, LAPH_EINVAL,
               "need 1..%d layers and a channel list", LAPH_PTNET_MAX_LAYERS);
    *out = nullptr;
    LAPH_CHECK(channels[0] == 1 && channels[layers] == 1, LAPH_EINVAL, "the first and last channel counts must be 1");
    for (int l = 0; l <= layers; l++)
        LAPH_CHECK(channels[l] == 1 || channels[l] == 2 || channels[l] == 4, LAPH_EINVAL,
                   "channel counts must be 1, 2 or 4");
    laph_ptnet *net = new laph_ptnet();
    try {
        net->device = c->device;
        net->layers = layers;
        net->ch.assign(channels, channels + layers + 1);
        for (int l = 0; l < layers; l++) {
            net->woff.push_back(net->nw);
            net->nw += (size_t)channels[l] * channels[l + 1] * 144;
            net->cmax = std::max(net->cmax, channels[l + 1]);
        }
        // small Gaussian weights plus 1/C_in times the identity on the self path, so that
        // the untrained net starts near a multiple of the identity
        std::mt19937_64 gen(seed);
        std::normal_distribution<float> nd(0.f, 1.f);
        std::vector<float> w(2 * net->nw);
        for (int l = 0; l < layers; l++) {
            int ci = channels[l], co = channels[l + 1];
            for (int o = 0; o < co; o++)
                for (int i = 0; i < ci; i++)
                    for (int d = 0; d < 9; d++)
                        for (int e = 0; e < 16; e++) {
                            size_t k = net->woff[l] + ((size_t)(o * ci + i) * 9 + d) * 16 + e;
                            float re = 0.02f * nd(gen), im = 0.02f * nd(gen);
                            if (d == 0 && (e % 5) == 0) re += 1.0f / ci;
                            w[2 * k] = re;
                            w[2 * k + 1] = im;
                        }
        }
        set_master(net, w);
    } catch (...) {
        delete net;
        throw;
    }
    *out = net;
    LAPH_API_END(c)
}

extern "C" int laph_ptnet_destroy(laph_ptnet_t net)
{
    if (!net) return LAPH_EINVAL;
    delete net;
    return LAPH_OK;
}

extern "C" int laph_ptnet_num_weights(laph_ptnet_t net, size_t *n)
{
    if (!net || !n) return LAPH_EINVAL;
    *n = net->nw;
    return LAPH_OK;
}

extern "C" int laph_ptnet_get_weights(laph_ptnet_t net, double *w)
{
    if (!net || !w) return LAPH_EINVAL;
    for (size_t i = 0; i < 2 * net->nw; i++) w[i] = net->w32[i];
    return LAPH_OK;
}

extern "C" int laph_ptnet_set_weights(laph_ptnet_t net, const double *w)
{
    if (!net || !w) return LAPH_EINVAL;
    std::vector<float> h(2 * net->nw);
    for (size_t i = 0; i < 2 * net->nw; i++) {
        if (!std::isfinite(w[i])) return LAPH_EINVAL;
        h[i] = (float)w[i];
    }
    set_master(net, h);
    return LAPH_OK;
}

extern "C" int laph_ptnet_forward(laph_ctx_t c, laph_ptnet_t net, const double *U, double bc_t, const double *in,
                                  double *out, int n_fields)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    check_net(c, net);
    LAPH_CHECK(U && in && out && n_fields > 0, LAPH_EINVAL, "null pointer or n_fields <= 0");
    long n = c->g.V * 12 * (long)n_fields;
    float2 *a = (float2 *)ctx_named(c, "net.in", sizeof(float2) * n);
    float2 *b = (float2 *)ctx_named(c, "net.out", sizeof(float2) * n);
    ptnet_prepare(c, net, U);
    hipLaunchKernelGGL(k_pt_from64, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, (const double2 *)in, a, n);
    LAPH_HIP(hipGetLastError());
    ptnet_forward(c, net, (float)bc_t, a, b, n_fields, 0);
    hipLaunchKernelGGL(k_pt_to64, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, (const float2 *)b,
                       (double2 *)out, n);
    LAPH_HIP(hipGetLastError());
    LAPH_HIP(hipStreamSynchronize(c->stream));
    LAPH_API_END(c)
}

extern "C" int laph_ptnet_backward(laph_ctx_t c, laph_ptnet_t net, const double *U, double bc_t, const double *in,
                                   const double *gout, double *gin, double *gw, int n_fields)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    check_net(c, net);
    LAPH_CHECK(U && in && gout && gw && n_fields > 0, LAPH_EINVAL, "null pointer or n_fields <= 0");
    long n = c->g.V * 12 * (long)n_fields;
    float2 *a = (float2 *)ctx_named(c, "net.in", sizeof(float2) * n);
    float2 *b = (float2 *)ctx_named(c, "net.out", sizeof(float2) * n);
    float2 *g = (float2 *)ctx_named(c, "net.g", sizeof(float2) * n);
    float2 *gi = gin ? (float2 *)ctx_named(c, "net.gin", sizeof(float2) * n) : nullptr;
    ptnet_prepare(c, net, U);
    hipLaunchKernelGGL(k_pt_from64, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, (const double2 *)in, a, n);
    hipLaunchKernelGGL(k_pt_from64, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, (const double2 *)gout, g, n);
    LAPH_HIP(hipGetLastError());
    ptnet_forward(c, net, (float)bc_t, a, b, n_fields, 1);
    ptnet_backward(c, net, (float)bc_t, g, gi, n_fields);
    if (gin) {
        hipLaunchKernelGGL(k_pt_to64, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, (const float2 *)gi,
                           (double2 *)gin, n);
        LAPH_HIP(hipGetLastError());
    }
    std::vector<float> h(2 * net->nw);
    LAPH_HIP(hipMemcpyAsync(h.data(), net->grad, sizeof(float2) * net->nw, hipMemcpyDeviceToHost, c->stream));
    LAPH_HIP(hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < 2 * net->nw; i++) gw[i] = h[i];
    LAPH_API_END(c)
}

extern "C" int laph_ptnet_train_step(laph_ctx_t c, laph_ptnet_t net, const double *U, double bc_t, const double *b,
                                     const double *x, int n_pairs, const laph_adam *opt, double *loss)
{
    LAPH_API_BEGIN(c)
    g_current_ctx = c;
    check_net(c, net);
    LAPH_CHECK(U && b && x && opt && n_pairs > 0, LAPH_EINVAL, "null pointer or n_pairs <= 0");
    LAPH_CHECK(opt->lr > 0 && opt->beta1 >= 0 && opt->beta1 < 1 && opt->beta2 >= 0 && opt->beta2 < 1 &&
                   opt->eps > 0 && opt->loss_parity >= -1 && opt->loss_parity <= 1,
               LAPH_EINVAL, "bad optimiser parameters");
    long V = c->g.V;
    long n = V * 12 * (long)n_pairs;
    float2 *a = (float2 *)ctx_named(c, "net.in", sizeof(float2) * n);
    float2 *o = (float2 *)ctx_named(c, "net.out", sizeof(float2) * n);
    float2 *g = (float2 *)ctx_named(c, "net.g", sizeof(float2) * n);
    ptnet_prepare(c, net, U);
    hipLaunchKernelGGL(k_pt_from64, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, (const double2 *)b, a, n);
    LAPH_HIP(hipGetLastError());
    ptnet_forward(c, net, (float)bc_t, a, o, n_pairs, 1);
    // relative loss sum_r |N(b_r) - x_r|^2 / |x_r|^2 over the selected parity
    long chunk = 16 * kPtBS;
    int nblk = (int)((V + chunk - 1) / chunk);
    double *part = (double *)ctx_named(c, "net.part", sizeof(double) * nblk * n_pairs);
    double *inv = (double *)ctx_named(c, "net.inv", sizeof(double) * n_pairs);
    std::vector<double> hp((size_t)nblk * n_pairs), hinv(n_pairs);
    hipLaunchKernelGGL(k_pt_loss, dim3(nblk, n_pairs), dim3(kPtBS), 0, c->stream, (const float2 *)nullptr,
                       (const double2 *)x, (const double *)nullptr, (float2 *)nullptr, part, c->g.ns, V,
                       opt->loss_parity, chunk);
    LAPH_HIP(hipGetLastError());
    LAPH_HIP(hipMemcpyAsync(hp.data(), part, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, c->stream));
    LAPH_HIP(hipStreamSynchronize(c->stream));
    for (int r = 0; r < n_pairs; r++) {
        double s = 0;
        for (int k = 0; k < nblk; k++) s += hp[(size_t)r * nblk + k];
        LAPH_CHECK(s > 0, LAPH_EINVAL, "target %d is zero on the selected sites", r);
        hinv[r] = 1.0 / s;
    }
    LAPH_HIP(hipMemcpyAsync(inv, hinv.data(), sizeof(double) * n_pairs, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_pt_loss, dim3(nblk, n_pairs), dim3(kPtBS), 0, c->stream, (const float2 *)o,
                       (const double2 *)x, (const double *)inv, g, part, c->g.ns, V, opt->loss_parity, chunk);
    LAPH_HIP(hipGetLastError());
    ptnet_backward(c, net, (float)bc_t, g, nullptr, n_pairs);
    // the optimiser state goes to the device for the step and comes back
    const size_t wb = sizeof(float2) * net->nw;
    float2 *w32 = (float2 *)ctx_named(c, "net.w32", wb), *m1 = (float2 *)ctx_named(c, "net.m1", wb),
           *m2 = (float2 *)ctx_named(c, "net.m2", wb);
    uint32_t *wbf_new = (uint32_t *)ctx_named(c, "net.wbf_new", sizeof(uint32_t) * net->nw);
    LAPH_HIP(hipMemcpyAsync(w32, net->w32.data(), wb, hipMemcpyHostToDevice, c->stream));
    LAPH_HIP(hipMemcpyAsync(m1, net->m1.data(), wb, hipMemcpyHostToDevice, c->stream));
    LAPH_HIP(hipMemcpyAsync(m2, net->m2.data(), wb, hipMemcpyHostToDevice, c->stream));
    const long step = net->step + 1;
    float bc1 = 1.f - std::pow((float)opt->beta1, (float)step);
    float bc2 = 1.f - std::pow((float)opt->beta2, (float)step);
    hipLaunchKernelGGL(k_pt_adam, dim3(nblocks_for((long)net->nw, 256)), dim3(256), 0, c->stream, w32, wbf_new, m1,
                       m2, (const float2 *)net->grad, (long)net->nw, (float)opt->lr, (float)opt->beta1,
                       (float)opt->beta2, (float)opt->eps, bc1, bc2);
    LAPH_HIP(hipGetLastError());
    std::vector<float> nw32(2 * net->nw), nm1(2 * net->nw), nm2(2 * net->nw);
    LAPH_HIP(hipMemcpyAsync(nw32.data(), w32, wb, hipMemcpyDeviceToHost, c->stream));
    LAPH_HIP(hipMemcpyAsync(nm1.data(), m1, wb, hipMemcpyDeviceToHost, c->stream));
    LAPH_HIP(hipMemcpyAsync(nm2.data(), m2, wb, hipMemcpyDeviceToHost, c->stream));
    LAPH_HIP(hipMemcpyAsync(hp.data(), part, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, c->stream));
    LAPH_HIP(hipStreamSynchronize(c->stream));
    net->w32.swap(nw32);
    net->m1.swap(nm1);
    net->m2.swap(nm2);
    net->step = step;
    if (loss) {
        double s = 0;
        for (int r = 0; r < n_pairs; r++) {
            double q = 0;
            for (int k = 0; k < nblk; k++) q += hp[(size_t)r * nblk + k];
            s += q * hinv[r];
        }
        *loss = s / n_pairs;
    }
    LAPH_API_END(c)
}

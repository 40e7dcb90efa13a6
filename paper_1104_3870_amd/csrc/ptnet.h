// Gauge-equivariant parallel-transport network (learned preconditioner), internal API.
//
// Net layout of a batch of fields: float2 a[((r*C + c)*V + s)*12 + k] with s the
// lexicographic site (x fastest) and k = alpha*3 + colour, i.e. the canonical spinor order
// in FP32 with a channel axis.  Links: float2 [V][4][9] (canonical order, FP32).
#pragma once

#include "laph_impl.h"

struct laph_ptnet {
    int device = 0;
    int layers = 0;
    std::vector<int> ch;       // channels[0..layers], ch[0] = ch[layers] = 1
    std::vector<size_t> woff;  // offset (complex elements) of each layer's weights
    size_t nw = 0;             // total complex weights
    int cmax = 1;              // widest layer
    // persistent state in host memory (a few KB): FP32 master weights and Adam moments,
    // (re, im) interleaved
    std::vector<float> w32, m1, m2;
    long step = 0;
    // device copies for the running call, in the context's scratch (ptnet_prepare)
    const float2 *links = nullptr;   // FP32 links of the call's field
    const uint32_t *wbf = nullptr;   // BF16 working copy (bf16(re) | bf16(im) << 16)
    float2 *grad = nullptr;          // weight gradients dL/dW^*
    const float2 *act0 = nullptr;    // input of the last forward pass that kept activations
    std::vector<const float2 *> acts;  // inputs of layers 1.. kept for the backward pass
    std::vector<uint32_t> wbf_h;     // staging of the BF16 copy (alive while its upload runs)
};

// FP32 links of U and the BF16 weights in the context's scratch for this call
void ptnet_prepare(laph_ctx *c, laph_ptnet *net, const double *U);
// out = N(in) for nrhs fields in the net layout (1 channel in and out).  With keep != 0 the
// layer inputs are kept for ptnet_backward.
void ptnet_forward(laph_ctx *c, laph_ptnet *net, float bct, const float2 *in, float2 *out, int nrhs, int keep);
// with g = dL/d(out)^* (net layout) after ptnet_forward(keep = 1): writes dL/dW^* into
// net->grad and, if gin is not null, dL/d(in)^* into gin
void ptnet_backward(laph_ctx *c, laph_ptnet *net, float bct, const float2 *g, float2 *gin, int nrhs);
// even-odd FP64 half vector of one right-hand side ([12][Vh]) <-> net layout, other
// parity zero / dropped
void eo_to_net(laph_ctx *c, const double2 *half, int par, float2 *full);
void net_to_eo(laph_ctx *c, const float2 *full, int par, double2 *half);
// odd part of N(gamma_4 eta) for R canonical FP64 sources, as the FP64 even-odd batch
// xo[(k*Vh + i)*R + r] (initial guess of the odd-site system: x = K^-1 gamma_4 eta)
void ptnet_initial_guess(laph_ctx *c, laph_ptnet *net, float bct, const double *eta, int R, double2 *xo);
// workspace scratch of the network's calls (see ptnet.hip)
size_t ptnet_scratch_bytes(const Geom &g, const laph_ptnet *net, int nrhs, int what);

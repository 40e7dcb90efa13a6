// Whole-spinor loads and stores in every storage precision and layout.
#pragma once

#include "dslash.h"

template <class SP>
struct alignas(16) Spin12 {
    typename SP::E v[12];
};

// o[k] = component k (alpha*3 + c) of right-hand side r at site i, in arithmetic type A
template <class SP, typename A>
__device__ __forceinline__ void ld_spinor12(const typename SP::E *base, const float *nrm, long Vh, int R, long i, int r,
                                            Cx<A> (&o)[12])
{
    float sc = 1.0f;
    if constexpr (SP::kNorm) sc = nrm[i * R + r];
    if constexpr (SP::kAoS) {
        Spin12<SP> pk = *reinterpret_cast<const Spin12<SP> *>(base + (i * R + r) * 12);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            auto c = SP::ld(&pk.v[k], 0, sc);
            o[k] = {(A)c.re, (A)c.im};
        }
    } else {
#pragma unroll
        for (int k = 0; k < 12; k++) {
            auto c = SP::ld(base, SP::idx(k, i, r, Vh, R), sc);
            o[k] = {(A)c.re, (A)c.im};
        }
    }
}

template <class SP, typename A>
__device__ __forceinline__ void st_spinor12(typename SP::E *base, float *nrm, long Vh, int R, long i, int r,
                                            const Cx<A> (&v)[12])
{
    using SA = typename SP::A;
    float inv = 1.0f;
    if constexpr (SP::kNorm) {
        float m = 0.0f;
#pragma unroll
        for (int k = 0; k < 12; k++) m = fmaxf(m, fmaxf(fabsf((float)v[k].re), fabsf((float)v[k].im)));
        // sites below 1e-30 (far tails of a source on one time slice) keep scale 1 and
        // flush to zero in FP16; a denormal scale would make 1/scale infinite
        float sc = m > 1e-30f ? m : 1.0f;
        nrm[i * R + r] = sc;
        inv = 1.0f / sc;
    }
    if constexpr (SP::kAoS) {
        Spin12<SP> pk;
#pragma unroll
        for (int k = 0; k < 12; k++) SP::st(&pk.v[k], 0, Cx<SA>{(SA)v[k].re, (SA)v[k].im}, inv);
        *reinterpret_cast<Spin12<SP> *>(base + (i * R + r) * 12) = pk;
    } else {
#pragma unroll
        for (int k = 0; k < 12; k++) SP::st(base, SP::idx(k, i, r, Vh, R), Cx<SA>{(SA)v[k].re, (SA)v[k].im}, inv);
    }
}

// Whole-spinor loads and stores in every storage precision and layout.
#pragma once

#include "dslash.h"

template <class SP>
struct alignas(16) Spin12 {
    typename SP::E v[12];
};

// Low-precision batches store each (site, right-hand side) record of 12 complex numbers as
// C = sizeof(record) / 16 chunks of 16 bytes, chunk q of site i and right-hand side r at
// byte ((i C + q) R + r) 16: the R records of a site are interleaved chunk by chunk, so a
// wave-wide 16-byte access of consecutive right-hand sides is contiguous.
template <class SP>
__device__ __forceinline__ Spin12<SP> ld_rec(const typename SP::E *base, long i, int R, int r)
{
    constexpr int C = sizeof(Spin12<SP>) / 16;
    Spin12<SP> pk;
    const uint4 *b = reinterpret_cast<const uint4 *>(base);
#pragma unroll
    for (int q = 0; q < C; q++) reinterpret_cast<uint4 *>(&pk)[q] = b[((size_t)i * C + q) * R + r];
    return pk;
}
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

// NT: non-temporal stores (streamed past L2, so that they do not evict lines a stencil
// still reads)
template <class SP, bool NT = false>
__device__ __forceinline__ void st_rec(typename SP::E *base, long i, int R, int r, const Spin12<SP> &pk)
{
    constexpr int C = sizeof(Spin12<SP>) / 16;
    if constexpr (NT) {
        u32x4_t *b = reinterpret_cast<u32x4_t *>(base);
#pragma unroll
        for (int q = 0; q < C; q++)
            __builtin_nontemporal_store(reinterpret_cast<const u32x4_t *>(&pk)[q], &b[((size_t)i * C + q) * R + r]);
    } else {
        uint4 *b = reinterpret_cast<uint4 *>(base);
#pragma unroll
        for (int q = 0; q < C; q++) b[((size_t)i * C + q) * R + r] = reinterpret_cast<const uint4 *>(&pk)[q];
    }
}

template <bool NT>
__device__ __forceinline__ void st_scale(float *p, float v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// o[k] = component k (alpha*3 + c) of right-hand side r at site i, in arithmetic type A
template <class SP, typename A>
__device__ __forceinline__ void ld_spinor12(const typename SP::E *base, const float *nrm, long Vh, int R, long i, int r,
                                            Cx<A> (&o)[12])
{
    float sc = 1.0f;
    if constexpr (SP::kNorm) sc = nrm[i * R + r];
    if constexpr (SP::kAoS) {
        Spin12<SP> pk = ld_rec<SP>(base, i, R, r);
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

template <class SP, typename A, bool NT = false>
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
        st_scale<NT>(&nrm[i * R + r], sc);
        inv = 1.0f / sc;
    }
    if constexpr (SP::kAoS) {
        Spin12<SP> pk;
#pragma unroll
        for (int k = 0; k < 12; k++) SP::st(&pk.v[k], 0, Cx<SA>{(SA)v[k].re, (SA)v[k].im}, inv);
        st_rec<SP, NT>(base, i, R, r, pk);
    } else {
#pragma unroll
        for (int k = 0; k < 12; k++) SP::st(base, SP::idx(k, i, r, Vh, R), Cx<SA>{(SA)v[k].re, (SA)v[k].im}, inv);
    }
}

// store v; return the stored record and its scale (a later load returns scale times the
// record's values)
template <class SP, bool NT = false>
__device__ __forceinline__ void st_spinor12_rec(typename SP::E *base, float *nrm, long i, int R, int r,
                                                const Cx<float> (&v)[12], Spin12<SP> &pk, float &sc)
{
    static_assert(SP::kAoS, "record layouts only");
    float inv = 1.0f;
    sc = 1.0f;
    if constexpr (SP::kNorm) {
        float m = 0.0f;
#pragma unroll
        for (int k = 0; k < 12; k++) m = fmaxf(m, fmaxf(fabsf(v[k].re), fabsf(v[k].im)));
        sc = m > 1e-30f ? m : 1.0f;
        st_scale<NT>(&nrm[i * R + r], sc);
        inv = 1.0f / sc;
    }
#pragma unroll
    for (int k = 0; k < 12; k++) SP::st(&pk.v[k], 0, Cx<float>{v[k].re, v[k].im}, inv);
    st_rec<SP, NT>(base, i, R, r, pk);
}

// store v and replace it by the values a later load returns (storage rounding and scale)
template <class SP, bool NT = false>
__device__ __forceinline__ void st_spinor12_round(typename SP::E *base, float *nrm, long Vh, int R, long i, int r,
                                                  Cx<float> (&v)[12])
{
    static_assert(SP::kAoS, "record layouts only");
    float inv = 1.0f, sc = 1.0f;
    if constexpr (SP::kNorm) {
        float m = 0.0f;
#pragma unroll
        for (int k = 0; k < 12; k++) m = fmaxf(m, fmaxf(fabsf(v[k].re), fabsf(v[k].im)));
        sc = m > 1e-30f ? m : 1.0f;
        st_scale<NT>(&nrm[i * R + r], sc);
        inv = 1.0f / sc;
    }
    Spin12<SP> pk;
#pragma unroll
    for (int k = 0; k < 12; k++) SP::st(&pk.v[k], 0, Cx<float>{v[k].re, v[k].im}, inv);
    st_rec<SP, NT>(base, i, R, r, pk);
#pragma unroll
    for (int k = 0; k < 12; k++) {
        auto c = SP::ld(&pk.v[k], 0, sc);
        v[k] = {(float)c.re, (float)c.im};
    }
}


// Batched complex FP64 products C = A B on the FP64 matrix cores (v_mfma_f64_16x16x4f64),
// the dense contractions of the hadron functions: momentum overlaps of displaced LapH
// vectors, the baryon eigenvector tensor and the baryon functions of noise fields.
//
// A block of 256 lanes (four waves) computes a 64 x 64 tile of C; each wave a 32 x 32
// quadrant as 2 x 2 tiles of 16 x 16.  K is staged through LDS KT values at a time by the
// problem's own stager (so that operands can be formed on the way: a conjugate, a phase),
// real and imaginary parts in separate arrays.  A complex
// product takes four real MFMAs per K step of 4: C_re += A_re B_re - A_im B_im,
// C_im += A_re B_im + A_im B_re.
//
// Lane layout of the 16 x 16 x 4 FP64 MFMA (lane l of 64): A operand A[l % 16][l / 16],
// B operand B[l / 16][l % 16], result element v of lane l at C[l / 16 + 4 v][l % 16].
#pragma once

#include <hip/hip_runtime.h>

namespace zg {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kTM = 64, kTN = 64;  // block tile
constexpr int kPad = 4;            // LDS row padding (doubles)

template <int KT>
struct Tile {
    double ar[KT][kTM + kPad], ai[KT][kTM + kPad];  // A[m][k] stored as [k][m]
    double br[KT][kTN + kPad], bi[KT][kTN + kPad];  // B[k][n]
};

// Each lane stages kPer = kTM KT / 256 elements of A and of B per K tile; the global loads
// of tile k + 1 are issued into registers before the products of tile k, and written to
// LDS (with the operands formed: a conjugate, a phase) after them.
//
// S provides: int K; __device__ bool tile(long &batch, int &m0, int &n0) const (false: the
// block has nothing to do); a register type S::Reg<KT>; __device__ void load(Reg<KT> &r,
// long batch, int m0, int n0, int k0) const (the global loads of one K tile, zeros outside
// the problem, no arithmetic on the loaded values); __device__ void put(Tile<KT> &t, const
// Reg<KT> &r) const (all KT rows into LDS; called by every lane, followed by a barrier);
// __device__ void store(long batch, int m, int n, double re, double im) const (m, n
// absolute; called only for m < M, n < N, which store checks itself through S::M/N).
template <int KT>
constexpr int kPer = kTM * KT / 256;

template <int KT, class S>
__global__ __launch_bounds__(256) void k_zgemm(const S s)
{
    static_assert(KT % 4 == 0, "K tile must be a multiple of the MFMA K step");
    static_assert(kTM == kTN && (kTM * KT) % 256 == 0, "whole elements per lane");
    __shared__ Tile<KT> sm;
    long batch;
    int m0, n0;
    if (!s.tile(batch, m0, n0)) return;  // uniform over the block
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
    const int lr = l & 15, lk = l >> 4;
    d4 cr[2][2], ci[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) {
            cr[i][j] = d4{0.0, 0.0, 0.0, 0.0};
            ci[i][j] = d4{0.0, 0.0, 0.0, 0.0};
        }
    typename S::template Reg<KT> reg;
    s.load(reg, batch, m0, n0, 0);
    for (int k0 = 0; k0 < s.K; k0 += KT) {
        s.put(sm, reg);
        __syncthreads();
        if (k0 + KT < s.K) s.load(reg, batch, m0, n0, k0 + KT);
        // one MFMA K step at a time: its operands are what stays live beside the next tile's
        // loads
#pragma unroll 1
        for (int kk = 0; kk < KT; kk += 4) {
            double ar[2], ai[2], an[2], br[2], bi[2];
#pragma unroll
            for (int i = 0; i < 2; i++) {
                ar[i] = sm.ar[kk + lk][wm + 16 * i + lr];
                ai[i] = sm.ai[kk + lk][wm + 16 * i + lr];
                an[i] = -ai[i];
            }
#pragma unroll
            for (int j = 0; j < 2; j++) {
                br[j] = sm.br[kk + lk][wn + 16 * j + lr];
                bi[j] = sm.bi[kk + lk][wn + 16 * j + lr];
            }
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < 2; j++) {
                    cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], cr[i][j], 0, 0, 0);
                    cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(an[i], bi[j], cr[i][j], 0, 0, 0);
                    ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], ci[i][j], 0, 0, 0);
                    ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], ci[i][j], 0, 0, 0);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int m = m0 + wm + 16 * i + lk + 4 * v, n = n0 + wn + 16 * j + lr;
                if (m < s.M && n < s.N) s.store(batch, m, n, cr[i][j][v], ci[i][j][v]);
            }
}

}  // namespace zg

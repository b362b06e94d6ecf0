// Helpers shared by the MLP kernels (FP32 and reduced-precision forms).
#pragma once

#include "common.h"

namespace prenom {

__device__ __forceinline__ floatx4 relu4(floatx4 v)
{
    floatx4 r;
    r[0] = fmaxf(v[0], 0.0f);
    r[1] = fmaxf(v[1], 0.0f);
    r[2] = fmaxf(v[2], 0.0f);
    r[3] = fmaxf(v[3], 0.0f);
    return r;
}

__device__ __forceinline__ floatx4 mask_pos(floatx4 g, floatx4 h)
{
    floatx4 r;
    r[0] = h[0] > 0.0f ? g[0] : 0.0f;
    r[1] = h[1] > 0.0f ? g[1] : 0.0f;
    r[2] = h[2] > 0.0f ? g[2] : 0.0f;
    r[3] = h[3] > 0.0f ? g[3] : 0.0f;
    return r;
}

// Orders one wave's LDS writes before its later LDS reads (and reads before
// later overwrites): a wave's LDS operations execute in program order, so
// only compiler reordering has to be prevented.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float sigmoidf_(float z) { return 1.0f / (1.0f + __expf(-z)); }


// Per-block LDS and launch parameters of the backward kernels.
constexpr int kBwdWaves = 8;      // waves per block
constexpr int kBwdMaxBlocks = 256;
constexpr int kStagePad = 4;      // floats of padding per staged row

// Blocks of the backward grid for n_s samples (each block writes one partial dW).
inline int bwd_blocks(int64_t n_s)
{
    const int64_t n_tiles = (n_s + 15) / 16;
    int64_t b = (n_tiles + kBwdWaves * 16 - 1) / (kBwdWaves * 16);  // >= 16 tiles per wave
    b = b < 1 ? 1 : b;
    return (int)(b > kBwdMaxBlocks ? kBwdMaxBlocks : b);
}

// Stage the tile's delta (D layout, out tiles) and h (D layout) for the
// dW = delta h^T contraction over the 16 samples.
template <int OTILES, int ITILES, int DP, int HP>
__device__ __forceinline__ void stage_dw(float* __restrict__ sD, float* __restrict__ sH,
                                         const floatx4 (&delta)[OTILES], const floatx4 (&h)[ITILES], int q, int j)
{
#pragma unroll
    for (int to = 0; to < OTILES; ++to)
#pragma unroll
        for (int r = 0; r < 4; ++r) sD[j * DP + 16 * to + 4 * q + r] = delta[to][r];
#pragma unroll
    for (int ti = 0; ti < ITILES; ++ti)
#pragma unroll
        for (int r = 0; r < 4; ++r) sH[j * HP + 16 * ti + 4 * q + r] = h[ti][r];
}

// Add (or, for the first wave, store) one dW accumulator set into the
// block's LDS reduction buffer (D layout: row 16 to + 4 q + r, col 16 ti + j).
template <int OTILES, int ITILES>
__device__ __forceinline__ void merge_dw(float* __restrict__ dst, const floatx4 (&dw)[OTILES][ITILES], int rows,
                                         int cols, int q, int j, bool first)
{
#pragma unroll
    for (int to = 0; to < OTILES; ++to)
#pragma unroll
        for (int ti = 0; ti < ITILES; ++ti)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * to + 4 * q + r, col = 16 * ti + j;
                if (row < rows && col < cols) {
                    float* p = dst + row * cols + col;
                    *p = first ? dw[to][ti][r] : *p + dw[to][ti][r];
                }
            }
}

}  // namespace prenom

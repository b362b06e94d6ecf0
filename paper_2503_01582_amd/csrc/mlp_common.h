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

// ---------------------------------------------------------------- 128-wide weight gradient
// The weight-gradient kernels of the 128-wide MLP stage a chunk of
// kDwChunk samples in LDS: every layer's delta and activation rows (pitch PW
// floats), the input features (pitch PY, zero beyond IN) and the head adjoint
// dO, all loaded with coalesced vector reads; the MFMA operands are then read
// from LDS.  PW is chosen per operand pattern so those reads are free of bank
// conflicts (FP32: lanes q step one sample, PW = 16 mod 64; 16-bit operands:
// lanes q step four samples, PW = 4 mod 16).
constexpr int kDwChunk = 32;

template <int W, int D, int PW, int PY>
struct DwStage {
    static constexpr int DL = 0;                          // deltas [D][chunk][PW]
    static constexpr int AC = DL + D * kDwChunk * PW;     // activations [D][chunk][PW]
    static constexpr int Y = AC + D * kDwChunk * PW;      // inputs [chunk][PY]
    static constexpr int DO = Y + kDwChunk * PY;          // head adjoint [chunk][4]
    static constexpr int FLOATS = DO + kDwChunk * 4;
};

// Input features and head adjoint of samples [s0, min(s0 + kDwChunk, s_end))
// into LDS (zeros past the end; input columns >= IN zero).  y: level-major
// [L][n_s][2].
template <int IN, int W, int D, int PW, int PY>
__device__ __forceinline__ void dw_stage_inputs(float* __restrict__ lds, const float* __restrict__ y,
                                                const float4* __restrict__ sc, const float4* __restrict__ dout,
                                                int64_t n_s, int64_t s0, int64_t s_end)
{
    using St = DwStage<W, D, PW, PY>;
    for (int i = threadIdx.x; i < kDwChunk * (PY / 2); i += blockDim.x) {
        const int r = i / (PY / 2), l = i % (PY / 2);
        const int64_t s = s0 + r;
        float2 v = make_float2(0.0f, 0.0f);
        if (s < s_end && 2 * l < IN) v = reinterpret_cast<const float2*>(y)[(int64_t)l * n_s + s];
        *reinterpret_cast<float2*>(lds + St::Y + r * PY + 2 * l) = v;
    }
    if (threadIdx.x < kDwChunk) {
        const int r = threadIdx.x;
        const int64_t s = s0 + r;
        floatx4 o = {0.0f, 0.0f, 0.0f, 0.0f};
        if (s < s_end) {  // d sigma / d o0 = sigma, d c / d o = c (1 - c)
            const float4 g = dout[s], v = sc[s];
            o = {g.x * v.x, g.y * v.y * (1.0f - v.y), g.z * v.z * (1.0f - v.z), g.w * v.w * (1.0f - v.w)};
        }
        *reinterpret_cast<floatx4*>(lds + St::DO + r * 4) = o;
    }
}

// Every layer's activation and delta rows (FP32, [D][n_s][W]) of the chunk.
template <int IN, int W, int D, int PW, int PY>
__device__ __forceinline__ void dw_stage(float* __restrict__ lds, const float* __restrict__ y,
                                         const float4* __restrict__ sc, const float4* __restrict__ dout,
                                         const float* __restrict__ act, const float* __restrict__ dlt, int64_t n_s,
                                         int64_t s0, int64_t s_end)
{
    using St = DwStage<W, D, PW, PY>;
    constexpr int V = W / 4;  // float4 per row
    for (int i = threadIdx.x; i < D * kDwChunk * V; i += blockDim.x) {
        const int k = i / (kDwChunk * V), rem = i % (kDwChunk * V), r = rem / V, c = rem % V;
        const int64_t s = s0 + r;
        floatx4 a = {0.0f, 0.0f, 0.0f, 0.0f}, d = {0.0f, 0.0f, 0.0f, 0.0f};
        if (s < s_end) {
            a = *reinterpret_cast<const floatx4*>(act + ((int64_t)k * n_s + s) * W + 4 * c);
            d = *reinterpret_cast<const floatx4*>(dlt + ((int64_t)k * n_s + s) * W + 4 * c);
        }
        *reinterpret_cast<floatx4*>(lds + St::AC + (k * kDwChunk + r) * PW + 4 * c) = a;
        *reinterpret_cast<floatx4*>(lds + St::DL + (k * kDwChunk + r) * PW + 4 * c) = d;
    }
    dw_stage_inputs<IN, W, D, PW, PY>(lds, y, sc, dout, n_s, s0, s_end);
}

}  // namespace prenom

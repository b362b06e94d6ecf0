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

// Maxima of |dy| per (level, block of kScatterBlockSamples samples), which fix
// the hash-table gradient's fixed-point scale, taken by the batched MLP
// backward as it writes dy: per wave and tile a DPP row maximum over the 16
// samples, one LDS atomic max per (tile, level) on the bit pattern (non-
// negative floats order as unsigned integers; NaN is dropped by fmaxf, as
// the scatter's own pass drops it), then one store per (block, level) when
// the work item ends.  A work item starts at a multiple of kBmTiles tiles of
// its object and spans at most kBmSlots blocks.
constexpr int kBmTiles = kScatterBlockSamples / 16;
constexpr int kBmSlots = 32;
constexpr int kBmMaxTiles = kBmTiles * kBmSlots;  // 1024 tiles per work item
constexpr int kBmLevels = 16;                     // the compiled MLP inputs have at most 32 features
struct DyMaxLds {
    uint32_t v[kBmSlots][kBmLevels];
};

__device__ __forceinline__ void dymax_clear(DyMaxLds& bm)
{
    for (int i = threadIdx.x; i < kBmSlots * kBmLevels; i += blockDim.x) (&bm.v[0][0])[i] = 0u;
}

// Lanes (q, j) of a wave hold dy of sample j of `tile` for levels lv and
// lv + 1 (features 2 lv .. 2 lv + 3); `ok`: the sample exists and lv < L.
// Called by every lane of the wave.
__device__ __forceinline__ void dymax_note(DyMaxLds& bm, int64_t tile, int64_t tile_begin, int lv, floatx4 g, bool ok,
                                           int j, bool& bad)
{
    float m0 = ok ? fmaxf(fabsf(g[0]), fabsf(g[1])) : 0.0f;
    float m1 = ok ? fmaxf(fabsf(g[2]), fabsf(g[3])) : 0.0f;
    bad |= ok && !(isfinite(g[0]) && isfinite(g[1]) && isfinite(g[2]) && isfinite(g[3]));
    m0 = fmaxf(m0, dpp_f32<0x101>(m0));
    m1 = fmaxf(m1, dpp_f32<0x101>(m1));
    m0 = fmaxf(m0, dpp_f32<0x102>(m0));
    m1 = fmaxf(m1, dpp_f32<0x102>(m1));
    m0 = fmaxf(m0, dpp_f32<0x104>(m0));
    m1 = fmaxf(m1, dpp_f32<0x104>(m1));
    m0 = fmaxf(m0, dpp_f32<0x108>(m0));
    m1 = fmaxf(m1, dpp_f32<0x108>(m1));
    if (j == 0 && ok) {
        const int slot = (int)((tile - tile_begin) / kBmTiles);
        atomicMax(&bm.v[slot][lv], __float_as_uint(m0));
        atomicMax(&bm.v[slot][lv + 1], __float_as_uint(m1));
    }
}

// After a barrier: the work item's block maxima to block_max ([L][n_blocks]
// of the object) and the non-finite flag.
__device__ __forceinline__ void dymax_flush(const DyMaxLds& bm, float* __restrict__ block_max, int64_t n_blocks,
                                            int n_levels, int64_t tile_begin, int64_t tile_end)
{
    const int64_t b0 = tile_begin / kBmTiles;
    const int n_slots = (int)((tile_end - tile_begin + kBmTiles - 1) / kBmTiles);
    for (int i = threadIdx.x; i < n_slots * n_levels; i += blockDim.x) {
        const int slot = i / n_levels, l = i % n_levels;
        if (b0 + slot < n_blocks) block_max[(int64_t)l * n_blocks + b0 + slot] = __uint_as_float(bm.v[slot][l]);
    }
}


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

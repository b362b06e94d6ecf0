// Reduced-precision form of the object-NeRF MLP: BF16 or FP16 operands on
// v_mfma_f32_16x16x16_{bf16,f16} with FP32 accumulation.  The FP32 master
// weights are converted once per block into LDS fragments; activations,
// deltas and every gradient stay FP32 in registers and are rounded only when
// they become an MFMA operand.
//
// Operand layouts of the 16x16x16 instruction (lane l, q = l/16, j = l%16):
// A[i][k] holds k = 4q..4q+3 of row i = j in lane l; B[k][n] holds
// k = 4q..4q+3 of column n = j; D[i][n] sits at lane n + 16*(i/4), register
// i%4.  So the four output registers of a 16-neuron tile are exactly the B
// operand of the next layer over that tile (k = 4q + r), with no permutation;
// weight fragments hold W[16 to + j][16 ti + 4q .. 4q+3].
//
// The weight gradient contracts over the 16 samples of a tile with one MFMA
// per (out tile, in tile), after the same per-wave LDS transpose as the FP32
// form; the 8 waves of a block merge their dW in LDS and write one partial.
#include "mlp_common.h"

namespace prenom {
namespace {

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));

struct Bf16Op {
    using vec = short4_t;
    static __device__ __forceinline__ short cvt(float x) { return __builtin_bit_cast(short, (__bf16)x); }
    static __device__ __forceinline__ float back(short h)
    {
        return __builtin_bit_cast(float, (uint32_t)(uint16_t)h << 16);
    }
    static __device__ __forceinline__ floatx4 mma(vec a, vec b, floatx4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    }
};

struct F16Op {
    using vec = half4_t;
    static __device__ __forceinline__ _Float16 cvt(float x) { return (_Float16)x; }
    static __device__ __forceinline__ float back(_Float16 h) { return (float)h; }
    static __device__ __forceinline__ floatx4 mma(vec a, vec b, floatx4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
    }
};

template <class P>
__device__ __forceinline__ typename P::vec pack(float a, float b, float c, float d)
{
    typename P::vec v;
    v[0] = P::cvt(a);
    v[1] = P::cvt(b);
    v[2] = P::cvt(c);
    v[3] = P::cvt(d);
    return v;
}

template <class P>
__device__ __forceinline__ typename P::vec pack(floatx4 x)
{
    return pack<P>(x[0], x[1], x[2], x[3]);
}

template <class P>
__device__ __forceinline__ floatx4 unpack(typename P::vec v)
{
    return {P::back(v[0]), P::back(v[1]), P::back(v[2]), P::back(v[3])};
}

// ReLU masks of the 128-wide MLP, kept beside its stored activations as bits
// (the decision of the FP32 pre-activation, whatever the 16-bit activation
// rounds to): one 32-bit word per (layer, sample, lane group q), bit 4 to + r
// for neuron 16 to + 4 q + r.  The backward chain reads these 16 bytes per
// sample and layer instead of the 256-byte activation row.
__device__ __forceinline__ uint32_t relu_mask_bits(const floatx4* h, int n_tiles)
{
    uint32_t m = 0;
    for (int to = 0; to < n_tiles; ++to)
#pragma unroll
        for (int r = 0; r < 4; ++r) m |= (h[to][r] > 0.0f ? 1u : 0u) << (4 * to + r);
    return m;
}

__device__ __forceinline__ floatx4 mask_by_bits(floatx4 g, uint32_t m, int to)
{
    return {(m >> (4 * to)) & 1u ? g[0] : 0.0f, (m >> (4 * to + 1)) & 1u ? g[1] : 0.0f,
            (m >> (4 * to + 2)) & 1u ? g[2] : 0.0f, (m >> (4 * to + 3)) & 1u ? g[3] : 0.0f};
}

// Layout of the 128-wide MLP's activation buffer (mlp_act_floats floats):
// the activations, then the deltas, of every hidden layer in the MFMA type,
// each in the accumulator layout of its 16-sample tiles (for layer k, tile
// t, neuron tile to: 64 groups of 4 values, group 16 q + j holding neurons
// 16 to + 4 q .. + 3 of sample 16 t + j, so one wave's store of a neuron tile
// is 512 contiguous bytes); then the ReLU mask words [D][n_s][4].
template <int W>
__device__ __forceinline__ int64_t wide_vec(int k, int64_t n_s, int64_t s, int to, int q)
{
    const int64_t n_t = (n_s + 15) >> 4;
    return (((int64_t)k * n_t + (s >> 4)) * (W / 16) + to) * 64 + q * 16 + (s & 15);
}

template <int W, int D, class P>
__device__ __forceinline__ typename P::vec* wide_deltas(typename P::vec* a16, int64_t n_s)
{
    return a16 + (int64_t)D * ((n_s + 15) >> 4) * 4 * W;
}

template <int W, int D, class P>
__device__ __forceinline__ uint32_t* wide_masks(typename P::vec* a16, int64_t n_s)
{
    return reinterpret_cast<uint32_t*>(a16 + (int64_t)2 * D * ((n_s + 15) >> 4) * 4 * W);
}

template <int IN, int W, int D>
struct NetLp {
    static constexpr int KB1 = (IN + 15) / 16;  // 16-feature K-blocks of layer 1 (zero-padded)
    static constexpr int OT = W / 16;         // 16-neuron tiles of a hidden layer
    static constexpr int IT = (IN + 15) / 16; // 16-feature tiles of the input
    static constexpr int F1 = 0;                        // [OT][KB1]
    static constexpr int FH = F1 + OT * KB1;            // [D-1][OT][OT]
    static constexpr int FO = FH + (D - 1) * OT * OT;   // [OT]
    static constexpr int N_FWD = FO + OT;
    static constexpr int BO = N_FWD;                    // [OT]
    static constexpr int BH = BO + OT;                  // [D-1][OT][OT]
    static constexpr int B1 = BH + (D - 1) * OT * OT;   // [IT][OT]
    static constexpr int N_ALL = B1 + IT * OT;
    static constexpr int OFF_W1 = 0;
    static constexpr int OFF_H = W * IN;
    static constexpr int OFF_OUT = W * IN + (D - 1) * W * W;
    static constexpr int N_PARAMS = OFF_OUT + 4 * W;
    static_assert(IN % 8 == 0 && W % 16 == 0 && D >= 1, "shape");
};

// Weight fragments: fragment f, lane l holds 4 consecutive K values.
template <int IN, int W, int D, class P>
__device__ __forceinline__ void load_fragments_lp(const float* __restrict__ w, typename P::vec* __restrict__ frag, int n_frag, int f0 = 0)
{
    using N = NetLp<IN, W, D>;
    for (int idx = threadIdx.x; idx < n_frag * 64; idx += blockDim.x) {
        const int f = f0 + (idx >> 6), l = idx & 63, q = l >> 4, j = l & 15;
        float v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float x;
            if (f < N::FH) {  // W1[16 to + j][16 m + 4 q + r], features >= IN zero
                const int to = f / N::KB1, m = f % N::KB1, col = 16 * m + 4 * q + r;
                x = col < IN ? w[N::OFF_W1 + (16 * to + j) * IN + col] : 0.0f;
            } else if (f < N::FO) {  // Wk[16 to + j][16 ti + 4 q + r]
                const int g = f - N::FH, k = g / (N::OT * N::OT), rem = g % (N::OT * N::OT);
                const int to = rem / N::OT, ti = rem % N::OT;
                x = w[N::OFF_H + k * W * W + (16 * to + j) * W + 16 * ti + 4 * q + r];
            } else if (f < N::N_FWD) {  // Wout[j][16 ti + 4 q + r], rows >= 4 zero
                const int ti = f - N::FO;
                x = j < 4 ? w[N::OFF_OUT + j * W + 16 * ti + 4 * q + r] : 0.0f;
            } else if (f < N::BH) {  // Wout^T over the 4 outputs: k = 4 q + r < 4
                const int to = f - N::BO;
                x = q == 0 ? w[N::OFF_OUT + r * W + 16 * to + j] : 0.0f;
            } else if (f < N::B1) {  // Wk^T: Wk[16 ti + 4 q + r][16 to + j]
                const int g = f - N::BH, k = g / (N::OT * N::OT), rem = g % (N::OT * N::OT);
                const int to = rem / N::OT, ti = rem % N::OT;
                x = w[N::OFF_H + k * W * W + (16 * ti + 4 * q + r) * W + 16 * to + j];
            } else {  // W1^T: W1[16 ti + 4 q + r][16 to + j], columns >= IN zero
                const int g = f - N::B1, to = g / N::OT, ti = g % N::OT, col = 16 * to + j;
                x = col < IN ? w[N::OFF_W1 + (16 * ti + 4 * q + r) * IN + col] : 0.0f;
            }
            v[r] = x;
        }
        frag[idx] = pack<P>(v[0], v[1], v[2], v[3]);
    }
}

// Layer-1 inputs of one lane: features 16 m + 4 q + r of sample s (levels
// 8 m + 2 q and 8 m + 2 q + 1 of the level-major feature array); features
// beyond IN are zero.
template <int IN, int KB1>
__device__ __forceinline__ void load_inputs_lp(const float2* __restrict__ y, int64_t n_s, int64_t s, bool valid, int q,
                                               floatx4 (&yf)[KB1])
{
#pragma unroll
    for (int m = 0; m < KB1; ++m) {
        float2 a = make_float2(0.0f, 0.0f), b = make_float2(0.0f, 0.0f);
        const int l0 = 8 * m + 2 * q;
        if (valid && 2 * l0 < IN) a = y[(int64_t)l0 * n_s + s];
        if (valid && 2 * (l0 + 1) < IN) b = y[(int64_t)(l0 + 1) * n_s + s];
        yf[m] = {a.x, a.y, b.x, b.y};
    }
}

// acc[to] = sum_ti A(fragment f0 + to * stride + ti) x b[ti], K-blocks outer
// and output tiles inner (independent accumulators interleave), with a
// scheduling fence every 4 K-blocks so fragment loads are not all hoisted.
template <class P, int OT, int KT>
__device__ __forceinline__ void layer_lp_ks_outer(const typename P::vec* __restrict__ frag, int lane, int f0, int stride,
                                                  const typename P::vec (&b)[KT], floatx4 (&acc)[OT])
{
#pragma unroll
    for (int to = 0; to < OT; ++to) acc[to] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ti = 0; ti < KT; ++ti) {
#pragma unroll
        for (int to = 0; to < OT; ++to) acc[to] = P::mma(frag[(f0 + to * stride + ti) * 64 + lane], b[ti], acc[to]);
        if ((ti & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
}

template <int IN, int W, int D, class P>
__device__ __forceinline__ void chain_lp(const typename P::vec* __restrict__ frag, int lane,
                                         const floatx4 (&yf)[NetLp<IN, W, D>::KB1],
                                         floatx4 (&hs)[D][NetLp<IN, W, D>::OT], floatx4& o)
{
    using N = NetLp<IN, W, D>;
    if constexpr (W >= kWideWidth) {
        typename P::vec b1[N::KB1];
#pragma unroll
        for (int m = 0; m < N::KB1; ++m) b1[m] = pack<P>(yf[m]);
        floatx4 acc[N::OT];
        layer_lp_ks_outer<P, N::OT, N::KB1>(frag, lane, N::F1, N::KB1, b1, acc);
#pragma unroll
        for (int to = 0; to < N::OT; ++to) hs[0][to] = relu4(acc[to]);
#pragma unroll
        for (int k = 1; k < D; ++k) {
            typename P::vec b[N::OT];
#pragma unroll
            for (int ti = 0; ti < N::OT; ++ti) b[ti] = pack<P>(hs[k - 1][ti]);
            layer_lp_ks_outer<P, N::OT, N::OT>(frag, lane, N::FH + (k - 1) * N::OT * N::OT, N::OT, b, acc);
#pragma unroll
            for (int to = 0; to < N::OT; ++to) hs[k][to] = relu4(acc[to]);
        }
    } else {
#pragma unroll
        for (int to = 0; to < N::OT; ++to) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int m = 0; m < N::KB1; ++m) acc = P::mma(frag[(N::F1 + to * N::KB1 + m) * 64 + lane], pack<P>(yf[m]), acc);
            hs[0][to] = relu4(acc);
        }
#pragma unroll
        for (int k = 1; k < D; ++k) {
#pragma unroll
            for (int to = 0; to < N::OT; ++to) {
                floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int ti = 0; ti < N::OT; ++ti)
                    acc = P::mma(frag[(N::FH + ((k - 1) * N::OT + to) * N::OT + ti) * 64 + lane], pack<P>(hs[k - 1][ti]), acc);
                hs[k][to] = relu4(acc);
            }
        }
    }
    o = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ti = 0; ti < N::OT; ++ti) o = P::mma(frag[(N::FO + ti) * 64 + lane], pack<P>(hs[D - 1][ti]), o);
}

template <int IN, int W, int D, class P>
__device__ __forceinline__ void mlp_fwd_tiles_lp(const typename P::vec* __restrict__ frag,
                                                 const float2* __restrict__ y, int64_t n_s, float4* __restrict__ sc,
                                                 float* __restrict__ act, int64_t tile0, int64_t end, int64_t step)
{
    using N = NetLp<IN, W, D>;
    const int lane = threadIdx.x & 63, q = lane >> 4, j = lane & 15;
    floatx4 yn[N::KB1];  // the next tile's inputs, loaded while the current tile runs
    if (tile0 < end) load_inputs_lp<IN, N::KB1>(y, n_s, tile0 * 16 + j, tile0 * 16 + j < n_s, q, yn);
    for (int64_t tile = tile0; tile < end; tile += step) {
        const int64_t s = tile * 16 + j;
        const bool valid = s < n_s;
        floatx4 yf[N::KB1];
#pragma unroll
        for (int m = 0; m < N::KB1; ++m) yf[m] = yn[m];
        const int64_t sn = (tile + step) * 16 + j;
        if (tile + step < end) load_inputs_lp<IN, N::KB1>(y, n_s, sn, sn < n_s, q, yn);
        floatx4 hs[D][N::OT];
        floatx4 o;
        chain_lp<IN, W, D, P>(frag, lane, yf, hs, o);
        if (q == 0 && valid) sc[s] = make_float4(__expf(o[0]), sigmoidf_(o[1]), sigmoidf_(o[2]), sigmoidf_(o[3]));
        if (act && valid) {  // stored already rounded: the values every later use sees
            typename P::vec* a16 = reinterpret_cast<typename P::vec*>(act);
            uint32_t* masks = wide_masks<W, D, P>(a16, n_s);
#pragma unroll
            for (int k = 0; k < D; ++k) {
#pragma unroll
                for (int to = 0; to < N::OT; ++to) a16[wide_vec<W>(k, n_s, s, to, q)] = pack<P>(hs[k][to]);
                masks[((int64_t)k * n_s + s) * 4 + q] = relu_mask_bits(hs[k], N::OT);
            }
        }
    }
}

template <int IN, int W, int D, class P>
__global__ __launch_bounds__(256) void k_mlp_fwd_lp(const float* __restrict__ w, const float2* __restrict__ y,
                                                    int64_t n_s, float4* __restrict__ sc, float* __restrict__ act)
{
    using N = NetLp<IN, W, D>;
    extern __shared__ __align__(16) unsigned char smem_f[];
    typename P::vec* frag = reinterpret_cast<typename P::vec*>(smem_f);
    load_fragments_lp<IN, W, D, P>(w, frag, N::N_FWD);
    __syncthreads();
    const int64_t wave0 = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x / 64);
    mlp_fwd_tiles_lp<IN, W, D, P>(frag, y, n_s, sc, act, wave0, (n_s + 15) / 16, n_waves);
}

// Three waves per SIMD: without the hint the 128-wide shapes take 154 VGPRs
// plus 28 AGPRs (two waves); with it they fit 170 registers, a couple of
// spilled registers in the two-layer shapes, and the 48-object forward drops
// from 4.48 to 4.30 ms on gfx950.
template <int IN, int W, int D, class P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_mlp_fwd_lp_batch(
    const MlpWork* __restrict__ work, const float* __restrict__ params, const float2* __restrict__ y,
    float4* __restrict__ sc, float* __restrict__ act)
{
    using N = NetLp<IN, W, D>;
    extern __shared__ __align__(16) unsigned char smem_f[];
    typename P::vec* frag = reinterpret_cast<typename P::vec*>(smem_f);
    const MlpWork wk = work[blockIdx.x];
    load_fragments_lp<IN, W, D, P>(params + wk.w_off, frag, N::N_FWD);
    __syncthreads();
    mlp_fwd_tiles_lp<IN, W, D, P>(frag, y + wk.y_off / 2, wk.n_s, sc + wk.s_off, act ? act + wk.a_off : nullptr,
                                  wk.tile_begin + (threadIdx.x >> 6), wk.tile_end, blockDim.x / 64);
}

template <int IN, int W, int D>
struct BwdLdsLp {
    static constexpr int IP = 16 * NetLp<IN, W, D>::IT;
    static constexpr int HW = (W > IP ? W : IP) + kStagePad;
    static constexpr int DW = W + kStagePad;
    static constexpr int PER_WAVE = 16 * (HW + DW);  // floats
};

template <int OTILES, int ITILES, int DP, int HP, class P>
__device__ __forceinline__ void accumulate_dw_lp(const float* __restrict__ sD, const float* __restrict__ sH,
                                                 floatx4 (&dw)[OTILES][ITILES], int q, int j)
{
    typename P::vec a[OTILES], b[ITILES];
#pragma unroll
    for (int to = 0; to < OTILES; ++to)
        a[to] = pack<P>(sD[(4 * q) * DP + 16 * to + j], sD[(4 * q + 1) * DP + 16 * to + j],
                        sD[(4 * q + 2) * DP + 16 * to + j], sD[(4 * q + 3) * DP + 16 * to + j]);
#pragma unroll
    for (int ti = 0; ti < ITILES; ++ti)
        b[ti] = pack<P>(sH[(4 * q) * HP + 16 * ti + j], sH[(4 * q + 1) * HP + 16 * ti + j],
                        sH[(4 * q + 2) * HP + 16 * ti + j], sH[(4 * q + 3) * HP + 16 * ti + j]);
#pragma unroll
    for (int to = 0; to < OTILES; ++to)
#pragma unroll
        for (int ti = 0; ti < ITILES; ++ti) dw[to][ti] = P::mma(a[to], b[ti], dw[to][ti]);
}

// Backward over tiles tile0, tile0 + step, ... < end of one object whose
// fragments are at the start of smem_lp; called by every thread of the block.
// bm (or null): also note the maxima of |dy| of the work item starting at tile
// tile_begin; bad: set on a non-finite dy.
template <int IN, int W, int D, class P>
__device__ __forceinline__ void mlp_bwd_tiles_lp(unsigned char* __restrict__ smem_lp, const float2* __restrict__ y,
                                 const float4* __restrict__ dout, int64_t n_s, float2* __restrict__ dy,
                                 float* __restrict__ dst, int64_t tile0, int64_t end, int64_t step,
                                 DyMaxLds* bm = nullptr, int64_t tile_begin = 0, bool* bad = nullptr)
{
    using N = NetLp<IN, W, D>;
    using B = BwdLdsLp<IN, W, D>;
    const typename P::vec* frag = reinterpret_cast<const typename P::vec*>(smem_lp);
    float* stage = reinterpret_cast<float*>(smem_lp + sizeof(typename P::vec) * N::N_ALL * 64);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4, j = lane & 15;
    float* sD = stage + wave * B::PER_WAVE;
    float* sH = sD + 16 * B::DW;

    floatx4 dW1[N::OT][N::IT];
    floatx4 dWh[D > 1 ? D - 1 : 1][N::OT][N::OT];
    floatx4 dWo[1][N::OT];
#pragma unroll
    for (int a = 0; a < N::OT; ++a) {
#pragma unroll
        for (int b = 0; b < N::IT; ++b) dW1[a][b] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int b = 0; b < N::OT; ++b)
#pragma unroll
            for (int k = 0; k < (D > 1 ? D - 1 : 1); ++k) dWh[k][a][b] = {0.0f, 0.0f, 0.0f, 0.0f};
        dWo[0][a] = {0.0f, 0.0f, 0.0f, 0.0f};
    }

    // the next tile's inputs and upstream gradient, loaded while the current tile runs
    floatx4 yn[N::KB1];
    float4 gn = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    auto load_tile = [&](int64_t t) {
        const int64_t st = t * 16 + j;
        const bool ok = t < end && st < n_s;
        load_inputs_lp<IN, N::KB1>(y, n_s, st, ok, q, yn);
        gn = ok && q == 0 ? dout[st] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    };
    load_tile(tile0);
    for (int64_t tile = tile0; tile < end; tile += step) {
        const int64_t s = tile * 16 + j;
        const bool valid = s < n_s;
        floatx4 yf[N::KB1];
#pragma unroll
        for (int m = 0; m < N::KB1; ++m) yf[m] = yn[m];
        const float4 gc = gn;
        load_tile(tile + step);
        floatx4 hs[D][N::OT];
        floatx4 o;
        chain_lp<IN, W, D, P>(frag, lane, yf, hs, o);

        // head adjoint in the output tile's own layout (rows 4q + r; only q == 0 is real)
        floatx4 dO[1] = {{0.0f, 0.0f, 0.0f, 0.0f}};
        if (q == 0 && valid) {
            const float4 g = gc;
            const float c1 = sigmoidf_(o[1]), c2 = sigmoidf_(o[2]), c3 = sigmoidf_(o[3]);
            dO[0] = {g.x * __expf(o[0]), g.y * c1 * (1.0f - c1), g.z * c2 * (1.0f - c2), g.w * c3 * (1.0f - c3)};
        }
        wave_lds_sync();
        stage_dw<1, N::OT, B::DW, B::HW>(sD, sH, dO, hs[D - 1], q, j);
        wave_lds_sync();
        accumulate_dw_lp<1, N::OT, B::DW, B::HW, P>(sD, sH, dWo, q, j);

        floatx4 delta[N::OT];
        const typename P::vec dOp = pack<P>(dO[0]);
#pragma unroll
        for (int to = 0; to < N::OT; ++to) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = P::mma(frag[(N::BO + to) * 64 + lane], dOp, acc);
            delta[to] = mask_pos(acc, hs[D - 1][to]);
        }
#pragma unroll
        for (int k = D - 1; k >= 1; --k) {
            wave_lds_sync();
            stage_dw<N::OT, N::OT, B::DW, B::HW>(sD, sH, delta, hs[k - 1], q, j);
            wave_lds_sync();
            accumulate_dw_lp<N::OT, N::OT, B::DW, B::HW, P>(sD, sH, dWh[k - 1], q, j);
            typename P::vec dp[N::OT];
#pragma unroll
            for (int ti = 0; ti < N::OT; ++ti) dp[ti] = pack<P>(delta[ti]);
#pragma unroll
            for (int to = 0; to < N::OT; ++to) {
                floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int ti = 0; ti < N::OT; ++ti)
                    acc = P::mma(frag[(N::BH + ((k - 1) * N::OT + to) * N::OT + ti) * 64 + lane], dp[ti], acc);
                delta[to] = mask_pos(acc, hs[k - 1][to]);
            }
        }
        // layer 1: stage delta and the inputs (features 16 m + 4 q + r of sample j)
        wave_lds_sync();
#pragma unroll
        for (int to = 0; to < N::OT; ++to)
#pragma unroll
            for (int r = 0; r < 4; ++r) sD[j * B::DW + 16 * to + 4 * q + r] = delta[to][r];
#pragma unroll
        for (int m = 0; m < N::KB1; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) sH[j * B::HW + 16 * m + 4 * q + r] = yf[m][r];  // zero beyond IN
        wave_lds_sync();
        accumulate_dw_lp<N::OT, N::IT, B::DW, B::HW, P>(sD, sH, dW1, q, j);
        typename P::vec dp[N::OT];
#pragma unroll
        for (int ti = 0; ti < N::OT; ++ti) dp[ti] = pack<P>(delta[ti]);
#pragma unroll
        for (int to = 0; to < N::IT; ++to) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ti = 0; ti < N::OT; ++ti) acc = P::mma(frag[(N::B1 + to * N::OT + ti) * 64 + lane], dp[ti], acc);
            const int f = 16 * to + 4 * q;  // features f..f+3 = levels f/2 and f/2 + 1
            if (valid && f < IN) {
                dy[(int64_t)(f >> 1) * n_s + s] = make_float2(acc[0], acc[1]);
                dy[(int64_t)((f >> 1) + 1) * n_s + s] = make_float2(acc[2], acc[3]);
            }
            if (bm) dymax_note(*bm, tile, tile_begin, f >> 1, acc, valid && f < IN, j, *bad);
        }
    }

    static_assert(N::N_PARAMS <= kBwdWaves * B::PER_WAVE, "reduction buffer");
    float* red = stage;
    __syncthreads();
    for (int wv = 0; wv < kBwdWaves; ++wv) {
        if (wave == wv) {
            merge_dw<N::OT, N::IT>(red + N::OFF_W1, dW1, W, IN, q, j, wv == 0);
#pragma unroll
            for (int k = 1; k < D; ++k)
                merge_dw<N::OT, N::OT>(red + N::OFF_H + (k - 1) * W * W, dWh[k - 1], W, W, q, j, wv == 0);
            merge_dw<1, N::OT>(red + N::OFF_OUT, dWo, 4, W, q, j, wv == 0);
        }
        __syncthreads();
    }
    for (int p = threadIdx.x; p < N::N_PARAMS; p += blockDim.x) dst[p] = red[p];
}

template <int IN, int W, int D, class P>
__global__ __launch_bounds__(64 * kBwdWaves) void k_mlp_bwd_lp(const float* __restrict__ w,
                                                               const float2* __restrict__ y,
                                                               const float4* __restrict__ dout, int64_t n_s,
                                                               float2* __restrict__ dy, float* __restrict__ partial)
{
    using N = NetLp<IN, W, D>;
    extern __shared__ __align__(16) unsigned char smem_lp[];
    load_fragments_lp<IN, W, D, P>(w, reinterpret_cast<typename P::vec*>(smem_lp), N::N_ALL);
    __syncthreads();
    const int64_t wave0 = (int64_t)blockIdx.x * kBwdWaves + (threadIdx.x >> 6);
    mlp_bwd_tiles_lp<IN, W, D, P>(smem_lp, y, dout, n_s, dy, partial + (int64_t)blockIdx.x * N::N_PARAMS, wave0,
                                  (n_s + 15) / 16, (int64_t)gridDim.x * kBwdWaves);
}

template <int IN, int W, int D, class P>
__global__ __launch_bounds__(64 * kBwdWaves) void k_mlp_bwd_lp_batch(const MlpWork* __restrict__ work,
                                                                     const float* __restrict__ params,
                                                                     const float2* __restrict__ y,
                                                                     const float4* __restrict__ dout,
                                                                     float2* __restrict__ dy,
                                                                     float* __restrict__ partial, int64_t slot_stride,
                                                                     float* __restrict__ block_max,
                                                                     int32_t* __restrict__ nonfinite)
{
    using N = NetLp<IN, W, D>;
    static_assert(IN / 2 <= kBmLevels, "levels");
    extern __shared__ __align__(16) unsigned char smem_lp[];
    __shared__ DyMaxLds bm;
    const MlpWork wk = work[blockIdx.x];
    dymax_clear(bm);
    load_fragments_lp<IN, W, D, P>(params + wk.w_off, reinterpret_cast<typename P::vec*>(smem_lp), N::N_ALL);
    __syncthreads();
    bool bad = false;
    mlp_bwd_tiles_lp<IN, W, D, P>(smem_lp, y + wk.y_off / 2, dout + wk.s_off, wk.n_s, dy + wk.y_off / 2,
                                  partial + (int64_t)blockIdx.x * slot_stride, wk.tile_begin + (threadIdx.x >> 6),
                                  wk.tile_end, kBwdWaves, &bm, wk.tile_begin, &bad);
    if (bad && nonfinite) *nonfinite = 1;
    __syncthreads();
    dymax_flush(bm, block_max + wk.bmax_off, wk.n_sblocks, IN / 2, wk.tile_begin, wk.tile_end);
}

// ---------------------------------------------------------------- 128 wide
// As in the FP32 form: the forward stores the hidden activations (in the
// MFMA type, each unit's ReLU decision beside them as bits: relu_mask_bits); a chain
// kernel with only the transposed fragments writes every layer's delta and
// dy; a weight-gradient kernel contracts deltas with activations over the
// block's samples (operands rounded to the MFMA type, FP32 accumulation),
// the waves splitting the output rows.
constexpr int kWideWavesLp = 4;
constexpr int kDwThreadsLp = 64 * kWideWavesLp;

// act16 / dlt16: the activations and deltas in the layout of wide_vec.
template <int IN, int W, int D, class P>
__device__ __forceinline__ void mlp_chain_bwd_tiles_lp(const typename P::vec* __restrict__ bfrag, const float4* __restrict__ sc,
                                       const float4* __restrict__ dout, const typename P::vec* __restrict__ act16,
                                       typename P::vec* __restrict__ dlt16, int64_t n_s, float2* __restrict__ dy,
                                       int64_t tile0, int64_t end, int64_t step, DyMaxLds* bm = nullptr,
                                       int64_t tile_begin = 0, bool* bad = nullptr)
{
    using N = NetLp<IN, W, D>;
    constexpr int BO = 0, BH = N::BH - N::N_FWD, B1 = N::B1 - N::N_FWD;
    const int lane = threadIdx.x & 63, q = lane >> 4, j = lane & 15;
    static_assert(N::OT * 4 <= 32, "mask bits per lane");
    const uint32_t* masks = wide_masks<W, D, P>(const_cast<typename P::vec*>(act16), n_s);
    // a tile's loads (head adjoint inputs on lanes q == 0, every layer's mask
    // word), issued one tile ahead so they overlap the current tile's work
    float4 gn = make_float4(0.0f, 0.0f, 0.0f, 0.0f), vn = gn;
    uint32_t mn[D];
    auto load_tile = [&](int64_t t) {
        const int64_t st = t * 16 + j;
        const bool ok = t < end && st < n_s;
        gn = vn = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (ok && q == 0) {
            gn = dout[st];
            vn = sc[st];
        }
#pragma unroll
        for (int k = 0; k < D; ++k) mn[k] = ok ? masks[((int64_t)k * n_s + st) * 4 + q] : 0u;
    };
    load_tile(tile0);
    for (int64_t tile = tile0; tile < end; tile += step) {
        const int64_t s = tile * 16 + j;
        const bool valid = s < n_s;
        const float4 g = gn, v = vn;
        uint32_t mc[D];
#pragma unroll
        for (int k = 0; k < D; ++k) mc[k] = mn[k];
        load_tile(tile + step);
        const floatx4 dO = {g.x * v.x, g.y * v.y * (1.0f - v.y), g.z * v.z * (1.0f - v.z), g.w * v.w * (1.0f - v.w)};
        const typename P::vec dOp = pack<P>(dO);
        floatx4 delta[N::OT];
        auto vi = [&](int k, int to) { return wide_vec<W>(k, n_s, s, to, q); };
        auto mask_of = [&](int k) { return mc[k]; };
        uint32_t mk = mask_of(D - 1);
#pragma unroll
        for (int to = 0; to < N::OT; ++to) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = P::mma(bfrag[(BO + to) * 64 + lane], dOp, acc);
            delta[to] = mask_by_bits(acc, mk, to);
            if (valid) dlt16[vi(D - 1, to)] = pack<P>(delta[to]);
        }
#pragma unroll
        for (int k = D - 1; k >= 1; --k) {
            mk = mask_of(k - 1);
            typename P::vec dp[N::OT];
#pragma unroll
            for (int ti = 0; ti < N::OT; ++ti) dp[ti] = pack<P>(delta[ti]);
            floatx4 nd[N::OT];
            layer_lp_ks_outer<P, N::OT, N::OT>(bfrag, lane, BH + (k - 1) * N::OT * N::OT, N::OT, dp, nd);
#pragma unroll
            for (int to = 0; to < N::OT; ++to) {
                delta[to] = mask_by_bits(nd[to], mk, to);
                if (valid) dlt16[vi(k - 1, to)] = pack<P>(delta[to]);
            }
        }
        typename P::vec dp[N::OT];
#pragma unroll
        for (int ti = 0; ti < N::OT; ++ti) dp[ti] = pack<P>(delta[ti]);
        floatx4 gy[N::IT];
        layer_lp_ks_outer<P, N::IT, N::OT>(bfrag, lane, B1, N::OT, dp, gy);
#pragma unroll
        for (int to = 0; to < N::IT; ++to) {
            const int f = 16 * to + 4 * q;
            if (valid && f < IN) {
                dy[(int64_t)(f >> 1) * n_s + s] = make_float2(gy[to][0], gy[to][1]);
                dy[(int64_t)((f >> 1) + 1) * n_s + s] = make_float2(gy[to][2], gy[to][3]);
            }
            if (bm) dymax_note(*bm, tile, tile_begin, f >> 1, gy[to], valid && f < IN, j, *bad);
        }
    }
}

// Weight gradient over samples [s_begin, s_end), staged kDwChunk samples at
// a time in LDS: MFMA K = 16 consecutive samples (lane q holds samples
// 4q .. 4q + 3 of the group of 16), operands rounded to the MFMA type.
// The chunk of samples is staged in 16-bit form, neuron-major: row n of a
// staged array holds neuron (or feature) n of the chunk's kDwChunk samples,
// so the 4 consecutive samples an MFMA operand needs in a lane are one 8-byte
// LDS read.  Rows are padded to kDwRowLp halfwords (80 bytes) to spread the 16
// rows a wave reads over the banks.  Layout, in halfwords:
//   DL [D][W][row]  deltas      AC [D][W][row]  activations
//   Y  [32][row]    inputs (rows >= IN zero)
//   DO [16][row]    head adjoint (rows >= 4 zero, written once)
constexpr int kDwRowLp = kDwChunk + 8;

template <int W, int D>
struct DwStageLp {
    static constexpr int DL = 0;
    static constexpr int AC = DL + D * W * kDwRowLp;
    static constexpr int Y = AC + D * W * kDwRowLp;
    static constexpr int DO = Y + 32 * kDwRowLp;
    static constexpr int HALVES = DO + 16 * kDwRowLp;
};

// 4 x 4 transpose of 16-bit values: in[r] holds columns 0..3 of row r (two
// per 32-bit word); out[c] holds rows 0..3 of column c.
__device__ __forceinline__ void transpose4x4_16(const uint2 (&in)[4], uint2 (&out)[4])
{
    out[0] = make_uint2((in[0].x & 0xffffu) | (in[1].x << 16), (in[2].x & 0xffffu) | (in[3].x << 16));
    out[1] = make_uint2((in[0].x >> 16) | (in[1].x & 0xffff0000u), (in[2].x >> 16) | (in[3].x & 0xffff0000u));
    out[2] = make_uint2((in[0].y & 0xffffu) | (in[1].y << 16), (in[2].y & 0xffffu) | (in[3].y << 16));
    out[3] = make_uint2((in[0].y >> 16) | (in[1].y & 0xffff0000u), (in[2].y >> 16) | (in[3].y & 0xffff0000u));
}

template <class P>
__device__ __forceinline__ uint2 bits(typename P::vec v)
{
    return __builtin_bit_cast(uint2, v);
}

// Staging of samples [s0, min(s0 + kDwChunk, s_end)) (zeros past the end),
// in two halves so the next chunk's global loads overlap the current chunk's
// MFMAs: dw_load_lp reads a thread's share into registers, dw_store_lp
// writes it to LDS.  act16 / dlt16: as laid out by wide_vec; y: level-major
// [L][n_s][2].  kDwThreadsLp threads.
template <int W, int D>
struct DwRegsLp {
    static constexpr int SG = kDwChunk / 4;              // 4-sample groups per chunk
    static constexpr int V = W / 4;                      // 4-neuron groups per row
    static constexpr int N_AD = 2 * D * SG * V;          // 4 x 4 blocks of deltas and activations
    static constexpr int PER = (N_AD + kDwThreadsLp - 1) / kDwThreadsLp;
    uint2 ad[PER][4];  // rows r = 0..3 (samples) of each block
    float2 yv[4];      // features 2l, 2l + 1 of 4 samples (threads < 16 SG)
    float4 g, v;       // head adjoint inputs of one sample (threads < kDwChunk)
};

template <int IN, int W, int D, class P>
__device__ __forceinline__ void dw_load_lp(DwRegsLp<W, D>& R, const float* __restrict__ y,
                                           const float4* __restrict__ sc, const float4* __restrict__ dout,
                                           const typename P::vec* __restrict__ act16,
                                           const typename P::vec* __restrict__ dlt16, int64_t n_s, int64_t s0,
                                           int64_t s_end)
{
    using Rg = DwRegsLp<W, D>;
#pragma unroll
    for (int u = 0; u < Rg::PER; ++u) {
        const int i = threadIdx.x + kDwThreadsLp * u;
        const int arr = i / (D * Rg::SG * Rg::V), rem = i % (D * Rg::SG * Rg::V);
        const int k = rem / (Rg::SG * Rg::V), r2 = rem % (Rg::SG * Rg::V), sg = r2 / Rg::V, c = r2 % Rg::V;
        const typename P::vec* src = arr == 0 ? dlt16 : act16;
        // the 4 samples of the group are consecutive in one tile: two 16-byte loads
        const int64_t sb = s0 + 4 * sg;
        uint4 w0 = make_uint4(0u, 0u, 0u, 0u), w1 = w0;
        if (i < Rg::N_AD && sb < s_end) {
            const uint4* p = reinterpret_cast<const uint4*>(src + wide_vec<W>(k, n_s, sb, c >> 2, c & 3));
            w0 = p[0];
            w1 = p[1];
        }
        R.ad[u][0] = sb < s_end ? make_uint2(w0.x, w0.y) : make_uint2(0u, 0u);
        R.ad[u][1] = sb + 1 < s_end ? make_uint2(w0.z, w0.w) : make_uint2(0u, 0u);
        R.ad[u][2] = sb + 2 < s_end ? make_uint2(w1.x, w1.y) : make_uint2(0u, 0u);
        R.ad[u][3] = sb + 3 < s_end ? make_uint2(w1.z, w1.w) : make_uint2(0u, 0u);
    }
    {
        const int l = threadIdx.x / Rg::SG, sg = threadIdx.x % Rg::SG;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t s = s0 + 4 * sg + r;
            R.yv[r] = threadIdx.x < 16 * Rg::SG && s < s_end && 2 * l < IN
                          ? reinterpret_cast<const float2*>(y)[(int64_t)l * n_s + s]
                          : make_float2(0.0f, 0.0f);
        }
    }
    {
        const int64_t s = s0 + threadIdx.x;
        const bool ok = threadIdx.x < kDwChunk && s < s_end;
        R.g = ok ? dout[s] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        R.v = ok ? sc[s] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
}

template <int IN, int W, int D, class P>
__device__ __forceinline__ void dw_store_lp(uint16_t* __restrict__ lds, const DwRegsLp<W, D>& R)
{
    using St = DwStageLp<W, D>;
    using Rg = DwRegsLp<W, D>;
    // activations and deltas: one 4 x 4 block (4 samples x 4 neurons) per item
#pragma unroll
    for (int u = 0; u < Rg::PER; ++u) {
        const int i = threadIdx.x + kDwThreadsLp * u;
        if (i < Rg::N_AD) {
            const int arr = i / (D * Rg::SG * Rg::V), rem = i % (D * Rg::SG * Rg::V);
            const int k = rem / (Rg::SG * Rg::V), r2 = rem % (Rg::SG * Rg::V), sg = r2 / Rg::V, c = r2 % Rg::V;
            uint2 out[4];
            transpose4x4_16(R.ad[u], out);
            uint16_t* base = lds + (arr == 0 ? St::DL : St::AC) + (k * W + 4 * c) * kDwRowLp + 4 * sg;
#pragma unroll
            for (int n = 0; n < 4; ++n) *reinterpret_cast<uint2*>(base + n * kDwRowLp) = out[n];
        }
    }
    // inputs: features 2l, 2l + 1 of 4 samples per item (rounded to P)
    if (threadIdx.x < 16 * Rg::SG) {
        const int l = threadIdx.x / Rg::SG, sg = threadIdx.x % Rg::SG;
        uint16_t* base = lds + St::Y + (2 * l) * kDwRowLp + 4 * sg;
        *reinterpret_cast<uint2*>(base) = bits<P>(pack<P>(R.yv[0].x, R.yv[1].x, R.yv[2].x, R.yv[3].x));
        *reinterpret_cast<uint2*>(base + kDwRowLp) = bits<P>(pack<P>(R.yv[0].y, R.yv[1].y, R.yv[2].y, R.yv[3].y));
    }
    // head adjoint (d sigma / d o0 = sigma, d c / d o = c (1 - c)) of one sample
    if (threadIdx.x < kDwChunk) {
        const float4 g = R.g, v = R.v;
        const float o[4] = {g.x * v.x, g.y * v.y * (1.0f - v.y), g.z * v.z * (1.0f - v.z), g.w * v.w * (1.0f - v.w)};
#pragma unroll
        for (int n = 0; n < 4; ++n)
            lds[St::DO + n * kDwRowLp + threadIdx.x] = __builtin_bit_cast(uint16_t, P::cvt(o[n]));
    }
}

// Weight gradient over samples [s_begin, s_end): dW = sum_s delta(s) h(s)^T
// per layer, MFMA K = 16 consecutive samples (lane q holds samples
// 4q .. 4q + 3 of the group of 16), operands rounded to the MFMA type, the 4
// waves splitting the output rows.  One partial per block.
template <int IN, int W, int D, class P>
__device__ __forceinline__ void mlp_dw_range_lp(uint16_t* __restrict__ lds, const float* __restrict__ y, const float4* __restrict__ sc,
                                const float4* __restrict__ dout, const typename P::vec* __restrict__ act16,
                                const typename P::vec* __restrict__ dlt16, int64_t n_s, int64_t s_begin,
                                int64_t s_end, float* __restrict__ dst)
{
    using N = NetLp<IN, W, D>;
    using St = DwStageLp<W, D>;
    constexpr int RT = N::OT / kWideWavesLp;
    static_assert(N::OT % kWideWavesLp == 0 && IN <= 32 && N::IT <= 2, "rows per wave, inputs");
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4, j = lane & 15;
    floatx4 aH[D > 1 ? D - 1 : 1][RT][N::OT], a1[RT][N::IT], aO[RT];
#pragma unroll
    for (int a = 0; a < RT; ++a) {
        aO[a] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t < N::IT; ++t) a1[a][t] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < (D > 1 ? D - 1 : 1); ++k)
#pragma unroll
            for (int t = 0; t < N::OT; ++t) aH[k][a][t] = {0.0f, 0.0f, 0.0f, 0.0f};
    }
    // rows 4..15 of the head adjoint stay zero (the A operand of the head's
    // 16-row tile); rows 0..3 are restaged with every chunk
    for (int i = threadIdx.x; i < 12 * kDwRowLp; i += blockDim.x) lds[St::DO + 4 * kDwRowLp + i] = 0;
    // 4 samples of staged row `row`, as an MFMA operand
    auto op = [&](int base, int row, int k0) {
        return __builtin_bit_cast(typename P::vec, *reinterpret_cast<const uint2*>(lds + base + row * kDwRowLp + k0));
    };
    static_assert(kDwThreadsLp >= 16 * (kDwChunk / 4) && kDwThreadsLp >= kDwChunk, "staging threads");
    DwRegsLp<W, D> R;
    if (s_begin < s_end) dw_load_lp<IN, W, D, P>(R, y, sc, dout, act16, dlt16, n_s, s_begin, s_end);
    for (int64_t c0 = s_begin; c0 < s_end; c0 += kDwChunk) {
        dw_store_lp<IN, W, D, P>(lds, R);
        __syncthreads();
        if (c0 + kDwChunk < s_end) dw_load_lp<IN, W, D, P>(R, y, sc, dout, act16, dlt16, n_s, c0 + kDwChunk, s_end);
#pragma unroll 1
        for (int ks = 0; ks < kDwChunk / 16; ++ks) {  // not unrolled: bounds the operands in flight
            const int k0 = 16 * ks + 4 * q;
            const typename P::vec dOp = op(St::DO, j, k0);
#pragma unroll
            for (int a = 0; a < RT; ++a)
                aO[a] = P::mma(dOp, op(St::AC + (D - 1) * W * kDwRowLp, 16 * (RT * wave + a) + j, k0), aO[a]);
#pragma unroll
            for (int k = 1; k < D; ++k) {
                typename P::vec av[RT];
#pragma unroll
                for (int a = 0; a < RT; ++a) av[a] = op(St::DL + k * W * kDwRowLp, 16 * (RT * wave + a) + j, k0);
#pragma unroll
                for (int t = 0; t < N::OT; ++t) {
                    const typename P::vec bv = op(St::AC + (k - 1) * W * kDwRowLp, 16 * t + j, k0);
#pragma unroll
                    for (int a = 0; a < RT; ++a) aH[k - 1][a][t] = P::mma(av[a], bv, aH[k - 1][a][t]);
                }
            }
            {
                typename P::vec av[RT], bv[N::IT];
#pragma unroll
                for (int a = 0; a < RT; ++a) av[a] = op(St::DL, 16 * (RT * wave + a) + j, k0);
#pragma unroll
                for (int t = 0; t < N::IT; ++t) bv[t] = op(St::Y, 16 * t + j, k0);
#pragma unroll
                for (int a = 0; a < RT; ++a)
#pragma unroll
                    for (int t = 0; t < N::IT; ++t) a1[a][t] = P::mma(av[a], bv[t], a1[a][t]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * (RT * wave + a) + 4 * q + r;
#pragma unroll
            for (int t = 0; t < N::IT; ++t) {
                const int col = 16 * t + j;
                if (col < IN) dst[N::OFF_W1 + row * IN + col] = a1[a][t][r];
            }
#pragma unroll
            for (int k = 1; k < D; ++k)
#pragma unroll
                for (int t = 0; t < N::OT; ++t) dst[N::OFF_H + (k - 1) * W * W + row * W + 16 * t + j] = aH[k - 1][a][t][r];
            if (q == 0) dst[N::OFF_OUT + r * W + 16 * (RT * wave + a) + j] = aO[a][r];
        }
}

template <int IN, int W, int D>
constexpr size_t dw_lds_bytes_lp()
{
    return sizeof(uint16_t) * (size_t)DwStageLp<W, D>::HALVES;
}

template <int IN, int W, int D, class P>
__global__ __launch_bounds__(256) void k_mlp_chain_bwd_lp(const float* __restrict__ w, const float4* __restrict__ sc,
                                                          const float4* __restrict__ dout, float* __restrict__ act,
                                                          int64_t n_s, float2* __restrict__ dy)
{
    using N = NetLp<IN, W, D>;
    extern __shared__ __align__(16) unsigned char smem_b[];
    typename P::vec* frag = reinterpret_cast<typename P::vec*>(smem_b);
    load_fragments_lp<IN, W, D, P>(w, frag, N::N_ALL - N::N_FWD, N::N_FWD);
    __syncthreads();
    const int64_t wave0 = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    typename P::vec* a16 = reinterpret_cast<typename P::vec*>(act);
    mlp_chain_bwd_tiles_lp<IN, W, D, P>(frag, sc, dout, a16, wide_deltas<W, D, P>(a16, n_s), n_s, dy, wave0,
                                        (n_s + 15) / 16, (int64_t)gridDim.x * (blockDim.x / 64));
}

template <int IN, int W, int D, class P>
__global__ __launch_bounds__(256) void k_mlp_chain_bwd_lp_batch(const MlpWork* __restrict__ work,
                                                                const float* __restrict__ params,
                                                                const float4* __restrict__ sc,
                                                                const float4* __restrict__ dout,
                                                                float* __restrict__ act, float2* __restrict__ dy,
                                                                float* __restrict__ block_max,
                                                                int32_t* __restrict__ nonfinite)
{
    using N = NetLp<IN, W, D>;
    static_assert(IN / 2 <= kBmLevels, "levels");
    extern __shared__ __align__(16) unsigned char smem_b[];
    __shared__ DyMaxLds bm;
    typename P::vec* frag = reinterpret_cast<typename P::vec*>(smem_b);
    const MlpWork wk = work[blockIdx.x];
    dymax_clear(bm);
    load_fragments_lp<IN, W, D, P>(params + wk.w_off, frag, N::N_ALL - N::N_FWD, N::N_FWD);
    __syncthreads();
    typename P::vec* a16 = reinterpret_cast<typename P::vec*>(act + wk.a_off);
    bool bad = false;
    mlp_chain_bwd_tiles_lp<IN, W, D, P>(frag, sc + wk.s_off, dout + wk.s_off, a16, wide_deltas<W, D, P>(a16, wk.n_s),
                                        wk.n_s, dy + wk.y_off / 2, wk.tile_begin + (threadIdx.x >> 6), wk.tile_end,
                                        blockDim.x / 64, &bm, wk.tile_begin, &bad);
    if (bad && nonfinite) *nonfinite = 1;
    __syncthreads();
    dymax_flush(bm, block_max + wk.bmax_off, wk.n_sblocks, IN / 2, wk.tile_begin, wk.tile_end);
}

template <int IN, int W, int D, class P>
__global__ __launch_bounds__(64 * kWideWavesLp) void k_mlp_dw_lp(const float* __restrict__ y,
                                                                 const float4* __restrict__ sc,
                                                                 const float4* __restrict__ dout,
                                                                 const float* __restrict__ act, int64_t n_s,
                                                                 int64_t tiles_per_block, float* __restrict__ partial)
{
    using N = NetLp<IN, W, D>;
    extern __shared__ __align__(16) uint16_t dw_lds[];
    const int64_t b = (int64_t)blockIdx.x * tiles_per_block * 16;
    const int64_t e = min(b + tiles_per_block * 16, n_s);
    const typename P::vec* a16 = reinterpret_cast<const typename P::vec*>(act);
    mlp_dw_range_lp<IN, W, D, P>(dw_lds, y, sc, dout, a16, wide_deltas<W, D, P>(const_cast<typename P::vec*>(a16), n_s), n_s, b, e,
                                 partial + (int64_t)blockIdx.x * N::N_PARAMS);
}

template <int IN, int W, int D, class P>
__global__ __launch_bounds__(64 * kWideWavesLp) void k_mlp_dw_lp_batch(const MlpWork* __restrict__ work,
                                                                       const float* __restrict__ y,
                                                                       const float4* __restrict__ sc,
                                                                       const float4* __restrict__ dout,
                                                                       const float* __restrict__ act,
                                                                       float* __restrict__ partial, int64_t slot_stride)
{
    extern __shared__ __align__(16) uint16_t dw_lds[];
    const MlpWork wk = work[blockIdx.x];
    const int64_t b = wk.tile_begin * 16, e = min(wk.tile_end * 16, wk.n_s);
    const typename P::vec* a16 = reinterpret_cast<const typename P::vec*>(act + wk.a_off);
    mlp_dw_range_lp<IN, W, D, P>(dw_lds, y + wk.y_off, sc + wk.s_off, dout + wk.s_off, a16,
                                 wide_deltas<W, D, P>(const_cast<typename P::vec*>(a16), wk.n_s), wk.n_s, b, e,
                                 partial + (int64_t)blockIdx.x * slot_stride);
}

template <class K>
hipError_t set_lds_lp(K kern, size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int IN, int W, int D, class P>
size_t fwd_lds_lp()
{
    return sizeof(typename P::vec) * (size_t)NetLp<IN, W, D>::N_FWD * 64;
}

template <int IN, int W, int D, class P>
size_t chain_lds_lp()
{
    return sizeof(typename P::vec) * (size_t)(NetLp<IN, W, D>::N_ALL - NetLp<IN, W, D>::N_FWD) * 64;
}

template <int IN, int W, int D, class P>
size_t bwd_lds_lp()
{
    return sizeof(typename P::vec) * (size_t)NetLp<IN, W, D>::N_ALL * 64 +
           sizeof(float) * (size_t)kBwdWaves * BwdLdsLp<IN, W, D>::PER_WAVE;
}

template <int IN, int W, int D, class P>
hipError_t fwd_lp(const float* w, const float* y, int64_t n_s, float* sc, float* act, hipStream_t s)
{
    const int64_t n_tiles = (n_s + 15) / 16;
    int64_t blocks = (n_tiles + 3) / 4;
    blocks = blocks > 2048 ? 2048 : blocks;
    const size_t lds = fwd_lds_lp<IN, W, D, P>();
    hipError_t e = set_lds_lp(k_mlp_fwd_lp<IN, W, D, P>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_mlp_fwd_lp<IN, W, D, P>), dim3((uint32_t)blocks), dim3(256), lds, s, w, (const float2*)y,
                       n_s, (float4*)sc, W >= kWideWidth ? act : nullptr);
    return hipGetLastError();
}

template <int IN, int W, int D, class P>
hipError_t bwd_lp(const float* w, const float* y, const float* dout, const float* sc, int64_t n_s, float* dy,
                  float* partial, float* act, hipStream_t s)
{
    if constexpr (W >= kWideWidth) {
        const int64_t n_tiles = (n_s + 15) / 16;
        int64_t blocks = (n_tiles + 3) / 4;
        blocks = blocks > 2048 ? 2048 : blocks;
        const size_t lds = chain_lds_lp<IN, W, D, P>();
        hipError_t e = set_lds_lp(k_mlp_chain_bwd_lp<IN, W, D, P>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_mlp_chain_bwd_lp<IN, W, D, P>), dim3((uint32_t)blocks), dim3(256), lds, s, w,
                           (const float4*)sc, (const float4*)dout, act, n_s, (float2*)dy);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int nb = bwd_blocks(n_s);
        const int64_t per = (n_tiles + nb - 1) / nb;
        const size_t dwl = dw_lds_bytes_lp<IN, W, D>();
        if ((e = set_lds_lp(k_mlp_dw_lp<IN, W, D, P>, dwl)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_mlp_dw_lp<IN, W, D, P>), dim3((uint32_t)nb), dim3(64 * kWideWavesLp), dwl, s, y,
                           (const float4*)sc, (const float4*)dout, act, n_s, per, partial);
        return hipGetLastError();
    } else {
        const size_t lds = bwd_lds_lp<IN, W, D, P>();
        auto kern = k_mlp_bwd_lp<IN, W, D, P>;
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3((uint32_t)bwd_blocks(n_s)), dim3(64 * kBwdWaves), lds, s, w, (const float2*)y,
                           (const float4*)dout, n_s, (float2*)dy, partial);
        return hipGetLastError();
    }
}

template <int IN, int W, int D, class P>
hipError_t fwd_lp_batch(const MlpWork* work, int n_blocks, const float* params, const float* y, float* sc, float* act,
                        hipStream_t s)
{
    const size_t lds = fwd_lds_lp<IN, W, D, P>();
    hipError_t e = set_lds_lp(k_mlp_fwd_lp_batch<IN, W, D, P>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_mlp_fwd_lp_batch<IN, W, D, P>), dim3((uint32_t)n_blocks), dim3(256), lds, s, work, params,
                       (const float2*)y, (float4*)sc, W >= kWideWidth ? act : nullptr);
    return hipGetLastError();
}

template <int IN, int W, int D, class P>
hipError_t bwd_lp_batch(const MlpWork* work, int n_blocks, const float* params, const float* y, const float* dout,
                        const float* sc, float* dy, float* partial, int64_t slot_stride, float* act, float* block_max,
                        int32_t* nonfinite, hipStream_t s)
{
    if constexpr (W >= kWideWidth) {
        const size_t lds = chain_lds_lp<IN, W, D, P>();
        hipError_t e = set_lds_lp(k_mlp_chain_bwd_lp_batch<IN, W, D, P>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_mlp_chain_bwd_lp_batch<IN, W, D, P>), dim3((uint32_t)n_blocks), dim3(256), lds, s, work,
                           params, (const float4*)sc, (const float4*)dout, act, (float2*)dy, block_max, nonfinite);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const size_t dwl = dw_lds_bytes_lp<IN, W, D>();
        if ((e = set_lds_lp(k_mlp_dw_lp_batch<IN, W, D, P>, dwl)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_mlp_dw_lp_batch<IN, W, D, P>), dim3((uint32_t)n_blocks), dim3(64 * kWideWavesLp), dwl, s,
                           work, y, (const float4*)sc, (const float4*)dout, act, partial, slot_stride);
        return hipGetLastError();
    } else {
        const size_t lds = bwd_lds_lp<IN, W, D, P>();
        auto kern = k_mlp_bwd_lp_batch<IN, W, D, P>;
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3((uint32_t)n_blocks), dim3(64 * kBwdWaves), lds, s, work, params,
                           (const float2*)y, (const float4*)dout, (float2*)dy, partial, slot_stride, block_max,
                           nonfinite);
        return hipGetLastError();
    }
}

#define PRENOM_FOR_EACH_MLP_LP(X) \
    X(16, 32, 1) \
    X(16, 32, 2) \
    X(16, 64, 1) \
    X(16, 64, 2) \
    X(16, 128, 1) \
    X(16, 128, 2) \
    X(24, 32, 1) \
    X(24, 32, 2) \
    X(24, 64, 1) \
    X(24, 64, 2) \
    X(24, 128, 1) \
    X(24, 128, 2) \
    X(32, 32, 1) \
    X(32, 32, 2) \
    X(32, 64, 1) \
    X(32, 64, 2) \
    X(32, 128, 1) \
    X(32, 128, 2)

template <class P>
hipError_t fwd_dispatch(const MlpShape& m, const float* w, const float* y, int64_t n_s, float* sc, float* act,
                        hipStream_t s)
{
#define X(I, Wd, Dp) \
    if (m.in_dim == I && m.width == Wd && m.hidden == Dp) return fwd_lp<I, Wd, Dp, P>(w, y, n_s, sc, act, s);
    PRENOM_FOR_EACH_MLP_LP(X)
#undef X
    return hipErrorInvalidValue;
}

template <class P>
hipError_t bwd_dispatch(const MlpShape& m, const float* w, const float* y, const float* dout, const float* sc,
                        int64_t n_s, float* dy, float* partial, float* act, hipStream_t s)
{
#define X(I, Wd, Dp)                                        \
    if (m.in_dim == I && m.width == Wd && m.hidden == Dp) \
        return bwd_lp<I, Wd, Dp, P>(w, y, dout, sc, n_s, dy, partial, act, s);
    PRENOM_FOR_EACH_MLP_LP(X)
#undef X
    return hipErrorInvalidValue;
}

template <class P>
hipError_t fwd_batch_dispatch(const MlpShape& m, const MlpWork* work, int n_blocks, const float* params, const float* y,
                              float* sc, float* act, hipStream_t s)
{
#define X(I, Wd, Dp)                                        \
    if (m.in_dim == I && m.width == Wd && m.hidden == Dp) \
        return fwd_lp_batch<I, Wd, Dp, P>(work, n_blocks, params, y, sc, act, s);
    PRENOM_FOR_EACH_MLP_LP(X)
#undef X
    return hipErrorInvalidValue;
}

template <class P>
hipError_t bwd_batch_dispatch(const MlpShape& m, const MlpWork* work, int n_blocks, const float* params,
                              const float* y, const float* dout, const float* sc, float* dy, float* partial,
                              int64_t slot_stride, float* act, float* block_max, int32_t* nonfinite, hipStream_t s)
{
#define X(I, Wd, Dp)                                                                                     \
    if (m.in_dim == I && m.width == Wd && m.hidden == Dp)                                              \
        return bwd_lp_batch<I, Wd, Dp, P>(work, n_blocks, params, y, dout, sc, dy, partial, slot_stride, act, \
                                          block_max, nonfinite, s);
    PRENOM_FOR_EACH_MLP_LP(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_mlp_fwd_lp(const MlpShape& m, const float* w, const float* y, int64_t n_s, float* sc, float* act,
                             hipStream_t s)
{
    if (n_s == 0) return hipSuccess;
    if (m.dtype == PRENOM_BF16) return fwd_dispatch<Bf16Op>(m, w, y, n_s, sc, act, s);
    if (m.dtype == PRENOM_F16) return fwd_dispatch<F16Op>(m, w, y, n_s, sc, act, s);
    return hipErrorInvalidValue;
}

hipError_t launch_mlp_bwd_lp(const MlpShape& m, const float* w, const float* y, const float* dout, const float* sc,
                             int64_t n_s, float* dy, float* partial, float* act, hipStream_t s)
{
    if (n_s == 0) return hipSuccess;
    if (m.dtype == PRENOM_BF16) return bwd_dispatch<Bf16Op>(m, w, y, dout, sc, n_s, dy, partial, act, s);
    if (m.dtype == PRENOM_F16) return bwd_dispatch<F16Op>(m, w, y, dout, sc, n_s, dy, partial, act, s);
    return hipErrorInvalidValue;
}

hipError_t launch_mlp_fwd_lp_batch(const MlpShape& m, const MlpWork* work, int n_blocks, const float* params,
                                   const float* y, float* sc, float* act, hipStream_t s)
{
    if (n_blocks == 0) return hipSuccess;
    if (m.dtype == PRENOM_BF16) return fwd_batch_dispatch<Bf16Op>(m, work, n_blocks, params, y, sc, act, s);
    if (m.dtype == PRENOM_F16) return fwd_batch_dispatch<F16Op>(m, work, n_blocks, params, y, sc, act, s);
    return hipErrorInvalidValue;
}

hipError_t launch_mlp_bwd_lp_batch(const MlpShape& m, const MlpWork* work, int n_blocks, const float* params,
                                   const float* y, const float* dout, const float* sc, float* dy, float* partial,
                                   int64_t slot_stride, float* act, float* block_max, int32_t* nonfinite,
                                   hipStream_t s)
{
    if (n_blocks == 0) return hipSuccess;
    if (m.dtype == PRENOM_BF16)
        return bwd_batch_dispatch<Bf16Op>(m, work, n_blocks, params, y, dout, sc, dy, partial, slot_stride, act,
                                          block_max, nonfinite, s);
    if (m.dtype == PRENOM_F16)
        return bwd_batch_dispatch<F16Op>(m, work, n_blocks, params, y, dout, sc, dy, partial, slot_stride, act,
                                         block_max, nonfinite, s);
    return hipErrorInvalidValue;
}

}  // namespace prenom

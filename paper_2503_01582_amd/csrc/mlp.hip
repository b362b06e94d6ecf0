// The shallow MLP of the object NeRF (Sec. III-B "Object-level NeRFs" and
// "Volume Rendering"): encoded position -> D bias-free ReLU layers of width W
// -> 4 linear outputs; density = exp(o0), colour = sigmoid(o1..3).
//
// Both passes run on the matrix cores with v_mfma_f32_16x16x4_f32, in the
// transposed form H^T = W X^T: a 16-sample tile is the N (column) dimension,
// neurons are rows.  Operand layouts of the 16x16x4 instruction (lane l,
// q = l/16, j = l%16):  A[i][k] at lane i + 16k, B[k][n] at lane n + 16k,
// D[i][n] at lane n + 16*(i/4), register i%4.  With that layout the output
// registers of one layer are directly the B operand of the next: register r of
// output tile ti holds neuron 16 ti + 4 q + r of sample j, so K-step (ti, r)
// of the next layer covers those neurons and the weight fragment is permuted
// to match.  Weights are permuted once per block into LDS "fragments" of 64
// floats (one value per lane), read conflict-free.
//
// Backward: the adjoint runs the same chain with W^T fragments; the weight
// gradient dW = delta h^T contracts over samples, so delta and h of the tile
// go through a per-wave LDS transpose and are accumulated in registers for all
// tiles the wave processes; the waves of a block then merge their dW in LDS
// (in wave order), each block writes one partial, and a reduction kernel sums
// the partials in FP64 into the gradient buffer.
#include "mlp_common.h"

namespace prenom {
namespace {

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int IN, int W, int D>
struct Net {
    static constexpr int KT1 = IN / 4;          // K-steps of layer 1
    static constexpr int OT = W / 16;           // 16-row tiles of a hidden layer
    static constexpr int KTH = W / 4;           // K-steps over a hidden layer
    static constexpr int IT = (IN + 15) / 16;   // 16-row tiles of the input
    // forward fragments
    static constexpr int F1 = 0;                         // [OT][KT1]
    static constexpr int FH = F1 + OT * KT1;             // [D-1][OT][KTH]
    static constexpr int FO = FH + (D - 1) * OT * KTH;   // [KTH]
    static constexpr int N_FWD = FO + KTH;
    // backward fragments
    static constexpr int BO = N_FWD;                     // [OT]
    static constexpr int BH = BO + OT;                   // [D-1][OT][KTH]
    static constexpr int B1 = BH + (D - 1) * OT * KTH;   // [IT][KTH]
    static constexpr int N_ALL = B1 + IT * KTH;
    // parameter offsets (row-major layers)
    static constexpr int OFF_W1 = 0;
    static constexpr int OFF_H = W * IN;                 // + (k-1)*W*W
    static constexpr int OFF_OUT = W * IN + (D - 1) * W * W;
    static constexpr int N_PARAMS = OFF_OUT + 4 * W;
    static_assert(IN % 4 == 0 && W % 16 == 0 && D >= 1, "shape");
};

// Builds weight fragments f0 .. f0 + n_frag - 1 of one block in LDS (at 0).
template <int IN, int W, int D>
__device__ __forceinline__ void load_fragments(const float* __restrict__ w, float* __restrict__ frag, int n_frag, int f0 = 0)
{
    using N = Net<IN, W, D>;
    for (int idx = threadIdx.x; idx < n_frag * 64; idx += blockDim.x) {
        const int f = f0 + (idx >> 6), l = idx & 63, q = l >> 4, j = l & 15;
        float v = 0.0f;
        if (f < N::FH) {  // W1[16 to + j][4 kk + q]
            const int to = f / N::KT1, kk = f % N::KT1;
            v = w[N::OFF_W1 + (16 * to + j) * IN + 4 * kk + q];
        } else if (f < N::FO) {  // Wk[16 to + j][16 ti + 4 q + r]
            const int g = f - N::FH, k = g / (N::OT * N::KTH), rem = g % (N::OT * N::KTH);
            const int to = rem / N::KTH, ks = rem % N::KTH, ti = ks >> 2, r = ks & 3;
            v = w[N::OFF_H + k * W * W + (16 * to + j) * W + 16 * ti + 4 * q + r];
        } else if (f < N::N_FWD) {  // Wout[j][16 ti + 4 q + r], rows >= 4 zero
            const int ks = f - N::FO, ti = ks >> 2, r = ks & 3;
            v = j < 4 ? w[N::OFF_OUT + j * W + 16 * ti + 4 * q + r] : 0.0f;
        } else if (f < N::BH) {  // Wout^T: A[i=j][k=q] = Wout[q][16 to + j]
            const int to = f - N::BO;
            v = w[N::OFF_OUT + q * W + 16 * to + j];
        } else if (f < N::B1) {  // Wk^T: Wk[16 ti + 4 q + r][16 to + j]
            const int g = f - N::BH, k = g / (N::OT * N::KTH), rem = g % (N::OT * N::KTH);
            const int to = rem / N::KTH, ks = rem % N::KTH, ti = ks >> 2, r = ks & 3;
            v = w[N::OFF_H + k * W * W + (16 * ti + 4 * q + r) * W + 16 * to + j];
        } else {  // W1^T: W1[16 ti + 4 q + r][16 to + j], cols >= IN zero
            const int g = f - N::B1, to = g / N::KTH, ks = g % N::KTH, ti = ks >> 2, r = ks & 3;
            const int col = 16 * to + j;
            v = col < IN ? w[N::OFF_W1 + (16 * ti + 4 * q + r) * IN + col] : 0.0f;
        }
        frag[idx] = v;
    }
}

// Layer-1 B operand of K-step kk: feature 4 kk + q of sample s, from the
// level-major feature array y [L][n][2].
template <int KT1>
__device__ __forceinline__ void load_inputs(const float* __restrict__ y, int64_t n_s, int64_t s, bool valid,
                                            int q, float (&yb)[KT1])
{
#pragma unroll
    for (int kk = 0; kk < KT1; ++kk) {
        const int level = 2 * kk + (q >> 1), comp = q & 1;
        yb[kk] = valid ? y[((int64_t)level * n_s + s) * 2 + comp] : 0.0f;
    }
}

// acc[to] = sum_ks A(fragment f0 + to * stride + ks) x B_ks over one layer,
// K-steps outer and output tiles inner: OT independent accumulators
// interleave, hiding MFMA latency when one wave runs per SIMD (the widest
// MLP).  B_ks = b[ks >> 2][ks & 3] (a previous layer's output registers).
template <int OT, int KS>
__device__ __forceinline__ void layer_ks_outer(const float* __restrict__ frag, int lane, int f0, int stride,
                                               const floatx4 (&b)[KS / 4], floatx4 (&acc)[OT])
{
#pragma unroll
    for (int to = 0; to < OT; ++to) acc[to] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
        for (int to = 0; to < OT; ++to) acc[to] = mfma4(frag[(f0 + to * stride + ks) * 64 + lane], b[ks >> 2][ks & 3], acc[to]);
        // keep the scheduler from hoisting the fragment loads of the whole
        // layer (it would hold hundreds of them in registers)
        if ((ks & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
}

// Forward through the hidden layers and the head; hs[k] = output of layer k.
template <int IN, int W, int D>
__device__ __forceinline__ void mlp_chain(const float* __restrict__ frag, int lane,
                                          const float (&yb)[Net<IN, W, D>::KT1],
                                          floatx4 (&hs)[D][Net<IN, W, D>::OT], floatx4& o)
{
    using N = Net<IN, W, D>;
    if constexpr (W >= kWideWidth) {
        floatx4 acc[N::OT];
#pragma unroll
        for (int to = 0; to < N::OT; ++to) acc[to] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kk = 0; kk < N::KT1; ++kk)
#pragma unroll
            for (int to = 0; to < N::OT; ++to) acc[to] = mfma4(frag[(N::F1 + to * N::KT1 + kk) * 64 + lane], yb[kk], acc[to]);
#pragma unroll
        for (int to = 0; to < N::OT; ++to) hs[0][to] = relu4(acc[to]);
#pragma unroll
        for (int k = 1; k < D; ++k) {
            layer_ks_outer<N::OT, N::KTH>(frag, lane, N::FH + (k - 1) * N::OT * N::KTH, N::KTH, hs[k - 1], acc);
#pragma unroll
            for (int to = 0; to < N::OT; ++to) hs[k][to] = relu4(acc[to]);
        }
    } else {
#pragma unroll
        for (int to = 0; to < N::OT; ++to) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kk = 0; kk < N::KT1; ++kk) acc = mfma4(frag[(N::F1 + to * N::KT1 + kk) * 64 + lane], yb[kk], acc);
            hs[0][to] = relu4(acc);
        }
#pragma unroll
        for (int k = 1; k < D; ++k) {
#pragma unroll
            for (int to = 0; to < N::OT; ++to) {
                floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int ks = 0; ks < N::KTH; ++ks)
                    acc = mfma4(frag[(N::FH + ((k - 1) * N::OT + to) * N::KTH + ks) * 64 + lane], hs[k - 1][ks >> 2][ks & 3],
                                acc);
                hs[k][to] = relu4(acc);
                __builtin_amdgcn_sched_barrier(0);  // bound fragment-load hoisting (registers)
            }
        }
    }
    o = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < N::KTH; ++ks) o = mfma4(frag[(N::FO + ks) * 64 + lane], hs[D - 1][ks >> 2][ks & 3], o);
}

// Forward over the 16-sample tiles tile0, tile0 + step, ... < end of one
// object whose fragments are in LDS.  act (or null): the hidden activations
// are also stored, h_k of sample s at act[(k n_s + s) W ...] (rows of W floats).
template <int IN, int W, int D>
__device__ __forceinline__ void mlp_fwd_tiles(const float* __restrict__ frag, const float* __restrict__ y, int64_t n_s,
                                              float4* __restrict__ sc, float* __restrict__ act, int64_t tile0,
                                              int64_t end, int64_t step)
{
    using N = Net<IN, W, D>;
    const int lane = threadIdx.x & 63, q = lane >> 4, j = lane & 15;
    float yn[N::KT1];  // the next tile's inputs, loaded while the current tile runs
    if (tile0 < end) load_inputs<N::KT1>(y, n_s, tile0 * 16 + j, tile0 * 16 + j < n_s, q, yn);
    for (int64_t tile = tile0; tile < end; tile += step) {
        const int64_t s = tile * 16 + j;
        const bool valid = s < n_s;
        float yb[N::KT1];
#pragma unroll
        for (int kk = 0; kk < N::KT1; ++kk) yb[kk] = yn[kk];
        const int64_t sn = (tile + step) * 16 + j;
        if (tile + step < end) load_inputs<N::KT1>(y, n_s, sn, sn < n_s, q, yn);
        floatx4 hs[D][N::OT];
        floatx4 o;
        mlp_chain<IN, W, D>(frag, lane, yb, hs, o);
        if (q == 0 && valid) sc[s] = make_float4(__expf(o[0]), sigmoidf_(o[1]), sigmoidf_(o[2]), sigmoidf_(o[3]));
        if (act && valid) {
#pragma unroll
            for (int k = 0; k < D; ++k)
#pragma unroll
                for (int to = 0; to < N::OT; ++to)
                    *reinterpret_cast<floatx4*>(act + ((int64_t)k * n_s + s) * W + 16 * to + 4 * q) = hs[k][to];
        }
    }
}

template <int IN, int W, int D>
__global__ __launch_bounds__(256) void k_mlp_fwd(const float* __restrict__ w, const float* __restrict__ y,
                                                 int64_t n_s, float4* __restrict__ sc, float* __restrict__ act)
{
    using N = Net<IN, W, D>;
    extern __shared__ float frag[];
    load_fragments<IN, W, D>(w, frag, N::N_FWD);
    __syncthreads();
    const int64_t wave0 = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x / 64);
    mlp_fwd_tiles<IN, W, D>(frag, y, n_s, sc, act, wave0, (n_s + 15) / 16, n_waves);
}

// Batched forward: block b works on tiles [tile_begin, tile_end) of object
// work[b].obj, whose weights start at w_off[obj] and whose features and head
// outputs live at y_off / s_off (activations at a_off when act is given).
template <int IN, int W, int D>
__global__ __launch_bounds__(256) void k_mlp_fwd_batch(const MlpWork* __restrict__ work, const float* __restrict__ params,
                                                       const float* __restrict__ y, float4* __restrict__ sc,
                                                       float* __restrict__ act)
{
    using N = Net<IN, W, D>;
    extern __shared__ float frag[];
    const MlpWork wk = work[blockIdx.x];
    load_fragments<IN, W, D>(params + wk.w_off, frag, N::N_FWD);
    __syncthreads();
    const int wave = threadIdx.x >> 6, n_waves = blockDim.x / 64;
    mlp_fwd_tiles<IN, W, D>(frag, y + wk.y_off, wk.n_s, sc + wk.s_off, act ? act + wk.a_off : nullptr,
                            wk.tile_begin + wave, wk.tile_end, n_waves);
}

constexpr int kStagePadF32 = 10;

template <int IN, int W, int D>
struct BwdLds {
    static constexpr int IP = 16 * Net<IN, W, D>::IT;           // input dim padded to 16
    // Row pitches padded by 10 floats: the staging stores (lane (q, j) at
    // row j, column 4 q + r) and the accumulation loads (row 4 ks + q, column
    // j) then spread over the LDS banks with at most 3-way conflicts on the
    // stores and 2-way on the loads for the 32- and 64-wide networks (a pad
    // of 4 gave 4-way on both).
    static constexpr int HW = (W > IP ? W : IP) + kStagePadF32;  // H row pitch
    static constexpr int DW = W + kStagePadF32;                  // Delta row pitch
    static constexpr int PER_WAVE = 16 * (HW + DW);
};

template <int OTILES, int ITILES, int DP, int HP>
__device__ __forceinline__ void accumulate_dw(const float* __restrict__ sD, const float* __restrict__ sH,
                                              floatx4 (&dw)[OTILES][ITILES], int q, int j)
{
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        float a[OTILES], b[ITILES];
#pragma unroll
        for (int to = 0; to < OTILES; ++to) a[to] = sD[(4 * ks + q) * DP + 16 * to + j];
#pragma unroll
        for (int ti = 0; ti < ITILES; ++ti) b[ti] = sH[(4 * ks + q) * HP + 16 * ti + j];
#pragma unroll
        for (int to = 0; to < OTILES; ++to)
#pragma unroll
            for (int ti = 0; ti < ITILES; ++ti) dw[to][ti] = mfma4(a[to], b[ti], dw[to][ti]);
    }
}

// Backward over tiles tile0, tile0 + step, ... < end (per wave) of one object
// whose fragments are in LDS (lds[0 .. N_ALL*64)); writes dy and the block's
// merged dW to dst.  Called by every thread of the block.
// bm (or null): also note the maxima of |dy| of the work item starting at tile
// tile_begin; bad: set on a non-finite dy.
template <int IN, int W, int D>
__device__ __forceinline__ void mlp_bwd_tiles(float* __restrict__ lds, const float* __restrict__ y, const float4* __restrict__ dout,
                              int64_t n_s, float2* __restrict__ dy, float* __restrict__ dst, int64_t tile0,
                              int64_t end, int64_t step, DyMaxLds* bm = nullptr, int64_t tile_begin = 0,
                              bool* bad = nullptr)
{
    using N = Net<IN, W, D>;
    using B = BwdLds<IN, W, D>;
    const float* frag = lds;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4, j = lane & 15;
    float* sD = lds + N::N_ALL * 64 + wave * B::PER_WAVE;
    float* sH = sD + 16 * B::DW;

    floatx4 dW1[N::OT][N::IT];
    floatx4 dWh[D > 1 ? D - 1 : 1][N::OT][N::OT];
    floatx4 dWo[1][N::OT];
#pragma unroll
    for (int a = 0; a < N::OT; ++a) {
#pragma unroll
        for (int b = 0; b < N::IT; ++b) dW1[a][b] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int b = 0; b < N::OT; ++b) {
#pragma unroll
            for (int k = 0; k < (D > 1 ? D - 1 : 1); ++k) dWh[k][a][b] = {0.0f, 0.0f, 0.0f, 0.0f};
        }
        dWo[0][a] = {0.0f, 0.0f, 0.0f, 0.0f};
    }

    // the next tile's inputs and upstream gradient, loaded while the current tile runs
    float yn[N::KT1];
    float4 gn = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    auto load_tile = [&](int64_t t) {
        const int64_t st = t * 16 + j;
        const bool ok = t < end && st < n_s;
        load_inputs<N::KT1>(y, n_s, st, ok, q, yn);
        gn = ok && q == 0 ? dout[st] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    };
    load_tile(tile0);
    for (int64_t tile = tile0; tile < end; tile += step) {
        const int64_t s = tile * 16 + j;
        const bool valid = s < n_s;
        float yb[N::KT1];
#pragma unroll
        for (int kk = 0; kk < N::KT1; ++kk) yb[kk] = yn[kk];
        const float4 gc = gn;
        load_tile(tile + step);
        floatx4 hs[D][N::OT];
        floatx4 o;
        mlp_chain<IN, W, D>(frag, lane, yb, hs, o);

        // head adjoint: lanes with q == 0 hold the 4 outputs of sample j
        float dq0 = 0.0f, dq1 = 0.0f, dq2 = 0.0f, dq3 = 0.0f;
        if (q == 0 && valid) {
            const float4 g = gc;
            const float sig = __expf(o[0]);
            const float c1 = sigmoidf_(o[1]), c2 = sigmoidf_(o[2]), c3 = sigmoidf_(o[3]);
            dq0 = g.x * sig;
            dq1 = g.y * c1 * (1.0f - c1);
            dq2 = g.z * c2 * (1.0f - c2);
            dq3 = g.w * c3 * (1.0f - c3);
        }
        // B operand of the head adjoint: lane l holds output q of sample j
        const float v0 = __shfl(dq0, j), v1 = __shfl(dq1, j), v2 = __shfl(dq2, j), v3 = __shfl(dq3, j);
        const float dqb = q == 0 ? v0 : (q == 1 ? v1 : (q == 2 ? v2 : v3));

        // dW_out += dO h_D^T  (dO staged as a 16-row block with rows >= 4 zero)
        {
            floatx4 dO[1];
            dO[0] = {q == 0 ? v0 : 0.0f, q == 0 ? v1 : 0.0f, q == 0 ? v2 : 0.0f, q == 0 ? v3 : 0.0f};
            // D layout for rows 4q+r: only q == 0 carries real rows 0..3
            wave_lds_sync();
            stage_dw<1, N::OT, B::DW, B::HW>(sD, sH, dO, hs[D - 1], q, j);
            wave_lds_sync();
            accumulate_dw<1, N::OT, B::DW, B::HW>(sD, sH, dWo, q, j);
        }
        // delta of the last hidden layer
        floatx4 delta[N::OT];
#pragma unroll
        for (int to = 0; to < N::OT; ++to) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = mfma4(frag[(N::BO + to) * 64 + lane], dqb, acc);
            delta[to] = mask_pos(acc, hs[D - 1][to]);
        }
        // hidden layers, last to first
#pragma unroll
        for (int k = D - 1; k >= 1; --k) {
            wave_lds_sync();
            stage_dw<N::OT, N::OT, B::DW, B::HW>(sD, sH, delta, hs[k - 1], q, j);
            wave_lds_sync();
            accumulate_dw<N::OT, N::OT, B::DW, B::HW>(sD, sH, dWh[k - 1], q, j);
            floatx4 nd[N::OT];
#pragma unroll
            for (int to = 0; to < N::OT; ++to) {
                floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int ks = 0; ks < N::KTH; ++ks)
                    acc = mfma4(frag[(N::BH + ((k - 1) * N::OT + to) * N::KTH + ks) * 64 + lane], delta[ks >> 2][ks & 3],
                                acc);
                nd[to] = mask_pos(acc, hs[k - 1][to]);
            }
#pragma unroll
            for (int to = 0; to < N::OT; ++to) delta[to] = nd[to];
        }
        // layer 1: dW_1 += delta y^T (y staged from its B-operand layout)
        wave_lds_sync();
#pragma unroll
        for (int to = 0; to < N::OT; ++to)
#pragma unroll
            for (int r = 0; r < 4; ++r) sD[j * B::DW + 16 * to + 4 * q + r] = delta[to][r];
#pragma unroll
        for (int kk = 0; kk < N::KT1; ++kk) sH[j * B::HW + 4 * kk + q] = yb[kk];
#pragma unroll
        for (int c = IN + q; c < B::IP; c += 4) sH[j * B::HW + c] = 0.0f;
        wave_lds_sync();
        accumulate_dw<N::OT, N::IT, B::DW, B::HW>(sD, sH, dW1, q, j);
        // dy = W_1^T delta_1
#pragma unroll
        for (int to = 0; to < N::IT; ++to) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < N::KTH; ++ks)
                acc = mfma4(frag[(N::B1 + to * N::KTH + ks) * 64 + lane], delta[ks >> 2][ks & 3], acc);
            const int f = 16 * to + 4 * q;  // features f..f+3 = levels f/2, f/2 + 1
            if (valid && f < IN) {
                dy[(int64_t)(f >> 1) * n_s + s] = make_float2(acc[0], acc[1]);
                dy[(int64_t)((f >> 1) + 1) * n_s + s] = make_float2(acc[2], acc[3]);
            }
            if (bm) dymax_note(*bm, tile, tile_begin, f >> 1, acc, valid && f < IN, j, *bad);
        }
    }

    // block reduction of the 8 waves' dW (in wave order, so it is
    // deterministic), in the staging area, then one partial per block
    static_assert(N::N_PARAMS <= kBwdWaves * B::PER_WAVE, "reduction buffer");
    float* red = lds + N::N_ALL * 64;
    __syncthreads();
    for (int w = 0; w < kBwdWaves; ++w) {
        if (wave == w) {
            merge_dw<N::OT, N::IT>(red + N::OFF_W1, dW1, W, IN, q, j, w == 0);
#pragma unroll
            for (int k = 1; k < D; ++k)
                merge_dw<N::OT, N::OT>(red + N::OFF_H + (k - 1) * W * W, dWh[k - 1], W, W, q, j, w == 0);
            merge_dw<1, N::OT>(red + N::OFF_OUT, dWo, 4, W, q, j, w == 0);
        }
        __syncthreads();
    }
    for (int p = threadIdx.x; p < N::N_PARAMS; p += blockDim.x) dst[p] = red[p];
}

template <int IN, int W, int D>
__global__ __launch_bounds__(64 * kBwdWaves) void k_mlp_bwd(const float* __restrict__ w,
                                                            const float* __restrict__ y,
                                                            const float4* __restrict__ dout, int64_t n_s,
                                                            float2* __restrict__ dy, float* __restrict__ partial)
{
    using N = Net<IN, W, D>;
    extern __shared__ float lds[];
    load_fragments<IN, W, D>(w, lds, N::N_ALL);
    __syncthreads();
    const int64_t wave0 = (int64_t)blockIdx.x * kBwdWaves + (threadIdx.x >> 6);
    mlp_bwd_tiles<IN, W, D>(lds, y, dout, n_s, dy, partial + (int64_t)blockIdx.x * N::N_PARAMS, wave0,
                            (n_s + 15) / 16, (int64_t)gridDim.x * kBwdWaves);
}

// Batched backward: block b on tiles [tile_begin, tile_end) of object
// work[b].obj; partial dW slot b.
template <int IN, int W, int D>
__global__ __launch_bounds__(64 * kBwdWaves) void k_mlp_bwd_batch(const MlpWork* __restrict__ work,
                                                                  const float* __restrict__ params,
                                                                  const float* __restrict__ y,
                                                                  const float4* __restrict__ dout,
                                                                  float2* __restrict__ dy, float* __restrict__ partial,
                                                                  int64_t slot_stride, float* __restrict__ block_max,
                                                                  int32_t* __restrict__ nonfinite)
{
    using N = Net<IN, W, D>;
    static_assert(IN / 2 <= kBmLevels, "levels");
    extern __shared__ float lds[];
    __shared__ DyMaxLds bm;
    const MlpWork wk = work[blockIdx.x];
    dymax_clear(bm);
    load_fragments<IN, W, D>(params + wk.w_off, lds, N::N_ALL);
    __syncthreads();
    bool bad = false;
    mlp_bwd_tiles<IN, W, D>(lds, y + wk.y_off, dout + wk.s_off, wk.n_s, dy + wk.y_off / 2,
                            partial + (int64_t)blockIdx.x * slot_stride, wk.tile_begin + (threadIdx.x >> 6),
                            wk.tile_end, kBwdWaves, &bm, wk.tile_begin, &bad);
    if (bad && nonfinite) *nonfinite = 1;
    __syncthreads();
    dymax_flush(bm, block_max + wk.bmax_off, wk.n_sblocks, IN / 2, wk.tile_begin, wk.tile_end);
}

// Sum of the per-block partial weight gradients.  A block takes kRedParams
// consecutive parameters (lane = parameter, coalesced) and kRedGroups waves;
// wave w sums slots w, w + kRedGroups, ... in FP64, then the group sums are
// added in wave order (a fixed order: the result does not depend on timing).
constexpr int kRedParams = 64, kRedGroups = 16;

__device__ __forceinline__ void reduce_slots(const float* __restrict__ src, int64_t n_slots, int64_t stride,
                                             bool active, float* __restrict__ dst, double (*part)[kRedParams])
{
    const int i = threadIdx.x % kRedParams, grp = threadIdx.x / kRedParams;
    // four slots in flight per thread, summed in a fixed order
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (active) {
        int64_t sl = grp;
        for (; sl + 3 * kRedGroups < n_slots; sl += 4 * kRedGroups) {
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] += (double)src[(sl + u * kRedGroups) * stride];
        }
        for (; sl < n_slots; sl += kRedGroups) acc[0] += (double)src[sl * stride];
    }
    part[grp][i] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    if (grp == 0 && active) {
        double sum = 0.0;
        for (int k = 0; k < kRedGroups; ++k) sum += part[k][i];
        *dst += (float)sum;
    }
}

__global__ __launch_bounds__(kRedParams * kRedGroups) void k_reduce_partials(const float* __restrict__ partial,
                                                                              int n_slots, int64_t n_mlp,
                                                                              float* __restrict__ g)
{
    __shared__ double part[kRedGroups][kRedParams];
    const int64_t p = (int64_t)blockIdx.x * kRedParams + threadIdx.x % kRedParams;
    const bool active = p < n_mlp;
    const int64_t pc = active ? p : 0;
    reduce_slots(partial + pc, n_slots, n_mlp, active, g + pc, part);
}

// ---------------------------------------------------------------- 128 wide
// One wave cannot hold the 128 x 128 weight gradient in registers (256 VGPRs
// per lane) beside the chain, and the forward plus transposed fragments
// (2 x 88 KB) exceed LDS.  So the widest MLP stores its hidden activations in
// the forward and runs its backward as two kernels:
//   chain : transposed fragments only; ReLU masks from the stored
//           activations, head adjoint from the stored head outputs; writes
//           every layer's delta and dy;
//   dW    : dW_k = sum_s delta_k(s) h_{k-1}(s)^T over the block's samples on
//           MFMA, the 4 waves splitting the output rows; one partial per block.
constexpr int kWideWaves = 4;

template <int IN, int W, int D>
__device__ __forceinline__ void mlp_chain_bwd_tiles(const float* __restrict__ bfrag, const float4* __restrict__ sc,
                                    const float4* __restrict__ dout, const float* __restrict__ act,
                                    float* __restrict__ dlt, int64_t n_s, float2* __restrict__ dy, int64_t tile0,
                                    int64_t end, int64_t step, DyMaxLds* bm = nullptr, int64_t tile_begin = 0,
                                    bool* bad = nullptr)
{
    using N = Net<IN, W, D>;
    constexpr int BO = 0, BH = N::BH - N::N_FWD, B1 = N::B1 - N::N_FWD;  // fragments rebased to the transposed set
    const int lane = threadIdx.x & 63, q = lane >> 4, j = lane & 15;
    // the next tile's upstream gradient and head outputs, loaded while the current tile runs
    float4 gn = make_float4(0.0f, 0.0f, 0.0f, 0.0f), vn = gn;
    auto load_tile = [&](int64_t t) {
        const int64_t st = t * 16 + j;
        const bool ok = t < end && st < n_s && q == 0;
        gn = ok ? dout[st] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        vn = ok ? sc[st] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    };
    load_tile(tile0);
    for (int64_t tile = tile0; tile < end; tile += step) {
        const int64_t s = tile * 16 + j;
        const bool valid = s < n_s;
        const float4 gc = gn, vc = vn;
        load_tile(tile + step);
        float dq0 = 0.0f, dq1 = 0.0f, dq2 = 0.0f, dq3 = 0.0f;
        if (q == 0 && valid) {  // d sigma / d o0 = sigma, d c / d o = c (1 - c)
            const float4 g = gc, v = vc;
            dq0 = g.x * v.x;
            dq1 = g.y * v.y * (1.0f - v.y);
            dq2 = g.z * v.z * (1.0f - v.z);
            dq3 = g.w * v.w * (1.0f - v.w);
        }
        const float v0 = __shfl(dq0, j), v1 = __shfl(dq1, j), v2 = __shfl(dq2, j), v3 = __shfl(dq3, j);
        const float dqb = q == 0 ? v0 : (q == 1 ? v1 : (q == 2 ? v2 : v3));
        floatx4 hk[N::OT], delta[N::OT];
#pragma unroll
        for (int to = 0; to < N::OT; ++to)
            hk[to] = valid ? *reinterpret_cast<const floatx4*>(act + ((int64_t)(D - 1) * n_s + s) * W + 16 * to + 4 * q)
                           : floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int to = 0; to < N::OT; ++to) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = mfma4(bfrag[(BO + to) * 64 + lane], dqb, acc);
            delta[to] = mask_pos(acc, hk[to]);
            if (valid) *reinterpret_cast<floatx4*>(dlt + ((int64_t)(D - 1) * n_s + s) * W + 16 * to + 4 * q) = delta[to];
        }
#pragma unroll
        for (int k = D - 1; k >= 1; --k) {
#pragma unroll
            for (int to = 0; to < N::OT; ++to)
                hk[to] = valid ? *reinterpret_cast<const floatx4*>(act + ((int64_t)(k - 1) * n_s + s) * W + 16 * to + 4 * q)
                               : floatx4{0.0f, 0.0f, 0.0f, 0.0f};
            floatx4 nd[N::OT];
            layer_ks_outer<N::OT, N::KTH>(bfrag, lane, BH + (k - 1) * N::OT * N::KTH, N::KTH, delta, nd);
#pragma unroll
            for (int to = 0; to < N::OT; ++to) {
                delta[to] = mask_pos(nd[to], hk[to]);
                if (valid) *reinterpret_cast<floatx4*>(dlt + ((int64_t)(k - 1) * n_s + s) * W + 16 * to + 4 * q) = delta[to];
            }
        }
        floatx4 gy[N::IT];
        layer_ks_outer<N::IT, N::KTH>(bfrag, lane, B1, N::KTH, delta, gy);
#pragma unroll
        for (int to = 0; to < N::IT; ++to) {
            const floatx4 acc = gy[to];
            const int f = 16 * to + 4 * q;
            if (valid && f < IN) {
                dy[(int64_t)(f >> 1) * n_s + s] = make_float2(acc[0], acc[1]);
                dy[(int64_t)((f >> 1) + 1) * n_s + s] = make_float2(acc[2], acc[3]);
            }
            if (bm) dymax_note(*bm, tile, tile_begin, f >> 1, acc, valid && f < IN, j, *bad);
        }
    }
}

// Weight gradient over samples [s_begin, s_end) of one object, staged
// kDwChunk samples at a time in LDS: wave w owns rows [16 RT w, 16 RT (w+1))
// of W_1 and the hidden matrices and columns [16 RT w, 16 RT (w+1)) of W_out,
// so the block's partial is written without any merge.  MFMA K = 4
// consecutive samples.
constexpr int kDwPitchF32 = kWideWidth + 16;  // 144 = 16 mod 64: lanes q one sample apart, no bank conflict
constexpr int kDwPitchY = 48;

template <int IN, int W, int D>
__device__ __forceinline__ void mlp_dw_range(float* __restrict__ lds, const float* __restrict__ y, const float4* __restrict__ sc,
                             const float4* __restrict__ dout, const float* __restrict__ act,
                             const float* __restrict__ dlt, int64_t n_s, int64_t s_begin, int64_t s_end,
                             float* __restrict__ dst)
{
    using N = Net<IN, W, D>;
    constexpr int PW = kDwPitchF32, PY = kDwPitchY;
    using St = DwStage<W, D, PW, PY>;
    constexpr int RT = N::OT / kWideWaves;
    static_assert(N::OT % kWideWaves == 0 && W + 16 == PW, "rows per wave, pitch");
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
    for (int64_t c0 = s_begin; c0 < s_end; c0 += kDwChunk) {
        dw_stage<IN, W, D, PW, PY>(lds, y, sc, dout, act, dlt, n_s, c0, s_end);
        __syncthreads();
#pragma unroll 2
        for (int ks = 0; ks < kDwChunk / 4; ++ks) {
            const int r = 4 * ks + q;  // the lane's sample within the chunk
            // W_out: A[i][k] = dO_i (rows i >= 4 zero), B = h_{D-1}
            const float dOi = j < 4 ? lds[St::DO + r * 4 + j] : 0.0f;
            const float* hl = lds + St::AC + ((D - 1) * kDwChunk + r) * PW;
#pragma unroll
            for (int a = 0; a < RT; ++a) aO[a] = mfma4(dOi, hl[16 * (RT * wave + a) + j], aO[a]);
#pragma unroll
            for (int k = 1; k < D; ++k) {
                const float* dk = lds + St::DL + (k * kDwChunk + r) * PW;
                const float* hk = lds + St::AC + ((k - 1) * kDwChunk + r) * PW;
                float av[RT], bv[N::OT];
#pragma unroll
                for (int a = 0; a < RT; ++a) av[a] = dk[16 * (RT * wave + a) + j];
#pragma unroll
                for (int t = 0; t < N::OT; ++t) bv[t] = hk[16 * t + j];
#pragma unroll
                for (int a = 0; a < RT; ++a)
#pragma unroll
                    for (int t = 0; t < N::OT; ++t) aH[k - 1][a][t] = mfma4(av[a], bv[t], aH[k - 1][a][t]);
            }
            {
                const float* d0 = lds + St::DL + r * PW;
                const float* yr = lds + St::Y + r * PY;
                float av[RT], bv[N::IT];
#pragma unroll
                for (int a = 0; a < RT; ++a) av[a] = d0[16 * (RT * wave + a) + j];
#pragma unroll
                for (int t = 0; t < N::IT; ++t) bv[t] = yr[16 * t + j];
#pragma unroll
                for (int a = 0; a < RT; ++a)
#pragma unroll
                    for (int t = 0; t < N::IT; ++t) a1[a][t] = mfma4(av[a], bv[t], a1[a][t]);
            }
        }
        __syncthreads();
    }
    // D layout: row 16 (RT w + a) + 4 q + r, column 16 t + j
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
constexpr size_t dw_lds_bytes()
{
    return sizeof(float) * (size_t)DwStage<W, D, kDwPitchF32, kDwPitchY>::FLOATS;
}

template <int IN, int W, int D>
__global__ __launch_bounds__(256) void k_mlp_chain_bwd(const float* __restrict__ w, const float4* __restrict__ sc,
                                                       const float4* __restrict__ dout, float* __restrict__ act,
                                                       int64_t n_s, float2* __restrict__ dy)
{
    using N = Net<IN, W, D>;
    extern __shared__ float frag[];
    load_fragments<IN, W, D>(w, frag, N::N_ALL - N::N_FWD, N::N_FWD);
    __syncthreads();
    const int64_t wave0 = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    mlp_chain_bwd_tiles<IN, W, D>(frag, sc, dout, act, act + (int64_t)D * n_s * W, n_s, dy, wave0, (n_s + 15) / 16,
                                  (int64_t)gridDim.x * (blockDim.x / 64));
}

template <int IN, int W, int D>
__global__ __launch_bounds__(256) void k_mlp_chain_bwd_batch(const MlpWork* __restrict__ work,
                                                             const float* __restrict__ params,
                                                             const float4* __restrict__ sc,
                                                             const float4* __restrict__ dout, float* __restrict__ act,
                                                             float2* __restrict__ dy, float* __restrict__ block_max,
                                                             int32_t* __restrict__ nonfinite)
{
    using N = Net<IN, W, D>;
    static_assert(IN / 2 <= kBmLevels, "levels");
    extern __shared__ float frag[];
    __shared__ DyMaxLds bm;
    const MlpWork wk = work[blockIdx.x];
    dymax_clear(bm);
    load_fragments<IN, W, D>(params + wk.w_off, frag, N::N_ALL - N::N_FWD, N::N_FWD);
    __syncthreads();
    const float* a = act + wk.a_off;
    bool bad = false;
    mlp_chain_bwd_tiles<IN, W, D>(frag, sc + wk.s_off, dout + wk.s_off, a, act + wk.a_off + (int64_t)D * wk.n_s * W,
                                  wk.n_s, dy + wk.y_off / 2, wk.tile_begin + (threadIdx.x >> 6), wk.tile_end,
                                  blockDim.x / 64, &bm, wk.tile_begin, &bad);
    if (bad && nonfinite) *nonfinite = 1;
    __syncthreads();
    dymax_flush(bm, block_max + wk.bmax_off, wk.n_sblocks, IN / 2, wk.tile_begin, wk.tile_end);
}

template <int IN, int W, int D>
__global__ __launch_bounds__(64 * kWideWaves) void k_mlp_dw(const float* __restrict__ y, const float4* __restrict__ sc,
                                                            const float4* __restrict__ dout,
                                                            const float* __restrict__ act, int64_t n_s,
                                                            int64_t tiles_per_block, float* __restrict__ partial)
{
    using N = Net<IN, W, D>;
    extern __shared__ float dw_lds[];
    const int64_t b = (int64_t)blockIdx.x * tiles_per_block * 16;
    const int64_t e = min(b + tiles_per_block * 16, n_s);
    mlp_dw_range<IN, W, D>(dw_lds, y, sc, dout, act, act + (int64_t)D * n_s * W, n_s, b, e,
                           partial + (int64_t)blockIdx.x * N::N_PARAMS);
}

template <int IN, int W, int D>
__global__ __launch_bounds__(64 * kWideWaves) void k_mlp_dw_batch(const MlpWork* __restrict__ work,
                                                                  const float* __restrict__ y,
                                                                  const float4* __restrict__ sc,
                                                                  const float4* __restrict__ dout,
                                                                  const float* __restrict__ act,
                                                                  float* __restrict__ partial, int64_t slot_stride)
{
    extern __shared__ float dw_lds[];
    const MlpWork wk = work[blockIdx.x];
    const int64_t b = wk.tile_begin * 16, e = min(wk.tile_end * 16, wk.n_s);
    const float* a = act + wk.a_off;
    mlp_dw_range<IN, W, D>(dw_lds, y + wk.y_off, sc + wk.s_off, dout + wk.s_off, a, a + (int64_t)D * wk.n_s * W, wk.n_s,
                           b, e, partial + (int64_t)blockIdx.x * slot_stride);
}

// Batch: thread per (object, MLP parameter); the object's partials summed in FP64.
// Batched: parameter i of the batch's MLP gradients belongs to the last
// object with mlp_begin <= i.
__global__ __launch_bounds__(kRedParams * kRedGroups) void k_reduce_partials_batch(const MlpRed* __restrict__ reds,
                                                                                    int n_obj, int64_t n_total,
                                                                                    const float* __restrict__ partial,
                                                                                    float* __restrict__ g)
{
    __shared__ double part[kRedGroups][kRedParams];
    const int64_t i = (int64_t)blockIdx.x * kRedParams + threadIdx.x % kRedParams;
    const bool active = i < n_total;
    const int64_t ic = active ? i : 0;
    int lo = 0, hi = n_obj - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (reds[mid].mlp_begin <= ic)
            lo = mid;
        else
            hi = mid - 1;
    }
    const MlpRed& r = reds[lo];
    const int64_t p = ic - r.mlp_begin;
    reduce_slots(partial + r.partial_off + p, r.n_slots, r.n_mlp, active, g + r.g_off + p, part);
}

template <class K>
hipError_t set_lds(K kern, size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int IN, int W, int D>
size_t fwd_lds_bytes()
{
    return sizeof(float) * (size_t)Net<IN, W, D>::N_FWD * 64;
}

template <int IN, int W, int D>
size_t chain_bwd_lds_bytes()
{
    return sizeof(float) * (size_t)(Net<IN, W, D>::N_ALL - Net<IN, W, D>::N_FWD) * 64;
}

template <int IN, int W, int D>
hipError_t fwd_impl(const float* w, const float* y, int64_t n_s, float* sc, float* act, hipStream_t s)
{
    const int64_t n_tiles = (n_s + 15) / 16;
    int64_t blocks = (n_tiles + 3) / 4;
    blocks = blocks > 2048 ? 2048 : blocks;
    const size_t lds = fwd_lds_bytes<IN, W, D>();
    hipError_t e = set_lds(k_mlp_fwd<IN, W, D>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_mlp_fwd<IN, W, D>), dim3((uint32_t)blocks), dim3(256), lds, s, w, y, n_s, (float4*)sc,
                       W >= kWideWidth ? act : nullptr);
    return hipGetLastError();
}

template <int IN, int W, int D>
size_t bwd_lds_bytes()
{
    return sizeof(float) * ((size_t)Net<IN, W, D>::N_ALL * 64 + (size_t)kBwdWaves * BwdLds<IN, W, D>::PER_WAVE);
}

template <int IN, int W, int D>
hipError_t bwd_impl(const float* w, const float* y, const float* dout, const float* sc, int64_t n_s, float* dy,
                    float* partial, float* act, hipStream_t s)
{
    if constexpr (W >= kWideWidth) {
        const int64_t n_tiles = (n_s + 15) / 16;
        int64_t blocks = (n_tiles + 3) / 4;
        blocks = blocks > 2048 ? 2048 : blocks;
        const size_t lds = chain_bwd_lds_bytes<IN, W, D>();
        hipError_t e = set_lds(k_mlp_chain_bwd<IN, W, D>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_mlp_chain_bwd<IN, W, D>), dim3((uint32_t)blocks), dim3(256), lds, s, w,
                           (const float4*)sc, (const float4*)dout, act, n_s, (float2*)dy);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int nb = bwd_blocks(n_s);
        const int64_t per = (n_tiles + nb - 1) / nb;
        const size_t dwl = dw_lds_bytes<IN, W, D>();
        if ((e = set_lds(k_mlp_dw<IN, W, D>, dwl)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_mlp_dw<IN, W, D>), dim3((uint32_t)nb), dim3(64 * kWideWaves), dwl, s, y,
                           (const float4*)sc, (const float4*)dout, act, n_s, per, partial);
        return hipGetLastError();
    } else {
        const size_t lds = bwd_lds_bytes<IN, W, D>();
        auto kern = k_mlp_bwd<IN, W, D>;
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3((uint32_t)bwd_blocks(n_s)), dim3(64 * kBwdWaves), lds, s, w, y,
                           (const float4*)dout, n_s, (float2*)dy, partial);
        return hipGetLastError();
    }
}

template <int IN, int W, int D>
hipError_t fwd_batch_impl(const MlpWork* work, int n_blocks, const float* params, const float* y, float* sc, float* act,
                          hipStream_t s)
{
    const size_t lds = fwd_lds_bytes<IN, W, D>();
    hipError_t e = set_lds(k_mlp_fwd_batch<IN, W, D>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_mlp_fwd_batch<IN, W, D>), dim3((uint32_t)n_blocks), dim3(256), lds, s, work, params, y,
                       (float4*)sc, W >= kWideWidth ? act : nullptr);
    return hipGetLastError();
}

template <int IN, int W, int D>
hipError_t bwd_batch_impl(const MlpWork* work, int n_blocks, const float* params, const float* y, const float* dout,
                          const float* sc, float* dy, float* partial, int64_t slot_stride, float* act,
                          float* block_max, int32_t* nonfinite, hipStream_t s)
{
    if constexpr (W >= kWideWidth) {
        const size_t lds = chain_bwd_lds_bytes<IN, W, D>();
        hipError_t e = set_lds(k_mlp_chain_bwd_batch<IN, W, D>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_mlp_chain_bwd_batch<IN, W, D>), dim3((uint32_t)n_blocks), dim3(256), lds, s, work,
                           params, (const float4*)sc, (const float4*)dout, act, (float2*)dy, block_max, nonfinite);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const size_t dwl = dw_lds_bytes<IN, W, D>();
        if ((e = set_lds(k_mlp_dw_batch<IN, W, D>, dwl)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_mlp_dw_batch<IN, W, D>), dim3((uint32_t)n_blocks), dim3(64 * kWideWaves), dwl, s, work, y,
                           (const float4*)sc, (const float4*)dout, act, partial, slot_stride);
        return hipGetLastError();
    } else {
        const size_t lds = bwd_lds_bytes<IN, W, D>();
        auto kern = k_mlp_bwd_batch<IN, W, D>;
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3((uint32_t)n_blocks), dim3(64 * kBwdWaves), lds, s, work, params, y,
                           (const float4*)dout, (float2*)dy, partial, slot_stride, block_max, nonfinite);
        return hipGetLastError();
    }
}

}  // namespace

bool mlp_supported(const MlpShape& m)
{
    return (m.width == 32 || m.width == 64 || m.width == 128) && (m.in_dim == 16 || m.in_dim == 24 || m.in_dim == 32) &&
           (m.hidden == 1 || m.hidden == 2);
}

int mlp_bwd_waves(int64_t n_samples) { return bwd_blocks(n_samples); }

// Every supported (input features, width, hidden layers).
#define PRENOM_FOR_EACH_MLP(X) \
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

hipError_t launch_mlp_fwd(const MlpShape& m, const float* w, const float* y, int64_t n_s, float* sc, float* act,
                          hipStream_t s)
{
    if (n_s == 0) return hipSuccess;
#define X(I, Wd, Dp) \
    if (m.in_dim == I && m.width == Wd && m.hidden == Dp) return fwd_impl<I, Wd, Dp>(w, y, n_s, sc, act, s);
    PRENOM_FOR_EACH_MLP(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_mlp_bwd(const MlpShape& m, const float* w, const float* y, const float* dout, const float* sc,
                          int64_t n_s, float* dy, float* partial, float* act, hipStream_t s)
{
    if (n_s == 0) return hipSuccess;
#define X(I, Wd, Dp)                                        \
    if (m.in_dim == I && m.width == Wd && m.hidden == Dp) \
        return bwd_impl<I, Wd, Dp>(w, y, dout, sc, n_s, dy, partial, act, s);
    PRENOM_FOR_EACH_MLP(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_mlp_fwd_batch(const MlpShape& m, const MlpWork* work, int n_blocks, const float* params,
                                const float* y, float* sc, float* act, hipStream_t s)
{
    if (n_blocks == 0) return hipSuccess;
#define X(I, Wd, Dp)                                        \
    if (m.in_dim == I && m.width == Wd && m.hidden == Dp) \
        return fwd_batch_impl<I, Wd, Dp>(work, n_blocks, params, y, sc, act, s);
    PRENOM_FOR_EACH_MLP(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_mlp_bwd_batch(const MlpShape& m, const MlpWork* work, int n_blocks, const float* params,
                                const float* y, const float* dout, const float* sc, float* dy, float* partial,
                                int64_t slot_stride, float* act, float* block_max, int32_t* nonfinite,
                                hipStream_t s)
{
    if (n_blocks == 0) return hipSuccess;
#define X(I, Wd, Dp)                                                                                   \
    if (m.in_dim == I && m.width == Wd && m.hidden == Dp)                                            \
        return bwd_batch_impl<I, Wd, Dp>(work, n_blocks, params, y, dout, sc, dy, partial, slot_stride, act, \
                                         block_max, nonfinite, s);
    PRENOM_FOR_EACH_MLP(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_reduce_partials_batch(const MlpRed* reds, int n_obj, int64_t n_mlp_total, const float* partial,
                                        float* grads, hipStream_t s)
{
    if (n_mlp_total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_partials_batch, dim3((uint32_t)((n_mlp_total + kRedParams - 1) / kRedParams)),
                       dim3(kRedParams * kRedGroups), 0, s, reds, n_obj, n_mlp_total, partial, grads);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const float* partial, int n_slots, int64_t n_mlp, float* g_mlp, hipStream_t s)
{
    if (n_slots == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_partials, dim3((uint32_t)((n_mlp + kRedParams - 1) / kRedParams)),
                       dim3(kRedParams * kRedGroups), 0, s, partial, n_slots, n_mlp, g_mlp);
    return hipGetLastError();
}

}  // namespace prenom

// Volume rendering and losses (Sec. III-B "Volume Rendering", Eq. (5),
// (7)-(9)) and their adjoint.
//
// One 64-lane wavefront per ray, one lane per sample: the transmittance
// T_j = exp(-sum_{i<j} sigma_i delta_i) is an exclusive prefix scan of
// sigma delta across the wave, the adjoint's sum_{k>j} w_k a_k an exclusive
// suffix scan; rays longer than 64 samples are walked in 64-sample chunks
// with the scan carried between chunks.  FP32 scans; the batch loss is summed
// per block in FP64 and finished by one block.
#include "common.h"

namespace prenom {
namespace {

constexpr int kRaysPerBlock = 4;  // one wave per ray
constexpr int kMaxChunks = 4;     // S <= 256

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

// exclusive prefix sum over the 64 lanes
__device__ __forceinline__ float wave_excl_prefix(float x, int lane)
{
    float incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const float v = __shfl_up(incl, d);
        if (lane >= d) incl += v;
    }
    const float e = __shfl_up(incl, 1);
    return lane == 0 ? 0.0f : e;
}

// exclusive suffix sum (sum over lanes above this one)
__device__ __forceinline__ float wave_excl_suffix(float x, int lane)
{
    float incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const float v = __shfl_down(incl, d);
        if (lane + d < 64) incl += v;
    }
    const float e = __shfl_down(incl, 1);
    return lane == 63 ? 0.0f : e;
}

// Rays over which the loss of ray r is averaged: the whole call, or the
// ray's object in a batch.
__device__ __forceinline__ int64_t norm_rays(const CompositeArgs& a, int64_t r)
{
    if (!a.objs) return a.n_rays;
    int lo = 0, hi = a.n_obj - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.objs[mid].ray_begin <= r)
            lo = mid;
        else
            hi = mid - 1;
    }
    return a.objs[lo].n_rays;
}

struct RayTargets {
    float C[3];
    float D;
    bool obj;
};

__device__ __forceinline__ RayTargets load_targets(const CompositeArgs& a, int64_t r)
{
    RayTargets tg;
    for (int k = 0; k < 3; ++k) tg.C[k] = a.tgt_rgb ? a.tgt_rgb[3 * r + k] : 0.0f;
    tg.D = a.tgt_depth ? a.tgt_depth[r] : 0.0f;
    tg.obj = a.mask ? a.mask[r] != 0 : true;
    return tg;
}

__global__ __launch_bounds__(64 * kRaysPerBlock) void k_composite_fwd(CompositeArgs a)
{
    __shared__ double block_loss[kRaysPerBlock];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * kRaysPerBlock + wave;
    double ray_loss = 0.0;
    if (r < a.n_rays) {
        const int S = a.S;
        float bg[3] = {0.0f, 0.0f, 0.0f};
        if (a.bg)
            for (int k = 0; k < 3; ++k) bg[k] = a.bg[3 * r + k];
        float C[3] = {0.0f, 0.0f, 0.0f}, Dh = 0.0f, A = 0.0f, sig_sum = 0.0f, T_S = 1.0f;
        if (!(a.flags[r] & PRENOM_FLAG_MISS)) {
            float carry = 0.0f;
            for (int c0 = 0; c0 < S; c0 += 64) {
                const int jj = c0 + lane;
                const bool valid = jj < S;
                const int64_t sidx = r * S + jj;
                float4 v = valid ? reinterpret_cast<const float4*>(a.sc)[sidx] : make_float4(0, 0, 0, 0);
                const float dtj = valid ? a.dt[sidx] : 0.0f;
                const float tj = valid ? a.t[sidx] : 0.0f;
                const float tau = v.x * dtj;
                const float excl = wave_excl_prefix(tau, lane) + carry;
                const float w = expf(-excl) * (-expm1f(-tau));
                C[0] += w * v.y;
                C[1] += w * v.z;
                C[2] += w * v.w;
                Dh += w * tj;
                A += w;
                sig_sum += v.x;
                carry += wave_sum(tau);
            }
            for (int k = 0; k < 3; ++k) C[k] = wave_sum(C[k]);
            Dh = wave_sum(Dh);
            A = wave_sum(A);
            sig_sum = wave_sum(sig_sum);
            T_S = expf(-carry);
        }
        for (int k = 0; k < 3; ++k) C[k] += T_S * bg[k];
        if (lane == 0) {
            if (a.rgb) {
                for (int k = 0; k < 3; ++k) a.rgb[3 * r + k] = C[k];
                a.depth[r] = Dh;
                a.opacity[r] = A;
            }
            float* st = a.ray_state + 8 * r;
            st[0] = C[0];
            st[1] = C[1];
            st[2] = C[2];
            st[3] = Dh;
            st[4] = T_S;
            st[5] = sig_sum;
        }
        if (a.tgt_rgb) {
            const RayTargets tg = load_targets(a, r);
            const double n = (double)norm_rays(a, r);
            const double e0 = (double)C[0] - tg.C[0], e1 = (double)C[1] - tg.C[1], e2 = (double)C[2] - tg.C[2];
            const double ed = (double)Dh - tg.D;
            if (a.loss_mode == 0) {
                ray_loss = (e0 * e0 + e1 * e1 + e2 * e2) / (3.0 * n);
                ray_loss += tg.obj ? (double)a.lambda_d * ed * ed / n : (double)a.lambda_sigma * sig_sum / n;
            } else {
                ray_loss = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
                ray_loss += tg.obj ? (double)a.lambda_d * fabs(ed) : (double)a.lambda_sigma * sig_sum;
            }
        }
    }
    if (a.ray_loss && lane == 0 && r < a.n_rays) a.ray_loss[r] = ray_loss;
    if (a.loss_partial) {
        if (lane == 0) block_loss[wave] = ray_loss;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < kRaysPerBlock; ++w) s += block_loss[w];
            a.loss_partial[blockIdx.x] = s;
        }
    }
}

__global__ __launch_bounds__(1024) void k_loss_finalize(const double* __restrict__ partial, int n, float* loss)
{
    __shared__ double red[1024 / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) s += partial[i];
    s = wave_sum_d(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < 1024 / 64; ++w) tot += red[w];
        *loss = (float)tot;
    }
}

__global__ __launch_bounds__(256) void k_loss_objects(const ObjDev* __restrict__ objs,
                                                      const double* __restrict__ ray_loss, float* loss)
{
    __shared__ double red[4];
    const ObjDev& o = objs[blockIdx.x];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < o.n_rays; i += 256) s += ray_loss[o.ray_begin + i];
    s = wave_sum_d(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) loss[blockIdx.x] = (float)((red[0] + red[1]) + (red[2] + red[3]));
}

__global__ __launch_bounds__(64 * kRaysPerBlock) void k_composite_bwd(CompositeArgs a)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * kRaysPerBlock + wave;
    if (r >= a.n_rays) return;
    const int S = a.S;
    float4* dout = reinterpret_cast<float4*>(a.dout) + r * S;
    if (a.flags[r] & PRENOM_FLAG_MISS) {
        for (int jj = lane; jj < S; jj += 64) dout[jj] = make_float4(0, 0, 0, 0);
        return;
    }
    const float* st = a.ray_state + 8 * r;
    const float Ch[3] = {st[0], st[1], st[2]};
    const float Dh = st[3], T_S = st[4];

    // upstream gradients of this ray: dL/dC, dL/dD and the per-sample density term
    float gC[3], gD = 0.0f, gA = 0.0f, extra = 0.0f;
    if (a.d_rgb) {
        for (int k = 0; k < 3; ++k) gC[k] = a.d_rgb[3 * r + k];
        gD = a.d_depth ? a.d_depth[r] : 0.0f;
        gA = a.d_opacity ? a.d_opacity[r] : 0.0f;
    } else {
        const RayTargets tg = load_targets(a, r);
        const float n = (float)norm_rays(a, r);
        const float e[3] = {Ch[0] - tg.C[0], Ch[1] - tg.C[1], Ch[2] - tg.C[2]};
        const float ed = Dh - tg.D;
        if (a.loss_mode == 0) {
            for (int k = 0; k < 3; ++k) gC[k] = 2.0f * e[k] / (3.0f * n);
            if (tg.obj)
                gD = 2.0f * a.lambda_d * ed / n;
            else
                extra = a.lambda_sigma / n;
        } else {
            const float nrm = sqrtf(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
            for (int k = 0; k < 3; ++k) gC[k] = nrm > 0.0f ? e[k] / nrm : 0.0f;
            if (tg.obj)
                gD = a.lambda_d * (ed > 0.0f ? 1.0f : (ed < 0.0f ? -1.0f : 0.0f));
            else
                extra = a.lambda_sigma;
        }
    }
    if (a.loss_scale) {  // loss scaling: every downstream gradient is scaled
        const float sc = *a.loss_scale;
        gC[0] *= sc;
        gC[1] *= sc;
        gC[2] *= sc;
        gD *= sc;
        gA *= sc;
        extra *= sc;
    }
    float bg_term = 0.0f;
    if (a.bg) bg_term = T_S * (gC[0] * a.bg[3 * r] + gC[1] * a.bg[3 * r + 1] + gC[2] * a.bg[3 * r + 2]);

    // transmittance carried into each chunk
    const int n_chunks = (S + 63) / 64;
    float carry_in[kMaxChunks];
    {
        float c = 0.0f;
        for (int ch = 0; ch < n_chunks; ++ch) {
            carry_in[ch] = c;
            const int jj = ch * 64 + lane;
            const int64_t sidx = r * S + jj;
            const float tau = jj < S ? a.sc[4 * sidx] * a.dt[sidx] : 0.0f;
            c += wave_sum(tau);
        }
    }
    float suffix_carry = 0.0f;
    for (int ch = n_chunks - 1; ch >= 0; --ch) {
        const int jj = ch * 64 + lane;
        const bool valid = jj < S;
        const int64_t sidx = r * S + jj;
        const float4 v = valid ? reinterpret_cast<const float4*>(a.sc)[sidx] : make_float4(0, 0, 0, 0);
        const float dtj = valid ? a.dt[sidx] : 0.0f;
        const float tj = valid ? a.t[sidx] : 0.0f;
        const float tau = v.x * dtj;
        const float excl = wave_excl_prefix(tau, lane) + carry_in[ch];
        const float Tj = expf(-excl);
        const float Tj1 = expf(-(excl + tau));
        const float w = Tj * (-expm1f(-tau));
        const float aj = gC[0] * v.y + gC[1] * v.z + gC[2] * v.w + gD * tj + gA;
        const float wa = valid ? w * aj : 0.0f;
        const float suffix = wave_excl_suffix(wa, lane) + suffix_carry;
        const float dsig = dtj * (Tj1 * aj - suffix - bg_term) + extra;
        if (valid) dout[jj] = make_float4(dsig, w * gC[0], w * gC[1], w * gC[2]);
        suffix_carry += wave_sum(wa);
    }
}

}  // namespace

int composite_loss_blocks(int64_t n_rays) { return (int)((n_rays + kRaysPerBlock - 1) / kRaysPerBlock); }

hipError_t launch_composite_fwd(const CompositeArgs& a, hipStream_t s)
{
    if (a.n_rays == 0) return hipSuccess;
    hipLaunchKernelGGL(k_composite_fwd, dim3((uint32_t)composite_loss_blocks(a.n_rays)), dim3(64 * kRaysPerBlock), 0,
                       s, a);
    return hipGetLastError();
}

hipError_t launch_loss_finalize(const double* partial, int n_blocks, float* loss, hipStream_t s)
{
    hipLaunchKernelGGL(k_loss_finalize, dim3(1), dim3(1024), 0, s, partial, n_blocks, loss);
    return hipGetLastError();
}

hipError_t launch_loss_objects(const ObjDev* objs, int n_obj, const double* ray_loss, float* loss, hipStream_t s)
{
    if (n_obj == 0) return hipSuccess;
    hipLaunchKernelGGL(k_loss_objects, dim3((uint32_t)n_obj), dim3(256), 0, s, objs, ray_loss, loss);
    return hipGetLastError();
}

hipError_t launch_composite_bwd(const CompositeArgs& a, hipStream_t s)
{
    if (a.n_rays == 0) return hipSuccess;
    hipLaunchKernelGGL(k_composite_bwd, dim3((uint32_t)composite_loss_blocks(a.n_rays)), dim3(64 * kRaysPerBlock), 0,
                       s, a);
    return hipGetLastError();
}

}  // namespace prenom

// The optimisers.  Adam over every parameter (Sec. III-B, last paragraph),
// fused with zeroing the gradient it consumed and, when the tables are also
// kept in FP16, with rewriting that copy: pure streaming, 4 loads + 4 stores
// of FP32 per parameter, float4-vectorised.  Plain gradient descent, the
// inner step of meta-learning (Sec. III-A, Eq. (1)), fused the same way:
// 2 loads + 2 stores per parameter.
//
// With loss scaling the gradients arrive multiplied by the device scalar
// `loss_scale`.  One pass flags any non-finite entry; the update then unscales
// and applies Adam, or, when the flag is set, only clears the gradients; a
// one-thread kernel halves the scale after a non-finite step, doubles it after
// growth_interval finite ones, and clears the flag.  No host synchronisation.
#include "common.h"

namespace prenom {
namespace {

constexpr int kAdamBlock = 256;

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void adam_one(float& p, float& g, float& m, float& v, const AdamArgs& a, float inv_scale)
{
    const float gi = g * inv_scale;
    m = a.beta1 * m + (1.0f - a.beta1) * gi;
    v = a.beta2 * v + (1.0f - a.beta2) * gi * gi;
    p -= a.lr * (m * a.inv_c1) / (sqrtf(v * a.inv_c2) + a.eps);
    g = 0.0f;
}

__device__ __forceinline__ bool finite4(float4 g)
{
    return isfinite(g.x) && isfinite(g.y) && isfinite(g.z) && isfinite(g.w);
}

__global__ __launch_bounds__(kAdamBlock) void k_adam_check(AdamArgs a)
{
    const int64_t n4 = a.n >> 2;
    const int64_t stride = (int64_t)gridDim.x * kAdamBlock;
    bool ok = true;
    for (int64_t i = (int64_t)blockIdx.x * kAdamBlock + threadIdx.x; i < n4; i += stride)
        ok = ok && finite4(reinterpret_cast<const float4*>(a.g)[i]);
    if (blockIdx.x == 0 && threadIdx.x < (a.n & 3)) ok = ok && isfinite(a.g[(n4 << 2) + threadIdx.x]);
    if (__syncthreads_or(!ok) && threadIdx.x == 0) atomicOr(&a.scaler_state[0], 1);
}

__global__ __launch_bounds__(kAdamBlock) void k_adam(AdamArgs a)
{
    const int64_t n4 = a.n >> 2;
    const int64_t stride = (int64_t)gridDim.x * kAdamBlock;
    const bool skip = a.loss_scale && a.scaler_state[0] != 0;
    if (a.step_dev) {  // bias corrections of step *step_dev + 1, once per block
        __shared__ float s_c[2];
        if (threadIdx.x == 0) {
            const double k = (double)(*a.step_dev + 1);
            s_c[0] = (float)(1.0 / (1.0 - pow((double)a.beta1, k)));
            s_c[1] = (float)(1.0 / (1.0 - pow((double)a.beta2, k)));
        }
        __syncthreads();
        a.inv_c1 = s_c[0];
        a.inv_c2 = s_c[1];
    }
    const float inv_scale = a.loss_scale ? 1.0f / *a.loss_scale : 1.0f;
    for (int64_t i = (int64_t)blockIdx.x * kAdamBlock + threadIdx.x; i < n4; i += stride) {
        float4* g4 = reinterpret_cast<float4*>(a.g) + i;
        if (skip) {
            *g4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            continue;
        }
        float4 p = reinterpret_cast<float4*>(a.p)[i];
        float4 g = *g4;
        float4 m = reinterpret_cast<float4*>(a.m)[i];
        float4 v = reinterpret_cast<float4*>(a.v)[i];
        adam_one(p.x, g.x, m.x, v.x, a, inv_scale);
        adam_one(p.y, g.y, m.y, v.y, a, inv_scale);
        adam_one(p.z, g.z, m.z, v.z, a, inv_scale);
        adam_one(p.w, g.w, m.w, v.w, a, inv_scale);
        reinterpret_cast<float4*>(a.p)[i] = p;
        *g4 = g;
        reinterpret_cast<float4*>(a.m)[i] = m;
        reinterpret_cast<float4*>(a.v)[i] = v;
        if (a.table_f16 && (i << 2) < a.n_table) {
            half4_t h = {(_Float16)p.x, (_Float16)p.y, (_Float16)p.z, (_Float16)p.w};
            reinterpret_cast<half4_t*>(a.table_f16)[i] = h;
        }
    }
    // tail (n not a multiple of 4; never inside the tables): the first threads of block 0
    if (blockIdx.x == 0 && threadIdx.x < (a.n & 3)) {
        const int64_t i = (n4 << 2) + threadIdx.x;
        if (skip) {
            a.g[i] = 0.0f;
        } else {
            adam_one(a.p[i], a.g[i], a.m[i], a.v[i], a, inv_scale);
            if (a.table_f16 && i < a.n_table) reinterpret_cast<_Float16*>(a.table_f16)[i] = (_Float16)a.p[i];
        }
    }
}

__global__ __launch_bounds__(kAdamBlock) void k_sgd(AdamArgs a)
{
    const int64_t n4 = a.n >> 2;
    const int64_t stride = (int64_t)gridDim.x * kAdamBlock;
    const bool skip = a.loss_scale && a.scaler_state[0] != 0;
    const float step = a.lr * (a.loss_scale ? 1.0f / *a.loss_scale : 1.0f);
    for (int64_t i = (int64_t)blockIdx.x * kAdamBlock + threadIdx.x; i < n4; i += stride) {
        float4* g4 = reinterpret_cast<float4*>(a.g) + i;
        if (skip) {
            *g4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            continue;
        }
        float4 p = reinterpret_cast<float4*>(a.p)[i];
        const float4 g = *g4;
        p.x -= step * g.x;
        p.y -= step * g.y;
        p.z -= step * g.z;
        p.w -= step * g.w;
        reinterpret_cast<float4*>(a.p)[i] = p;
        *g4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (a.table_f16 && (i << 2) < a.n_table) {
            half4_t h = {(_Float16)p.x, (_Float16)p.y, (_Float16)p.z, (_Float16)p.w};
            reinterpret_cast<half4_t*>(a.table_f16)[i] = h;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < (a.n & 3)) {
        const int64_t i = (n4 << 2) + threadIdx.x;
        if (!skip) {
            a.p[i] -= step * a.g[i];
            if (a.table_f16 && i < a.n_table) reinterpret_cast<_Float16*>(a.table_f16)[i] = (_Float16)a.p[i];
        }
        a.g[i] = 0.0f;
    }
}

// After the update: advance the device step counter unless the step was
// skipped, then adjust the loss scale.
__global__ void k_finish_step(float* scale, int32_t* state, int32_t growth_interval, int64_t* step)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const bool skipped = scale && state[0] != 0;
    if (step && !skipped) *step += 1;
    if (!scale) return;
    int32_t good = state[1];
    if (state[0]) {
        *scale *= 0.5f;
        good = 0;
    } else if (growth_interval > 0 && ++good >= growth_interval) {
        *scale *= 2.0f;
        good = 0;
    }
    state[0] = 0;
    state[1] = good;
}

__global__ __launch_bounds__(kAdamBlock) void k_to_f16(const float* __restrict__ src, half4_t* __restrict__ dst,
                                                       int64_t n4)
{
    const int64_t stride = (int64_t)gridDim.x * kAdamBlock;
    for (int64_t i = (int64_t)blockIdx.x * kAdamBlock + threadIdx.x; i < n4; i += stride) {
        const float4 p = reinterpret_cast<const float4*>(src)[i];
        dst[i] = half4_t{(_Float16)p.x, (_Float16)p.y, (_Float16)p.z, (_Float16)p.w};
    }
}

int64_t stream_blocks(int64_t n4)
{
    int64_t blocks = (n4 + kAdamBlock - 1) / kAdamBlock;
    return blocks < 1 ? 1 : (blocks > (1 << 20) ? (1 << 20) : blocks);
}

}  // namespace

hipError_t launch_adam(const AdamArgs& a, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    const dim3 grid((uint32_t)stream_blocks(a.n >> 2));
    hipError_t e;
    if (a.loss_scale) {
        hipLaunchKernelGGL(k_adam_check, grid, dim3(kAdamBlock), 0, s, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_adam, grid, dim3(kAdamBlock), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (a.loss_scale || a.step_dev) {
        hipLaunchKernelGGL(k_finish_step, dim3(1), dim3(64), 0, s, a.loss_scale, a.scaler_state, a.growth_interval,
                           a.step_dev);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_sgd(const AdamArgs& a, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    const dim3 grid((uint32_t)stream_blocks(a.n >> 2));
    hipError_t e;
    if (a.loss_scale) {
        hipLaunchKernelGGL(k_adam_check, grid, dim3(kAdamBlock), 0, s, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_sgd, grid, dim3(kAdamBlock), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (a.loss_scale || a.step_dev) {
        hipLaunchKernelGGL(k_finish_step, dim3(1), dim3(64), 0, s, a.loss_scale, a.scaler_state, a.growth_interval,
                           a.step_dev);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_to_f16(const float* src, void* dst, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_f16, dim3((uint32_t)stream_blocks(n >> 2)), dim3(kAdamBlock), 0, s, src, (half4_t*)dst,
                       n >> 2);
    return hipGetLastError();
}

}  // namespace prenom

// Adam over every parameter (Sec. III-B, last paragraph), fused with zeroing
// the gradient it consumed.  Pure streaming: 4 loads + 4 stores of FP32 per
// parameter, float4-vectorised.
#include "common.h"

namespace prenom {
namespace {

constexpr int kAdamBlock = 256;

__device__ __forceinline__ void adam_one(float& p, float& g, float& m, float& v, const AdamArgs& a)
{
    const float gi = g;
    m = a.beta1 * m + (1.0f - a.beta1) * gi;
    v = a.beta2 * v + (1.0f - a.beta2) * gi * gi;
    p -= a.lr * (m * a.inv_c1) / (sqrtf(v * a.inv_c2) + a.eps);
    g = 0.0f;
}

__global__ __launch_bounds__(kAdamBlock) void k_adam(AdamArgs a)
{
    const int64_t n4 = a.n >> 2;
    const int64_t stride = (int64_t)gridDim.x * kAdamBlock;
    for (int64_t i = (int64_t)blockIdx.x * kAdamBlock + threadIdx.x; i < n4; i += stride) {
        float4 p = reinterpret_cast<float4*>(a.p)[i];
        float4 g = reinterpret_cast<float4*>(a.g)[i];
        float4 m = reinterpret_cast<float4*>(a.m)[i];
        float4 v = reinterpret_cast<float4*>(a.v)[i];
        adam_one(p.x, g.x, m.x, v.x, a);
        adam_one(p.y, g.y, m.y, v.y, a);
        adam_one(p.z, g.z, m.z, v.z, a);
        adam_one(p.w, g.w, m.w, v.w, a);
        reinterpret_cast<float4*>(a.p)[i] = p;
        reinterpret_cast<float4*>(a.g)[i] = g;
        reinterpret_cast<float4*>(a.m)[i] = m;
        reinterpret_cast<float4*>(a.v)[i] = v;
    }
    // tail (n not a multiple of 4): the first threads of block 0
    if (blockIdx.x == 0 && threadIdx.x < (a.n & 3)) {
        const int64_t i = (n4 << 2) + threadIdx.x;
        adam_one(a.p[i], a.g[i], a.m[i], a.v[i], a);
    }
}

}  // namespace

hipError_t launch_adam(const AdamArgs& a, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    int64_t blocks = ((a.n >> 2) + kAdamBlock - 1) / kAdamBlock;
    blocks = blocks < 1 ? 1 : (blocks > 8192 ? 8192 : blocks);
    hipLaunchKernelGGL(k_adam, dim3((uint32_t)blocks), dim3(kAdamBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace prenom

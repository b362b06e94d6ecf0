// Reptile's outer update (Sec. III-A, Eq. (2)): after q inner steps of a task
// trained from the meta-parameters theta, theta moves towards the task's
// result by the meta step size beta.  With several tasks trained from the
// same theta at once, theta moves by beta times the mean of their
// differences (one task: Eq. (2) exactly).  The same pass restarts every
// task slot from the new theta, with its FP16 copy and its Adam moments when
// the caller keeps them, so the next meta-iteration's inner steps can run
// without another copy.
//
// Pure streaming, float4-vectorised: per parameter, (B + 1) FP32 loads and
// (B + 1) FP32 stores, plus 8 B per task for cleared moments and 2 B per task
// for an FP16 copy.
#include "common.h"

namespace prenom {
namespace {

constexpr int kReptileBlock = 256;

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kReptileBlock) void k_reptile(ReptileArgs a)
{
    const int64_t n4 = a.n >> 2;
    const int64_t s4 = a.stride >> 2;
    const int64_t grid_stride = (int64_t)gridDim.x * kReptileBlock;
    const float scale = a.beta / (float)a.n_tasks;
    float4* theta = reinterpret_cast<float4*>(a.theta);
    float4* tasks = reinterpret_cast<float4*>(a.tasks);
    for (int64_t i = (int64_t)blockIdx.x * kReptileBlock + threadIdx.x; i < n4; i += grid_stride) {
        const float4 t = theta[i];
        float4 d = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        for (int b = 0; b < a.n_tasks; ++b) {
            const float4 x = tasks[b * s4 + i];
            d.x += x.x - t.x;
            d.y += x.y - t.y;
            d.z += x.z - t.z;
            d.w += x.w - t.w;
        }
        const float4 nw = make_float4(t.x + scale * d.x, t.y + scale * d.y, t.z + scale * d.z, t.w + scale * d.w);
        theta[i] = nw;
        // FP16 copy of the first n_f16 entries only: whole groups of 4 as one
        // store, a group that n_f16 cuts entry by entry
        const int64_t e0 = i << 2;
        const int lp = !a.tasks_f16 || e0 >= a.n_f16 ? 0 : (e0 + 4 <= a.n_f16 ? 4 : (int)(a.n_f16 - e0));
        const half4_t h = {(_Float16)nw.x, (_Float16)nw.y, (_Float16)nw.z, (_Float16)nw.w};
        for (int b = 0; b < a.n_tasks; ++b) {
            const int64_t j = b * s4 + i;
            tasks[j] = nw;
            if (a.m) {
                reinterpret_cast<float4*>(a.m)[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                reinterpret_cast<float4*>(a.v)[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
            if (lp == 4) {
                reinterpret_cast<half4_t*>(a.tasks_f16)[j] = h;
            } else {
                for (int e = 0; e < lp; ++e) reinterpret_cast<_Float16*>(a.tasks_f16)[4 * j + e] = h[e];
            }
        }
    }
    // tail (n not a multiple of 4): the first threads of block 0
    if (blockIdx.x == 0 && threadIdx.x < (a.n & 3)) {
        const int64_t i = (n4 << 2) + threadIdx.x;
        const float t = a.theta[i];
        float d = 0.0f;
        for (int b = 0; b < a.n_tasks; ++b) d += a.tasks[b * a.stride + i] - t;
        const float nw = t + scale * d;
        a.theta[i] = nw;
        for (int b = 0; b < a.n_tasks; ++b) {
            const int64_t j = b * a.stride + i;
            a.tasks[j] = nw;
            if (a.m) {
                a.m[j] = 0.0f;
                a.v[j] = 0.0f;
            }
            if (a.tasks_f16 && i < a.n_f16) reinterpret_cast<_Float16*>(a.tasks_f16)[j] = (_Float16)nw;
        }
    }
    if (a.step && blockIdx.x == 0 && threadIdx.x == 0) *a.step = 0;
}

}  // namespace

hipError_t launch_reptile(const ReptileArgs& a, hipStream_t s)
{
    if (a.n == 0 && !a.step) return hipSuccess;
    int64_t blocks = ((a.n >> 2) + kReptileBlock - 1) / kReptileBlock;
    blocks = blocks < 1 ? 1 : (blocks > 8192 ? 8192 : blocks);
    hipLaunchKernelGGL(k_reptile, dim3((uint32_t)blocks), dim3(kReptileBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace prenom

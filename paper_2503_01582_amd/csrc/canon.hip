// Canonical yaw search (Sec. III-B, "Object State Canonicalization",
// Eq. (3)).  An object stands on the ground (z up), so its pose in the
// category's canonical frame is searched over the yaw alone: for each of K
// yaws gamma_k = 2 pi k / K the cloud is turned about z, normalised into the
// unit cube by the midpoint and size of its extents (an axis of zero extent
// maps to 1/2), and scored by the sum of the prior's trilinear density over
// its points; the first yaw of largest score wins.
//
// K x |P| lookups of a grid that sits in L2, so the work is spread over a
// (point chunk, yaw) grid of blocks and done in four launches:
//   extents : per (chunk, yaw) the min and max of the turned points
//   combine : per yaw the extents over all chunks -> S_k, C_k (outputs)
//   score   : per (chunk, yaw) the density sum over the chunk's points
//   finish  : per yaw the chunk sums added in chunk order; the first maximum
// FP64 throughout, without contraction; every sum has a fixed order, so the
// result does not depend on scheduling.
#include "common.h"

#pragma clang fp contract(off)

namespace prenom {
namespace {

constexpr int kYawThreads = 256;
constexpr int64_t kYawChunk = 4096;  // points per block
constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ void yaw_rotation(int k, int K, double& c, double& s)
{
    const double g = 2.0 * kPi * (double)k / (double)K;
    c = cos(g);
    s = sin(g);
}

// Block-wide reductions in a fixed order (lane tree, then the 4 waves).
__device__ __forceinline__ double wave_min(double v)
{
    for (int d = 32; d >= 1; d >>= 1) v = fmin(v, __shfl_xor(v, d));
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int d = 32; d >= 1; d >>= 1) v = fmax(v, __shfl_xor(v, d));
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

__global__ __launch_bounds__(kYawThreads) void k_yaw_extents(YawArgs a)
{
    __shared__ double red[kYawThreads / 64][6];
    const int k = blockIdx.y;
    const int64_t c0 = (int64_t)blockIdx.x * kYawChunk;
    const int64_t c1 = c0 + kYawChunk < a.n ? c0 + kYawChunk : a.n;
    double cs, sn;
    yaw_rotation(k, a.K, cs, sn);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t j = c0 + threadIdx.x; j < c1; j += kYawThreads) {
        const double x = a.pts[3 * j], y = a.pts[3 * j + 1];
        const double q[3] = {cs * x - sn * y, sn * x + cs * y, (double)a.pts[3 * j + 2]};
        for (int d = 0; d < 3; ++d) {
            lo[d] = fmin(lo[d], q[d]);
            hi[d] = fmax(hi[d], q[d]);
        }
    }
    const int w = threadIdx.x >> 6;
    for (int d = 0; d < 3; ++d) {
        lo[d] = wave_min(lo[d]);
        hi[d] = wave_max(hi[d]);
    }
    if ((threadIdx.x & 63) == 0)
        for (int d = 0; d < 3; ++d) {
            red[w][d] = lo[d];
            red[w][3 + d] = hi[d];
        }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int d = threadIdx.x;
        double v = red[0][d];
        for (int i = 1; i < kYawThreads / 64; ++i) v = d < 3 ? fmin(v, red[i][d]) : fmax(v, red[i][d]);
        a.part_ext[((int64_t)k * a.n_chunks + blockIdx.x) * 6 + d] = v;
    }
}

// One block per yaw: extents over all chunks, then S_k = max - min and
// C_k = (max + min) / 2 per axis.
__global__ __launch_bounds__(kYawThreads) void k_yaw_combine(YawArgs a)
{
    __shared__ double red[kYawThreads / 64][6];
    const int k = blockIdx.x;
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int64_t c = threadIdx.x; c < a.n_chunks; c += kYawThreads) {
        const double* e = a.part_ext + ((int64_t)k * a.n_chunks + c) * 6;
        for (int d = 0; d < 3; ++d) {
            v[d] = fmin(v[d], e[d]);
            v[3 + d] = fmax(v[3 + d], e[3 + d]);
        }
    }
    const int w = threadIdx.x >> 6;
    for (int d = 0; d < 3; ++d) {
        v[d] = wave_min(v[d]);
        v[3 + d] = wave_max(v[3 + d]);
    }
    if ((threadIdx.x & 63) == 0)
        for (int d = 0; d < 6; ++d) red[w][d] = v[d];
    __syncthreads();
    if (threadIdx.x < 3) {
        const int d = threadIdx.x;
        double lo = red[0][d], hi = red[0][3 + d];
        for (int i = 1; i < kYawThreads / 64; ++i) {
            lo = fmin(lo, red[i][d]);
            hi = fmax(hi, red[i][3 + d]);
        }
        a.extents[3 * k + d] = hi - lo;
        a.centers[3 * k + d] = 0.5 * (hi + lo);
    }
}

__global__ __launch_bounds__(kYawThreads) void k_yaw_score(YawArgs a)
{
    __shared__ double red[kYawThreads / 64];
    const int k = blockIdx.y;
    const int64_t c0 = (int64_t)blockIdx.x * kYawChunk;
    const int64_t c1 = c0 + kYawChunk < a.n ? c0 + kYawChunk : a.n;
    double cs, sn;
    yaw_rotation(k, a.K, cs, sn);
    const double S[3] = {a.extents[3 * k], a.extents[3 * k + 1], a.extents[3 * k + 2]};
    const double C[3] = {a.centers[3 * k], a.centers[3 * k + 1], a.centers[3 * k + 2]};
    double sum = 0.0;
    for (int64_t j = c0 + threadIdx.x; j < c1; j += kYawThreads) {
        const double x = a.pts[3 * j], y = a.pts[3 * j + 1];
        const double q[3] = {cs * x - sn * y, sn * x + cs * y, (double)a.pts[3 * j + 2]};
        double u[3];
        for (int d = 0; d < 3; ++d) u[d] = S[d] > 0.0 ? (q[d] - C[d]) / S[d] + 0.5 : 0.5;
        sum += prior_at(a.F, a.R, u);
    }
    sum = wave_sum(sum);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = red[0];
        for (int i = 1; i < kYawThreads / 64; ++i) t += red[i];
        a.part_sum[(int64_t)k * a.n_chunks + blockIdx.x] = t;
    }
}

// One block: scores in chunk order, then the first index of the largest.
__global__ __launch_bounds__(1024) void k_yaw_finish(YawArgs a)
{
    __shared__ double best_v[16];
    __shared__ int best_k[16];
    double bv = -INFINITY;
    int bk = 0x7fffffff;
    for (int k = threadIdx.x; k < a.K; k += 1024) {
        double t = 0.0;
        for (int64_t c = 0; c < a.n_chunks; ++c) t += a.part_sum[(int64_t)k * a.n_chunks + c];
        a.scores[k] = t;
        if (t > bv || (t == bv && k < bk)) {
            bv = t;
            bk = k;
        }
    }
    for (int d = 32; d >= 1; d >>= 1) {
        const double ov = __shfl_xor(bv, d);
        const int ok = __shfl_xor(bk, d);
        if (ov > bv || (ov == bv && ok < bk)) {
            bv = ov;
            bk = ok;
        }
    }
    if ((threadIdx.x & 63) == 0) {
        best_v[threadIdx.x >> 6] = bv;
        best_k[threadIdx.x >> 6] = bk;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 16; ++i)
            if (best_v[i] > bv || (best_v[i] == bv && best_k[i] < bk)) {
                bv = best_v[i];
                bk = best_k[i];
            }
        // every score -inf or NaN: the first yaw, as a sequential first-maximum scan gives
        *a.best = bk == 0x7fffffff ? 0 : bk;
    }
}

}  // namespace

int64_t yaw_chunks(int64_t n) { return (n + kYawChunk - 1) / kYawChunk; }

hipError_t launch_canonical_yaw(const YawArgs& a, hipStream_t s)
{
    const dim3 grid((uint32_t)a.n_chunks, (uint32_t)a.K);
    hipError_t e;
    hipLaunchKernelGGL(k_yaw_extents, grid, dim3(kYawThreads), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_yaw_combine, dim3((uint32_t)a.K), dim3(kYawThreads), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_yaw_score, grid, dim3(kYawThreads), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_yaw_finish, dim3(1), dim3(1024), 0, s, a);
    return hipGetLastError();
}

}  // namespace prenom

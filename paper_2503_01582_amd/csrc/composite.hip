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

// Wave-wide sums and scans on DPP row operations (rows of 16 lanes) with
// v_readlane for the four row results, in place of LDS-routed shuffles.
// DPP controls: quad_perm [1,0,3,2] and [2,3,0,1] (0xB1, 0x4E), row_shr:n
// (0x110 + n: lane i reads lane i - n of its row, zero below the row start),
// row_shl:n (0x100 + n: lane i reads lane i + n, zero past the row end),
// row_half_mirror (0x141), row_mirror (0x140).
template <int kCtrl>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, 0xf, 0xf, true));
}

__device__ __forceinline__ float lane_value(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Sum over the 16 lanes of each row, in every lane of the row.
__device__ __forceinline__ float row_sum(float v)
{
    v += dpp<0xB1>(v);
    v += dpp<0x4E>(v);
    v += dpp<0x141>(v);
    v += dpp<0x140>(v);
    return v;
}

// Sum over the 64 lanes, in every lane.
__device__ __forceinline__ float wave_sum(float v)
{
    v = row_sum(v);
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
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
    float v = x;  // inclusive prefix within the row
    v += dpp<0x111>(v);
    v += dpp<0x112>(v);
    v += dpp<0x114>(v);
    v += dpp<0x118>(v);
    const float r0 = lane_value(v, 15), r1 = lane_value(v, 31), r2 = lane_value(v, 47);
    const int row = lane >> 4;
    const float before = row == 0 ? 0.0f : row == 1 ? r0 : row == 2 ? r0 + r1 : (r0 + r1) + r2;
    return dpp<0x111>(v) + before;  // the previous lane's inclusive prefix (0 at a row start)
}

// exclusive suffix sum (sum over lanes above this one)
__device__ __forceinline__ float wave_excl_suffix(float x, int lane)
{
    float v = x;  // inclusive suffix within the row
    v += dpp<0x101>(v);
    v += dpp<0x102>(v);
    v += dpp<0x104>(v);
    v += dpp<0x108>(v);
    const float r1 = lane_value(v, 16), r2 = lane_value(v, 32), r3 = lane_value(v, 48);
    const int row = lane >> 4;
    const float after = row == 3 ? 0.0f : row == 2 ? r3 : row == 1 ? r2 + r3 : r1 + (r2 + r3);
    return dpp<0x101>(v) + after;  // the next lane's inclusive suffix (0 at a row end)
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

// Per-ray optional inputs (targets, background), read whether or not their
// pointer is set: a missing input is read from a valid stand-in (the ray's
// first sample record, 4 floats, and its flag byte) and replaced by its
// default only where it is used, so these loads never wait behind a branch.
struct RayExtras {
    float C[3], D, bg[3];
    uint8_t mask;
};

__device__ __forceinline__ RayExtras load_extras(const CompositeArgs& a, int64_t r)
{
    const float* stand_in = a.sc + 4 * r * a.S;
    const float* c = a.tgt_rgb ? a.tgt_rgb + 3 * r : stand_in;
    const float* d = a.tgt_depth ? a.tgt_depth + r : stand_in;
    const float* b = a.bg ? a.bg + 3 * r : stand_in;
    const uint8_t* m = a.mask ? a.mask + r : a.flags + r;
    RayExtras x;
    for (int k = 0; k < 3; ++k) {
        x.C[k] = c[k];
        x.bg[k] = b[k];
    }
    x.D = d[0];
    x.mask = m[0];
    return x;
}

struct RayTargets {
    float C[3];
    float D;
    bool obj;
};

__device__ __forceinline__ RayTargets targets_of(const CompositeArgs& a, const RayExtras& x)
{
    RayTargets tg;
    for (int k = 0; k < 3; ++k) tg.C[k] = a.tgt_rgb ? x.C[k] : 0.0f;
    tg.D = a.tgt_depth ? x.D : 0.0f;
    tg.obj = a.mask ? x.mask != 0 : true;
    return tg;
}

// One lane's sample of a 64-sample chunk of ray r: (sigma, rgb), dt and t.
// Lanes past the end of the ray read sample 0 of the ray (S >= 1) and are
// masked where the values are used (their optical depth and density count as
// zero), so the loads are unconditional and are issued together with the
// ray's other inputs.
struct SampleIn {
    float4 v;
    float dt, t;
    bool valid;
};

__device__ __forceinline__ SampleIn load_sample(const CompositeArgs& a, int64_t r, int S, int jj)
{
    SampleIn x;
    x.valid = jj < S;
    const int64_t sidx = r * S + (x.valid ? jj : 0);
    x.v = reinterpret_cast<const float4*>(a.sc)[sidx];
    x.dt = a.dt[sidx];
    x.t = a.t[sidx];
    return x;
}

__global__ __launch_bounds__(64 * kRaysPerBlock) void k_composite_fwd(CompositeArgs a)
{
    __shared__ double block_loss[kRaysPerBlock];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * kRaysPerBlock + wave;
    double ray_loss = 0.0;
    if (r < a.n_rays) {
        const int S = a.S;
        // every input of the ray is requested before the first wait
        const uint8_t flags = a.flags[r];
        const SampleIn first = load_sample(a, r, S, lane);
        const RayExtras ex = load_extras(a, r);
        float C[3] = {0.0f, 0.0f, 0.0f}, Dh = 0.0f, A = 0.0f, sig_sum = 0.0f, T_S = 1.0f;
        if (!(flags & PRENOM_FLAG_MISS)) {
            float carry = 0.0f;
            for (int c0 = 0; c0 < S; c0 += 64) {
                const SampleIn x = c0 == 0 ? first : load_sample(a, r, S, c0 + lane);
                const float4 v = x.v;
                const float tj = x.t;
                const float tau = x.valid ? v.x * x.dt : 0.0f;  // w = 0 past the end
                const float excl = wave_excl_prefix(tau, lane) + carry;
                const float w = expf(-excl) * (-expm1f(-tau));
                C[0] += w * v.y;
                C[1] += w * v.z;
                C[2] += w * v.w;
                Dh += w * tj;
                A += w;
                sig_sum += x.valid ? v.x : 0.0f;
                carry += wave_sum(tau);
            }
            for (int k = 0; k < 3; ++k) C[k] = wave_sum(C[k]);
            Dh = wave_sum(Dh);
            A = wave_sum(A);
            sig_sum = wave_sum(sig_sum);
            T_S = expf(-carry);
        }
        for (int k = 0; k < 3; ++k) C[k] += a.bg ? T_S * ex.bg[k] : 0.0f;
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
            const RayTargets tg = targets_of(a, ex);
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
    // every input of the ray is requested before the first wait
    const uint8_t flags = a.flags[r];
    const SampleIn first = load_sample(a, r, S, lane);
    const float* st = a.ray_state + 8 * r;
    const float Ch[3] = {st[0], st[1], st[2]};
    const float Dh = st[3], T_S = st[4];
    const RayExtras ex = load_extras(a, r);
    float gin[3] = {0.0f, 0.0f, 0.0f}, gdin = 0.0f, gain = 0.0f;
    if (a.d_rgb) {
        for (int k = 0; k < 3; ++k) gin[k] = a.d_rgb[3 * r + k];
        gdin = a.d_depth ? a.d_depth[r] : 0.0f;
        gain = a.d_opacity ? a.d_opacity[r] : 0.0f;
    }
    if (flags & PRENOM_FLAG_MISS) {
        for (int jj = lane; jj < S; jj += 64) dout[jj] = make_float4(0, 0, 0, 0);
        return;
    }

    // upstream gradients of this ray: dL/dC, dL/dD and the per-sample density term
    float gC[3], gD = 0.0f, gA = 0.0f, extra = 0.0f;
    if (a.d_rgb) {
        for (int k = 0; k < 3; ++k) gC[k] = gin[k];
        gD = gdin;
        gA = gain;
    } else {
        const RayTargets tg = targets_of(a, ex);
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
    if (a.bg) bg_term = T_S * (gC[0] * ex.bg[0] + gC[1] * ex.bg[1] + gC[2] * ex.bg[2]);

    // optical depth carried into each chunk (zero into the first, so a ray of
    // at most 64 samples needs no pass for it)
    const int n_chunks = (S + 63) / 64;
    float carry_in[kMaxChunks];
    carry_in[0] = 0.0f;
    if (n_chunks > 1) {
        float c = wave_sum(first.valid ? first.v.x * first.dt : 0.0f);
        for (int ch = 1; ch < n_chunks; ++ch) {
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
        const SampleIn x = ch == 0 ? first : load_sample(a, r, S, jj);
        const float4 v = x.v;
        const float dtj = x.dt;
        const float tj = x.t;
        const float tau = valid ? v.x * dtj : 0.0f;
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

// Volume rendering and losses (Sec. III-B "Volume Rendering", Eq. (5),
// (7)-(9)) and their adjoint.
//
// Sixteen lanes (one DPP row) per ray, four rays per wavefront.  A ray is
// walked in chunks of 64 samples; lane l holds samples l, l + 16, l + 32,
// l + 48 of the chunk (so each load and store of a row covers 16 consecutive
// samples).  The transmittance T_j = exp(-sum_{i<j} sigma_i delta_i) is an
// exclusive prefix scan of sigma delta along the ray and the adjoint's
// sum_{k>j} w_k a_k an exclusive suffix scan: one 16-lane row scan per sample
// slot, carried from slot to slot and from chunk to chunk.  Row scans and sums
// are DPP row operations (no LDS, no cross-row traffic), and the per-ray work
// (loss, upstream gradients) is shared by the four rays of a wavefront.  FP32
// scans; the loss is summed per block in FP64 and finished by one block.
#include "common.h"

namespace prenom {
namespace {

constexpr int kRow = 16;                        // lanes per ray
constexpr int kSlots = 4;                       // samples per lane and chunk
constexpr int kChunk = kRow * kSlots;           // 64 samples
constexpr int kWaves = 4;                       // waves per block
constexpr int kRaysPerBlock = kWaves * (64 / kRow);  // 16
constexpr int kMaxChunks = 4;                   // S <= 256

// DPP controls: quad_perm [1,0,3,2] and [2,3,0,1] (0xB1, 0x4E), row_shr:n
// (0x110 + n: lane i reads lane i - n of its row, zero below the row start),
// row_shl:n (0x100 + n: lane i reads lane i + n, zero past the row end),
// row_half_mirror (0x141), row_mirror (0x140).
template <int kCtrl>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, 0xf, 0xf, true));
}

// Sum over the 16 lanes of the row, in every lane of the row.
__device__ __forceinline__ float row_sum(float v)
{
    v += dpp<0xB1>(v);
    v += dpp<0x4E>(v);
    v += dpp<0x141>(v);
    v += dpp<0x140>(v);
    return v;
}

// Exclusive prefix sum over the lanes of the row (0 in its first lane).
__device__ __forceinline__ float row_excl_prefix(float x)
{
    float v = x;
    v += dpp<0x111>(v);
    v += dpp<0x112>(v);
    v += dpp<0x114>(v);
    v += dpp<0x118>(v);
    return dpp<0x111>(v);
}

// Exclusive suffix sum over the lanes of the row (0 in its last lane).
__device__ __forceinline__ float row_excl_suffix(float x)
{
    float v = x;
    v += dpp<0x101>(v);
    v += dpp<0x102>(v);
    v += dpp<0x104>(v);
    v += dpp<0x108>(v);
    return dpp<0x101>(v);
}

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

// Rays over which the loss of ray r is averaged: the whole call, or the
// ray's object in a batch.
__device__ __forceinline__ int64_t norm_rays(const CompositeArgs& a, int64_t r)
{
    if (!a.objs) return a.norm_rays > 0 ? a.norm_rays : a.n_rays;
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

// A lane's kSlots samples of one chunk of ray r: (sigma, rgb), dt and t.
// Samples past the end of the ray read sample 0 of the ray (S >= 1) and are
// masked where used, so every load is unconditional.
struct Slots {
    float4 v[kSlots];
    float dt[kSlots], t[kSlots];
    bool valid[kSlots];
};

__device__ __forceinline__ Slots load_slots(const CompositeArgs& a, int64_t r, int c0, int l)
{
    const int S = a.S;
    Slots x;
#pragma unroll
    for (int m = 0; m < kSlots; ++m) {
        const int j = c0 + l + kRow * m;
        x.valid[m] = j < S;
        const int64_t idx = r * S + (x.valid[m] ? j : 0);
        x.v[m] = reinterpret_cast<const float4*>(a.sc)[idx];
        x.dt[m] = a.dt[idx];
        x.t[m] = a.t[idx];
    }
    return x;
}

// Row of this lane's ray within the wave, and the ray (rows past the last ray
// work on the last ray and write nothing).
struct RayLane {
    int l, g;
    int64_t r, rc;
    bool live;
};

__device__ __forceinline__ RayLane ray_lane(const CompositeArgs& a)
{
    RayLane x;
    const int lane = threadIdx.x & 63;
    x.l = lane & (kRow - 1);
    x.g = lane / kRow;
    x.r = ((int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6)) * (64 / kRow) + x.g;
    x.live = x.r < a.n_rays;
    x.rc = x.live ? x.r : a.n_rays - 1;
    return x;
}

__global__ __launch_bounds__(64 * kWaves) void k_composite_fwd(CompositeArgs a)
{
    __shared__ double block_loss[kWaves];
    const RayLane rl = ray_lane(a);
    const int S = a.S;
    const int64_t r = rl.rc;
    // every input of the ray is requested before the first wait
    const uint8_t flags = a.flags[r];
    const Slots first = load_slots(a, r, 0, rl.l);
    const RayExtras ex = load_extras(a, r);

    float C[3] = {0.0f, 0.0f, 0.0f}, Dh = 0.0f, A = 0.0f, sig_sum = 0.0f, carry = 0.0f;
    for (int c0 = 0; c0 < S; c0 += kChunk) {
        const Slots x = c0 == 0 ? first : load_slots(a, r, c0, rl.l);
#pragma unroll
        for (int m = 0; m < kSlots; ++m) {
            const float4 v = x.v[m];
            const float tau = x.valid[m] ? v.x * x.dt[m] : 0.0f;  // w = 0 past the end
            const float excl = row_excl_prefix(tau) + carry;
            const float w = expf(-excl) * (-expm1f(-tau));
            C[0] += w * v.y;
            C[1] += w * v.z;
            C[2] += w * v.w;
            Dh += w * x.t[m];
            A += w;
            sig_sum += x.valid[m] ? v.x : 0.0f;
            carry += row_sum(tau);
        }
    }
    const bool miss = flags & PRENOM_FLAG_MISS;
    for (int k = 0; k < 3; ++k) C[k] = miss ? 0.0f : row_sum(C[k]);
    Dh = miss ? 0.0f : row_sum(Dh);
    A = miss ? 0.0f : row_sum(A);
    sig_sum = miss ? 0.0f : row_sum(sig_sum);
    const float T_S = miss ? 1.0f : expf(-carry);
    for (int k = 0; k < 3; ++k) C[k] += a.bg ? T_S * ex.bg[k] : 0.0f;
    if (rl.l == 0 && rl.live) {
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
    double ray_loss = 0.0;
    if (a.tgt_rgb && rl.live) {
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
    if (a.ray_loss && rl.l == 0 && rl.live) a.ray_loss[r] = ray_loss;
    if (a.loss_partial) {
        // the wave's rays in row order, then the waves in order
        double wl = 0.0;
#pragma unroll
        for (int g = 0; g < 64 / kRow; ++g) {
            const double v = __shfl(ray_loss, g * kRow);
            wl += v;
        }
        if ((threadIdx.x & 63) == 0) block_loss[threadIdx.x >> 6] = wl;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < kWaves; ++w) s += block_loss[w];
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

// One block per object (a batch has few objects, so each block takes 16
// waves and keeps four loads in flight per thread); the sums run in a fixed
// order.
constexpr int kLossObjThreads = 1024;
__global__ __launch_bounds__(kLossObjThreads) void k_loss_objects(const ObjDev* __restrict__ objs,
                                                                  const double* __restrict__ ray_loss, float* loss)
{
    __shared__ double red[kLossObjThreads / 64];
    const ObjDev& o = objs[blockIdx.x];
    const double* rl = ray_loss + o.ray_begin;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t i = threadIdx.x;
    for (; i + 3 * kLossObjThreads < o.n_rays; i += 4 * kLossObjThreads) {
#pragma unroll
        for (int u = 0; u < 4; ++u) s[u] += rl[i + u * kLossObjThreads];
    }
    for (; i < o.n_rays; i += kLossObjThreads) s[0] += rl[i];
    double t = wave_sum_d((s[0] + s[1]) + (s[2] + s[3]));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < kLossObjThreads / 64; ++w) tot += red[w];
        loss[blockIdx.x] = (float)tot;
    }
}

__global__ __launch_bounds__(64 * kWaves) void k_composite_bwd(CompositeArgs a)
{
    const RayLane rl = ray_lane(a);
    const int S = a.S;
    const int64_t r = rl.rc;
    // every input of the ray is requested before the first wait
    const uint8_t flags = a.flags[r];
    const Slots first = load_slots(a, r, 0, rl.l);
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
    const bool miss = flags & PRENOM_FLAG_MISS;

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

    // optical depth carried into each chunk (zero into the first)
    const int n_chunks = (S + kChunk - 1) / kChunk;
    float carry_in[kMaxChunks];
    carry_in[0] = 0.0f;
    if (n_chunks > 1) {
        float c = 0.0f;
#pragma unroll
        for (int m = 0; m < kSlots; ++m) c += row_sum(first.valid[m] ? first.v[m].x * first.dt[m] : 0.0f);
        for (int ch = 1; ch < n_chunks; ++ch) {
            carry_in[ch] = c;
            const Slots x = load_slots(a, r, ch * kChunk, rl.l);
#pragma unroll
            for (int m = 0; m < kSlots; ++m) c += row_sum(x.valid[m] ? x.v[m].x * x.dt[m] : 0.0f);
        }
    }
    float4* dout = reinterpret_cast<float4*>(a.dout) + r * S;
    float suffix_carry = 0.0f;
    for (int ch = n_chunks - 1; ch >= 0; --ch) {
        const int c0 = ch * kChunk;
        const Slots x = ch == 0 ? first : load_slots(a, r, c0, rl.l);
        // forward quantities of the chunk's slots, in ray order
        float tau[kSlots], excl[kSlots], w[kSlots], aj[kSlots], wa[kSlots];
        float carry = carry_in[ch];
#pragma unroll
        for (int m = 0; m < kSlots; ++m) {
            const float4 v = x.v[m];
            tau[m] = x.valid[m] ? v.x * x.dt[m] : 0.0f;
            excl[m] = row_excl_prefix(tau[m]) + carry;
            carry += row_sum(tau[m]);
            w[m] = expf(-excl[m]) * (-expm1f(-tau[m]));
            aj[m] = gC[0] * v.y + gC[1] * v.z + gC[2] * v.w + gD * x.t[m] + gA;
            wa[m] = x.valid[m] ? w[m] * aj[m] : 0.0f;
        }
        // adjoint: suffix sums of w a, last slot first
#pragma unroll
        for (int m = kSlots - 1; m >= 0; --m) {
            const float suffix = row_excl_suffix(wa[m]) + suffix_carry;
            suffix_carry += row_sum(wa[m]);
            const float Tj1 = expf(-(excl[m] + tau[m]));
            const float dsig = x.dt[m] * (Tj1 * aj[m] - suffix - bg_term) + extra;
            const int j = c0 + rl.l + kRow * m;
            if (rl.live && j < S)
                dout[j] = miss ? make_float4(0.0f, 0.0f, 0.0f, 0.0f)
                               : make_float4(dsig, w[m] * gC[0], w[m] * gC[1], w[m] * gC[2]);
        }
    }
}

}  // namespace

// Forward blocks (one loss partial each): kWaves waves of 64 / kRow rays.
int composite_loss_blocks(int64_t n_rays) { return (int)((n_rays + kRaysPerBlock - 1) / kRaysPerBlock); }
int composite_rays_per_block() { return kRaysPerBlock; }

hipError_t launch_composite_fwd(const CompositeArgs& a, hipStream_t s)
{
    if (a.n_rays == 0) return hipSuccess;
    hipLaunchKernelGGL(k_composite_fwd, dim3((uint32_t)composite_loss_blocks(a.n_rays)), dim3(64 * kWaves), 0, s, a);
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
    hipLaunchKernelGGL(k_loss_objects, dim3((uint32_t)n_obj), dim3(kLossObjThreads), 0, s, objs, ray_loss, loss);
    return hipGetLastError();
}

hipError_t launch_composite_bwd(const CompositeArgs& a, hipStream_t s)
{
    if (a.n_rays == 0) return hipSuccess;
    hipLaunchKernelGGL(k_composite_bwd, dim3((uint32_t)composite_loss_blocks(a.n_rays)), dim3(64 * kWaves), 0, s, a);
    return hipGetLastError();
}

}  // namespace prenom

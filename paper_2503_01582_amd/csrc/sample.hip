// Prior-based probabilistic ray sampling (Sec. III-B "Probabilistic Ray
// Sampling", Eq. (4)-(6) and the escape rule).
//
// One thread per ray.  The whole decision chain (object-frame transform, slab
// test, coarse midpoints, trilinear prior lookup, prefix sums of
// sigma_i * delta_i, the expm1 ratio that forms the CDF, the comparison with
// u_k) is evaluated in FP64 with contraction disabled, so the sampled bins do
// not hinge on FP32 rounding.  The CDF is never stored: the ray is walked
// twice over its N_c coarse bins -- once for the total mass, once merged with
// the ascending draws u_k -- recomputing each bin's prior value, which keeps
// the kernel free of per-thread arrays (no scratch memory).
#include "common.h"

#pragma clang fp contract(off)

namespace prenom {
namespace {

constexpr int kSampleBlock = 128;

// Trilinear, vertex-aligned lookup (value F[i] at i/(R-1)), x clamped.
__device__ double prior_at(const float* __restrict__ F, int R, const double xin[3])
{
    int i0[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double x = xin[a];
        x = x >= 0.0 ? x : 0.0;  // also maps NaN to 0
        x = x > 1.0 ? 1.0 : x;
        const double g = x * (double)(R - 1);
        int i = (int)floor(g);
        i = i > R - 2 ? R - 2 : i;
        i0[a] = i;
        f[a] = g - (double)i;
    }
    double s = 0.0;
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
                const double wx = cx ? f[0] : 1.0 - f[0];
                const double wy = cy ? f[1] : 1.0 - f[1];
                const double wz = cz ? f[2] : 1.0 - f[2];
                const double w = wx * wy * wz;
                const int64_t idx = (int64_t)(i0[0] + cx) +
                                    (int64_t)R * ((int64_t)(i0[1] + cy) + (int64_t)R * (i0[2] + cz));
                s += w * (double)F[idx];
            }
    return s;
}

struct RayFrame {
    double o[3], d[3];
    double tn, tf, len, delta;
};

// sigma_i * delta_i of coarse bin i (Eq. (4) with sigma_i = F(x_i)).
__device__ __forceinline__ double coarse_tau(const float* prior, int R, const RayFrame& r, int i)
{
    const double m = r.tn + ((double)i + 0.5) * r.delta;
    double x[3];
    for (int k = 0; k < 3; ++k) {
        double v = fma(m, r.d[k], r.o[k]);
        v = v >= 0.0 ? v : 0.0;
        v = v > 1.0 ? 1.0 : v;
        x[k] = v;
    }
    const double sig = prior_at(prior, R, x);
    return sig * r.delta * r.len;
}

// One ray.  A, prior and R are the ray's object's pose and prior (per
// object in a batch); everything else comes from `a`.
__device__ void sample_ray(const SampleArgs& a, const double* A_obj, const float* prior, int R, bool use_prior,
                           int64_t ray)
{
    const int Nc = a.n_coarse, Nr = a.n_fine;
    const int S = Nr + (a.include_coarse ? Nc : 0);

    RayFrame r;
    const float* ow = a.rays_o + 3 * ray;
    const float* dw = a.rays_d + 3 * ray;
    for (int k = 0; k < 3; ++k) {
        const double* A = A_obj + 4 * k;
        r.o[k] = A[0] * (double)ow[0] + A[1] * (double)ow[1] + A[2] * (double)ow[2] + A[3];
        r.d[k] = A[0] * (double)dw[0] + A[1] * (double)dw[1] + A[2] * (double)dw[2];
    }
    float* ro = a.ray_obj + 6 * ray;
    for (int k = 0; k < 3; ++k) {
        ro[k] = (float)r.o[k];
        ro[3 + k] = (float)r.d[k];
    }

    // slab test against [0,1]^3 and [near, far]
    double t_enter = -INFINITY, t_exit = INFINITY;
    bool hit = true;
    for (int k = 0; k < 3; ++k) {
        if (r.d[k] == 0.0) {
            if (r.o[k] < 0.0 || r.o[k] > 1.0) hit = false;
            continue;
        }
        const double ta = (0.0 - r.o[k]) / r.d[k];
        const double tb = (1.0 - r.o[k]) / r.d[k];
        const double lo = ta < tb ? ta : tb;
        const double hi = ta < tb ? tb : ta;
        t_enter = lo > t_enter ? lo : t_enter;
        t_exit = hi < t_exit ? hi : t_exit;
    }
    r.tn = a.near_t > t_enter ? a.near_t : t_enter;
    r.tf = a.far_t < t_exit ? a.far_t : t_exit;
    hit = hit && (r.tn < r.tf);

    float* tr = a.t + (int64_t)S * ray;
    float* dtr = a.dt + (int64_t)S * ray;
    int32_t* br = a.bins + (int64_t)Nr * ray;
    const float* xr = a.xi + (int64_t)Nr * ray;
    if (!hit) {
        for (int j = 0; j < S; ++j) {
            tr[j] = 0.0f;
            dtr[j] = 0.0f;
        }
        for (int k = 0; k < Nr; ++k) br[k] = -1;
        a.flags[ray] = PRENOM_FLAG_MISS;
        return;
    }
    r.len = sqrt(r.d[0] * r.d[0] + r.d[1] * r.d[1] + r.d[2] * r.d[2]);
    r.delta = Nc > 0 ? (r.tf - r.tn) / (double)Nc : 0.0;

    // pass 1: total prior mass along the ray
    bool escaped = false;
    double total_S = 0.0;
    if (use_prior) {
        for (int i = 0; i < Nc; ++i) total_S = total_S + coarse_tau(prior, R, r, i);
        escaped = (-expm1(-total_S)) < a.eps;
    }
    const bool cdf_draws = use_prior && !escaped;
    a.flags[ray] = (uint8_t)((use_prior ? 0 : PRENOM_FLAG_UNIFORM) | (escaped ? PRENOM_FLAG_ESCAPED : 0));

    // pass 2: draws in ascending u, merged with the coarse midpoints
    const double den = expm1(-total_S);
    int b = 0;
    double S_b1 = 0.0, C_b = 0.0, C_b1 = 1.0;
    if (cdf_draws) {
        S_b1 = 0.0 + coarse_tau(prior, R, r, 0);
        C_b1 = (Nc == 1) ? 1.0 : expm1(-S_b1) / den;
    }
    int ic = 0, j = 0;
    double prev = 0.0;
    auto emit = [&](double tv) {
        if (j > 0) dtr[j - 1] = (float)((tv - prev) * r.len);
        tr[j] = (float)tv;
        prev = tv;
        ++j;
    };
    for (int k = 0; k < Nr; ++k) {
        const double u = ((double)k + (double)xr[k]) / (double)Nr;
        double tk;
        if (!cdf_draws) {
            tk = r.tn + u * (r.tf - r.tn);
            br[k] = -1;
        } else {
            while (b + 1 < Nc && C_b1 < u) {  // the last CDF value is 1 > u for xi in (0,1)
                ++b;
                C_b = C_b1;
                S_b1 = S_b1 + coarse_tau(prior, R, r, b);
                C_b1 = (b + 1 == Nc) ? 1.0 : expm1(-S_b1) / den;
            }
            tk = r.tn + r.delta * ((double)b + (u - C_b) / (C_b1 - C_b));
            br[k] = b;
        }
        if (a.include_coarse) {
            while (ic < Nc) {
                const double m = r.tn + ((double)ic + 0.5) * r.delta;
                if (!(m <= tk)) break;
                emit(m);
                ++ic;
            }
        }
        emit(tk);
    }
    if (a.include_coarse)
        for (; ic < Nc; ++ic) emit(r.tn + ((double)ic + 0.5) * r.delta);
    dtr[S - 1] = (float)((r.tf - prev) * r.len);
}

__global__ __launch_bounds__(kSampleBlock) void k_sample(SampleArgs a)
{
    const int64_t ray = (int64_t)blockIdx.x * kSampleBlock + threadIdx.x;
    if (ray >= a.n) return;
    sample_ray(a, a.A, a.prior, a.R, a.use_prior != 0, ray);
}

// All rays of a batch: the ray's object (last with ray_begin <= ray) supplies
// pose and prior; a.use_prior == 0 forces uniform draws for every object.
__global__ __launch_bounds__(kSampleBlock) void k_sample_batch(SampleArgs a, const ObjDev* __restrict__ objs, int n_obj)
{
    const int64_t ray = (int64_t)blockIdx.x * kSampleBlock + threadIdx.x;
    if (ray >= a.n) return;
    const ObjDev& o = objs[find_object(objs, n_obj, ray)];
    sample_ray(a, o.A, o.prior, o.prior_res, a.use_prior != 0 && o.prior != nullptr, ray);
}

}  // namespace

hipError_t launch_sample_batch(const SampleArgs& a, const ObjDev* objs, int n_obj, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    const int64_t blocks = (a.n + kSampleBlock - 1) / kSampleBlock;
    hipLaunchKernelGGL(k_sample_batch, dim3((uint32_t)blocks), dim3(kSampleBlock), 0, s, a, objs, n_obj);
    return hipGetLastError();
}

hipError_t launch_sample(const SampleArgs& a, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    const int64_t blocks = (a.n + kSampleBlock - 1) / kSampleBlock;
    hipLaunchKernelGGL(k_sample, dim3((uint32_t)blocks), dim3(kSampleBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace prenom

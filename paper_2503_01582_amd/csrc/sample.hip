// Prior-based probabilistic ray sampling (Sec. III-B "Probabilistic Ray
// Sampling", Eq. (4)-(6) and the escape rule).
//
// One group of kRayLanes lanes per ray, four rays per wavefront.  The whole
// decision chain (object-frame transform, slab test, coarse midpoints,
// trilinear prior lookup, prefix sums of sigma_i * delta_i, the expm1 ratio
// that forms the CDF, the comparison with u_k) is evaluated in FP64 with
// contraction disabled, so the sampled bins do not hinge on FP32 rounding.
// The lanes of a group share the work of one ray:
//
//   * the N_c coarse bins' sigma_i * delta_i, bins spread over the lanes
//     (prior lookups in parallel), kept in LDS;
//   * the CDF value at the end of each bin, each lane summing the bins before
//     its own in bin order (the same FP64 additions, in the same order, as a
//     single sequential pass);
//   * the draws u_k, spread over the lanes: the bin of draw k is the first bin whose
//     CDF end reaches u_k, found by binary search when the CDF ends do not
//     decrease (always, for a non-negative prior); otherwise one lane walks
//     the bins for all draws in order;
//   * the merge of draws and midpoints by rank: before draw k come the
//     midpoints not above any earlier draw (a running maximum of per-draw
//     counts), before midpoint i the draws whose running count is <= i;
//   * t and dt written by consecutive lanes (coalesced).
#include "common.h"

#pragma clang fp contract(off)

namespace prenom {
namespace {

constexpr int kRayLanes = 16;                    // lanes per ray
constexpr int kRaysPerBlock = 64 / kRayLanes;    // rays per wavefront (one wavefront per block)

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

// LDS of one ray: tau[N_c], cdf[N_c] (FP64), draws[N_r] (FP64), out[S]
// (FP64), run[N_r] (int32 running midpoint counts), bin[N_r] (int32).
__host__ __device__ constexpr size_t sample_lds_bytes(int Nc, int Nr, int S)
{
    return (size_t)(2 * Nc + Nr + S) * sizeof(double) + (size_t)2 * Nr * sizeof(int32_t);
}

// Number of midpoints i in [0, Nc) with m_i <= tk (m_i ascends in i).
__device__ __forceinline__ int midpoints_upto(const RayFrame& r, int Nc, double tk)
{
    int lo = 0, hi = Nc;  // answer in [lo, hi]
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const double m = r.tn + ((double)mid + 0.5) * r.delta;
        if (m <= tk)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// One ray, by the kRayLanes lanes of one group of the wavefront (lane: the
// lane within the group; every lane of the group takes the same path, and
// shuffles stay inside the group).  A, prior and R are the ray's object's
// pose and prior (per object in a batch); everything else comes from `a`;
// lds is the group's own region.
__device__ void sample_ray(const SampleArgs& a, const double* A_obj, const float* prior, int R, bool use_prior,
                           int64_t ray, double* lds)
{
    constexpr int G = kRayLanes;
    const int lane = threadIdx.x % G;
    const uint64_t group_mask = ((1ull << G) - 1ull) << (threadIdx.x / G * G % 64);
    const int Nc = a.n_coarse, Nr = a.n_fine;
    const int S = Nr + (a.include_coarse ? Nc : 0);
    double* tau = lds;
    double* cdf = tau + Nc;
    double* draws = cdf + Nc;
    double* out = draws + Nr;
    int32_t* run = reinterpret_cast<int32_t*>(out + S);
    int32_t* bin = run + Nr;

    RayFrame r;
    const float* ow = a.rays_o + 3 * ray;
    const float* dw = a.rays_d + 3 * ray;
    for (int k = 0; k < 3; ++k) {
        const double* A = A_obj + 4 * k;
        r.o[k] = A[0] * (double)ow[0] + A[1] * (double)ow[1] + A[2] * (double)ow[2] + A[3];
        r.d[k] = A[0] * (double)dw[0] + A[1] * (double)dw[1] + A[2] * (double)dw[2];
    }
    if (lane < 6) {  // constant indices only, so the frame stays in registers
        const double v = lane == 0 ? r.o[0] : lane == 1 ? r.o[1] : lane == 2 ? r.o[2]
                       : lane == 3 ? r.d[0] : lane == 4 ? r.d[1] : r.d[2];
        a.ray_obj[6 * ray + lane] = (float)v;
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
        for (int j = lane; j < S; j += G) {
            tr[j] = 0.0f;
            dtr[j] = 0.0f;
        }
        for (int k = lane; k < Nr; k += G) br[k] = -1;
        if (lane == 0) a.flags[ray] = PRENOM_FLAG_MISS;
        return;
    }
    r.len = sqrt(r.d[0] * r.d[0] + r.d[1] * r.d[1] + r.d[2] * r.d[2]);
    r.delta = Nc > 0 ? (r.tf - r.tn) / (double)Nc : 0.0;

    // coarse bins: sigma_i delta_i, then the total mass (bin order)
    if (use_prior)
        for (int i = lane; i < Nc; i += G) tau[i] = coarse_tau(prior, R, r, i);
    __syncthreads();
    bool escaped = false;
    double total_S = 0.0;
    if (use_prior) {
        for (int i = 0; i < Nc; ++i) total_S = total_S + tau[i];
        escaped = (-expm1(-total_S)) < a.eps;
    }
    const bool cdf_draws = use_prior && !escaped;
    if (lane == 0)
        a.flags[ray] = (uint8_t)((use_prior ? 0 : PRENOM_FLAG_UNIFORM) | (escaped ? PRENOM_FLAG_ESCAPED : 0));

    // CDF at the end of each bin (1 at the last): prefix of the bins in order
    const double den = expm1(-total_S);
    bool ascending = true;
    if (cdf_draws) {
        for (int b = lane; b < Nc; b += G) {
            double Sb = 0.0;
            for (int i = 0; i <= b; ++i) Sb = Sb + tau[i];
            cdf[b] = (b + 1 == Nc) ? 1.0 : expm1(-Sb) / den;
        }
        __syncthreads();
        // Searching each draw's bin on its own equals the walk when the CDF
        // ends below the last bin do not decrease and the draws u_k do not
        // either (both hold for a non-negative prior and xi in [0, 1]).
        for (int b = lane; b + 2 < Nc; b += G)
            if (!(cdf[b] <= cdf[b + 1])) ascending = false;
        for (int k = lane; k + 1 < Nr; k += G)
            if (!(((double)k + (double)xr[k]) / (double)Nr <= ((double)(k + 1) + (double)xr[k + 1]) / (double)Nr))
                ascending = false;
        ascending = (__ballot(!ascending) & group_mask) == 0;  // over the group's lanes
        __syncthreads();
        if (!ascending && lane == 0) {  // sequential walk over the draws, in order
            int bb = 0;
            for (int k = 0; k < Nr; ++k) {
                const double u = ((double)k + (double)xr[k]) / (double)Nr;
                while (bb + 1 < Nc && cdf[bb] < u) ++bb;
                bin[k] = bb;
            }
        }
        __syncthreads();
    }

    // draws: inverse CDF within the bin (Eq. (6)), or uniform in [tn, tf]
    for (int k = lane; k < Nr; k += G) {
        const double u = ((double)k + (double)xr[k]) / (double)Nr;
        double tk;
        int bk = -1;
        if (!cdf_draws) {
            tk = r.tn + u * (r.tf - r.tn);
        } else {
            if (ascending) {  // first b in [0, Nc - 1) with cdf[b] >= u, else Nc - 1
                int lo = 0, hi = Nc - 1;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (cdf[mid] < u)
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                bk = lo;
            } else {
                bk = bin[k];
            }
            const double C_b = bk == 0 ? 0.0 : cdf[bk - 1];
            const double C_b1 = cdf[bk];
            tk = r.tn + r.delta * ((double)bk + (u - C_b) / (C_b1 - C_b));
        }
        br[k] = bk;
        draws[k] = tk;
        run[k] = a.include_coarse ? midpoints_upto(r, Nc, tk) : 0;
    }
    __syncthreads();

    // ranks: midpoints emitted before draw k = max over k' <= k of the counts
    if (a.include_coarse) {
        int carry = 0;  // running maximum, G draws at a time
        for (int k0 = 0; k0 < Nr; k0 += G) {
            const int k = k0 + lane;
            int v = k < Nr ? run[k] : 0;
#pragma unroll
            for (int d = 1; d < G; d <<= 1) {
                const int up = __shfl_up(v, d, G);
                if (lane >= d) v = v > up ? v : up;
            }
            v = v > carry ? v : carry;
            if (k < Nr) run[k] = v;
            carry = __shfl(v, G - 1, G);
        }
        __syncthreads();
        for (int k = lane; k < Nr; k += G) out[k + run[k]] = draws[k];
        for (int i = lane; i < Nc; i += G) {
            int lo = 0, hi = Nr;  // draws before midpoint i: first k with run[k] > i
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (run[mid] <= i)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            out[i + lo] = r.tn + ((double)i + 0.5) * r.delta;
        }
    } else {
        for (int k = lane; k < Nr; k += G) out[k] = draws[k];
    }
    __syncthreads();
    for (int j = lane; j < S; j += G) {
        const double tv = out[j];
        const double next = j + 1 < S ? out[j + 1] : r.tf;
        tr[j] = (float)tv;
        dtr[j] = (float)((next - tv) * r.len);
    }
}

// LDS of one ray, in doubles (the regions of a block's rays follow each other).
__device__ __forceinline__ size_t ray_lds_doubles(const SampleArgs& a)
{
    return sample_lds_bytes(a.n_coarse, a.n_fine, a.n_fine + (a.include_coarse ? a.n_coarse : 0)) / sizeof(double);
}

__global__ __launch_bounds__(64) void k_sample(SampleArgs a)
{
    extern __shared__ double lds[];
    const int g = threadIdx.x / kRayLanes;
    const int64_t ray = (int64_t)blockIdx.x * kRaysPerBlock + g;
    if (ray >= a.n) return;  // the whole group
    sample_ray(a, a.A, a.prior, a.R, a.use_prior != 0, ray, lds + g * ray_lds_doubles(a));
}

// All rays of a batch: the ray's object (last with ray_begin <= ray) supplies
// pose and prior; a.use_prior == 0 forces uniform draws for every object.
__global__ __launch_bounds__(64) void k_sample_batch(SampleArgs a, const ObjDev* __restrict__ objs, int n_obj)
{
    extern __shared__ double lds[];
    const int g = threadIdx.x / kRayLanes;
    const int64_t ray = (int64_t)blockIdx.x * kRaysPerBlock + g;
    if (ray >= a.n) return;  // the whole group
    const ObjDev& o = objs[find_object(objs, n_obj, ray)];
    sample_ray(a, o.A, o.prior, o.prior_res, a.use_prior != 0 && o.prior != nullptr, ray,
               lds + g * ray_lds_doubles(a));
}

size_t sample_lds(const SampleArgs& a)
{
    return kRaysPerBlock * sample_lds_bytes(a.n_coarse, a.n_fine, a.n_fine + (a.include_coarse ? a.n_coarse : 0));
}

}  // namespace

// One block (one wavefront) per kRaysPerBlock rays.
hipError_t launch_sample_batch(const SampleArgs& a, const ObjDev* objs, int n_obj, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    const int64_t blocks = (a.n + kRaysPerBlock - 1) / kRaysPerBlock;
    if (blocks > (int64_t)UINT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sample_batch, dim3((uint32_t)blocks), dim3(64), sample_lds(a), s, a, objs, n_obj);
    return hipGetLastError();
}

hipError_t launch_sample(const SampleArgs& a, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    const int64_t blocks = (a.n + kRaysPerBlock - 1) / kRaysPerBlock;
    if (blocks > (int64_t)UINT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sample, dim3((uint32_t)blocks), dim3(64), sample_lds(a), s, a);
    return hipGetLastError();
}

}  // namespace prenom

// Multi-resolution hash encoding, forward (Sec. III-B "Object-level NeRFs":
// sample positions are normalised and encoded with the hash grid of Mueller
// et al. 2022 before the MLP).  The backward lives in scatter.hip.
//
// Layout: tables [L][T][2] (one float2 per row), features y level-major
// [L][n_samples][2], so a wavefront of one level writes 64 consecutive float2
// (512 contiguous bytes).  The launch grid is (sample blocks, levels): one
// thread per (sample, level), 8 float2 gathers each.
#include "common.h"

namespace prenom {
namespace {

constexpr int kEncBlock = 256;

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float2 to_f2(float2 v) { return v; }
__device__ __forceinline__ float2 to_f2(half2_t v) { return make_float2((float)v[0], (float)v[1]); }

// Two consecutive table rows (an aligned row pair), and one row read through
// a buffer resource.
template <typename Row>
struct RowPair;
template <>
struct RowPair<float2> {
    typedef float4 type;
    __device__ static float2 lo(float4 v) { return make_float2(v.x, v.y); }
    __device__ static float2 hi(float4 v) { return make_float2(v.z, v.w); }
    __device__ static float2 row(__amdgpu_buffer_rsrc_t r, uint32_t off)
    {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
        return make_float2(__uint_as_float(v[0]), __uint_as_float(v[1]));
    }
};
template <>
struct RowPair<half2_t> {
    typedef half4_t type;
    __device__ static float2 lo(half4_t v) { return make_float2((float)v[0], (float)v[1]); }
    __device__ static float2 hi(half4_t v) { return make_float2((float)v[2], (float)v[3]); }
    __device__ static float2 row(__amdgpu_buffer_rsrc_t r, uint32_t off)
    {
        const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
        return to_f2(__builtin_bit_cast(half2_t, v));
    }
};

// Raw buffer descriptor over `bytes` bytes at p (third word for the gfx9
// family: raw, untyped 32-bit data).  Loads at offsets past `bytes` return
// zero without a memory access.  p and bytes are the same in every lane (one
// level table per block); reading them from the first lane keeps the
// descriptor in scalar registers.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_buffer(const void* p, uint32_t bytes)
{
    // readfirstlane returns int: each word goes through uint32_t so that the
    // low word is zero-extended, not sign-extended, into the 64-bit address.
    const uint64_t a = (uint64_t)(uintptr_t)p;
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32));
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
    const uint64_t u = ((uint64_t)hi << 32) | (uint64_t)lo;
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>((uintptr_t)u), (short)0,
                                             __builtin_amdgcn_readfirstlane((int)bytes), 0x00020000);
}
constexpr uint32_t kOutOfRange = 0x80000000u;  // past any level table (T <= 2^24 rows of <= 8 bytes)

// Table rows are float2 (FP32 tables) or two halves (the FP16 copy).
// Plain gather: the 8 corner rows, all loads issued before the blend.
template <typename Row>
__device__ __forceinline__ float2 gather_blend_rows(const Row* __restrict__ level_table, const Corners& c)
{
    Row v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = level_table[c.row[e]];
    float2 acc = make_float2(0.0f, 0.0f);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const float2 f = to_f2(v[e]);
        acc.x = fmaf(c.w[e], f.x, acc.x);
        acc.y = fmaf(c.w[e], f.y, acc.y);
    }
    return acc;
}

// Paired gather.  Corners 2p and 2p + 1 differ only in x; on a hashed level
// their rows share an aligned row pair whenever x is even (x and x + 1 then
// hash to rows differing in bit 0 only).  Each pair is fetched as one aligned
// two-row load, plus a one-row buffer load whose offset is out of range (no
// memory access) in the lanes whose second corner lies inside that pair:
// about 1.5 cache-line requests per corner pair instead of 2, with no
// branches.  The blend adds the corners in the order e = 0..7 as above.
template <typename Row>
__device__ __forceinline__ float2 gather_blend_pairs(const Row* __restrict__ level_table, uint32_t n_rows,
                                                     const Corners& c)
{
    typedef RowPair<Row> RP;
    const __amdgpu_buffer_rsrc_t rsrc = raw_buffer(level_table, n_rows * (uint32_t)sizeof(Row));
    typename RP::type pv[4];
    float2 other[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {  // issue all loads first
        const uint32_t r0 = c.row[2 * p], r1 = c.row[2 * p + 1];
        pv[p] = *reinterpret_cast<const typename RP::type*>(level_table + (r0 & ~1u));
        other[p] = RP::row(rsrc, (r0 >> 1) != (r1 >> 1) ? r1 * (uint32_t)sizeof(Row) : kOutOfRange);
    }
    float2 acc = make_float2(0.0f, 0.0f);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const uint32_t r0 = c.row[2 * p], r1 = c.row[2 * p + 1];
        const float2 lo = RP::lo(pv[p]), hi = RP::hi(pv[p]);
        const float2 f0 = (r0 & 1u) ? hi : lo;
        const float2 f1 = (r0 >> 1) != (r1 >> 1) ? other[p] : ((r1 & 1u) ? hi : lo);
        acc.x = fmaf(c.w[2 * p], f0.x, acc.x);
        acc.y = fmaf(c.w[2 * p], f0.y, acc.y);
        acc.x = fmaf(c.w[2 * p + 1], f1.x, acc.x);
        acc.y = fmaf(c.w[2 * p + 1], f1.y, acc.y);
    }
    return acc;
}

// Hashed levels of at least 2^kPairMinLog2 rows take the paired gather; the
// others (dense levels, small tables), whose corner rows mostly hit in cache
// anyway, take the plain one.  The choice is the same for the whole block.
// Measured on gfx950 (single object, 65536 rays x 64 samples, 16 levels of
// 2^19 rows): 1.11 ms paired against 1.24 ms plain.  The batched encode keeps
// the plain gather: on 24 objects with tables of 2^14..2^19 rows the paired
// one was slower at every threshold tried (3.84 ms from 2^17, 3.98 ms from
// 2^14, against 3.69 ms plain).
constexpr int kPairMinLog2 = 17;

template <typename Row>
__device__ __forceinline__ float2 gather_blend(const Row* __restrict__ level_table, const GridInfo& g, int l,
                                               const Corners& c)
{
    const bool dense = (g.dense_mask >> l) & 1u;
    if (!dense && g.log2_table >= kPairMinLog2) return gather_blend_pairs(level_table, 1u << g.log2_table, c);
    return gather_blend_rows(level_table, c);
}

template <typename Row>
__global__ __launch_bounds__(kEncBlock) void k_encode_samples(GridInfo g, const Row* __restrict__ table,
                                                              const float* __restrict__ ray_obj,
                                                              const float* __restrict__ t, int64_t n_s,
                                                              int32_t S, float2* __restrict__ y)
{
    const int64_t s = (int64_t)blockIdx.x * kEncBlock + threadIdx.x;
    const int l = blockIdx.y;
    if (s >= n_s) return;
    const int64_t ray = s / S;
    const float* ro = ray_obj + 6 * ray;
    const float ts = t[s];
    Corners c;
    level_corners(g, l, sample_coord(ts, ro[3], ro[0]), sample_coord(ts, ro[4], ro[1]),
                  sample_coord(ts, ro[5], ro[2]), c);
    const Row* lt = table + ((int64_t)l << g.log2_table);
    y[(int64_t)l * n_s + s] = gather_blend(lt, g, l, c);
}

// The same, one block per (level, block of kScatterBlockSamples samples), also
// counting the records of the hash-table gradient in an LDS histogram over
// the level's table tiles: one per corner of every sample, except that a
// corner repeating the previous lane's row joins that lane's record
// (run_heads); place applies the same rule to the same corners.
template <typename Row>
__global__ __launch_bounds__(kScatterBlockSamples) void k_encode_samples_hist(GridInfo g, const Row* __restrict__ table,
                                                                          const float* __restrict__ ray_obj,
                                                                          const float* __restrict__ t, int64_t n_s,
                                                                          int32_t S, float2* __restrict__ y,
                                                                          TileHist h)
{
    __shared__ uint32_t hist[kMaxTilesPerLevel];
    const int l = blockIdx.y;
    const int bx = blockIdx.x;
    const int nt = h.tiles[l];
    for (int i = threadIdx.x; i < nt; i += kScatterBlockSamples) hist[i] = 0;
    __syncthreads();
    const int64_t s = (int64_t)bx * kScatterBlockSamples + threadIdx.x;
    const bool has = s < n_s;  // a prefix of every wave
    const int64_t sc = has ? s : n_s - 1;
    const float* ro = ray_obj + 6 * (sc / S);
    const float ts = t[sc];
    Corners c;
    level_corners(g, l, sample_coord(ts, ro[3], ro[0]), sample_coord(ts, ro[4], ro[1]),
                  sample_coord(ts, ro[5], ro[2]), c);
    const uint32_t heads = run_heads(c, has);  // one record per run of a repeated corner
    if (has) {
        const Row* lt = table + ((int64_t)l << g.log2_table);
        y[(int64_t)l * n_s + s] = gather_blend(lt, g, l, c);
    }
    count_records(hist, c, heads, nt);
    __syncthreads();
    uint32_t* out = h.counts + (int64_t)h.tile_base[l] * h.n_blocks + bx;
    for (int i = threadIdx.x; i < nt; i += kScatterBlockSamples) out[(int64_t)i * h.n_blocks] = hist[i];
}

// Batched, with the tile histograms: one block per item (object, level,
// block of kScatterBlockSamples samples) of the batch's hash-table gradient,
// numbered as its scatter numbers them (sobjs[i] and objs[i] describe object
// i); the same run rule as k_encode_samples_hist.
__global__ __launch_bounds__(kScatterBlockSamples) void k_encode_batch_hist(const ObjDev* __restrict__ objs,
                                                                        const ScatterObj* __restrict__ sobjs,
                                                                        int n_obj, const float* __restrict__ params,
                                                                        const half2_t* __restrict__ params_f16,
                                                                        const float* __restrict__ ray_obj,
                                                                        const float* __restrict__ t, int32_t S,
                                                                        float2* __restrict__ y,
                                                                        uint32_t* __restrict__ counts)
{
    __shared__ uint32_t hist[kMaxTilesPerLevel];
    const int64_t item = blockIdx.x;
    int lo = 0, hi = n_obj - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sobjs[mid].item_off <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    const ScatterObj& so = sobjs[lo];
    const ObjDev& o = objs[lo];
    const uint32_t rem = (uint32_t)(item - so.item_off);
    const int l = (int)(rem / (uint32_t)so.n_blocks);
    const int bx = (int)(rem - (uint32_t)l * (uint32_t)so.n_blocks);
    const int nt = so.tiles[l];
    for (int i = threadIdx.x; i < nt; i += kScatterBlockSamples) hist[i] = 0;
    __syncthreads();
    const int64_t n_s = so.n_s;
    const int64_t s = (int64_t)bx * kScatterBlockSamples + threadIdx.x;
    const bool has = s < n_s;  // a prefix of every wave
    const int64_t gs = so.s_begin + (has ? s : n_s - 1);
    const float* ro = ray_obj + 6 * (gs / S);
    const float ts = t[gs];
    Corners c;
    level_corners(o.grid, l, sample_coord(ts, ro[3], ro[0]), sample_coord(ts, ro[4], ro[1]),
                  sample_coord(ts, ro[5], ro[2]), c);
    const uint32_t heads = run_heads(c, has);
    if (has) {
        const int64_t row0 = (int64_t)l << o.grid.log2_table;  // rows of float2 / half2
        float2 v;
        if (o.table_dtype == PRENOM_F16)
            v = gather_blend_rows(params_f16 + o.param_off / 2 + row0, c);
        else
            v = gather_blend_rows(reinterpret_cast<const float2*>(params + o.param_off) + row0, c);
        y[o.y_off / 2 + (int64_t)l * n_s + s] = v;
    }
    count_records(hist, c, heads, nt);
    __syncthreads();
    uint32_t* out = counts + so.count_off + (int64_t)so.tile_base[l] * so.n_blocks + bx;
    for (int i = threadIdx.x; i < nt; i += kScatterBlockSamples) out[(int64_t)i * so.n_blocks] = hist[i];
}

__global__ __launch_bounds__(kEncBlock) void k_encode_points(GridInfo g, const float2* __restrict__ table,
                                                             const float* __restrict__ pos, int64_t n,
                                                             float2* __restrict__ y,
                                                             int32_t* __restrict__ corner_idx)
{
    const int64_t i = (int64_t)blockIdx.x * kEncBlock + threadIdx.x;
    const int l = blockIdx.y;
    if (i >= n) return;
    const float* p = pos + 3 * i;
    Corners c;
    level_corners(g, l, fminf(fmaxf(p[0], 0.0f), 1.0f), fminf(fmaxf(p[1], 0.0f), 1.0f),
                  fminf(fmaxf(p[2], 0.0f), 1.0f), c);
    const float2* lt = table + ((int64_t)l << g.log2_table);
    y[(int64_t)l * n + i] = gather_blend(lt, g, l, c);
    if (corner_idx) {
        int32_t* ci = corner_idx + ((int64_t)l * n + i) * 8;
#pragma unroll
        for (int e = 0; e < 8; ++e) ci[e] = (int32_t)c.row[e];
    }
}

// Encoding of the R^3 grid vertices (i, j, k) / (R - 1), vertex p = (k R + j) R + i
// (x fastest); each coordinate is rounded from FP64 to FP32, like a sample
// position.  Used to refresh the density prior from the NeRF.
template <typename Row>
__global__ __launch_bounds__(kEncBlock) void k_encode_grid(GridInfo g, const Row* __restrict__ table, int32_t R,
                                                           int64_t p0, int64_t cnt, float2* __restrict__ y)
{
    const int64_t q = (int64_t)blockIdx.x * kEncBlock + threadIdx.x;
    const int l = blockIdx.y;
    if (q >= cnt) return;
    const int64_t p = p0 + q;
    const int64_t i = p % R, j = (p / R) % R, k = p / ((int64_t)R * R);
    const double d = (double)(R - 1);  // correctly rounded FP64 quotients, then FP32
    Corners c;
    level_corners(g, l, (float)((double)i / d), (float)((double)j / d), (float)((double)k / d), c);
    const Row* lt = table + ((int64_t)l << g.log2_table);
    y[(int64_t)l * cnt + q] = gather_blend(lt, g, l, c);
}

// out[p] = sigma of head output p (sc rows are (sigma, r, g, b)).
__global__ __launch_bounds__(256) void k_density_grid(const float4* __restrict__ sc, int64_t n, float* __restrict__ out)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < n) out[p] = sc[p].x;
}

dim3 enc_grid(int64_t n, int L) { return dim3((uint32_t)((n + kEncBlock - 1) / kEncBlock), (uint32_t)L); }

}  // namespace

hipError_t launch_encode_samples(const GridInfo& g, const float* table, const void* table_f16,
                                 const float* ray_obj, const float* t, int64_t n_rays, int32_t S, float* y,
                                 hipStream_t s, const TileHist* hist)
{
    const int64_t n_s = n_rays * S;
    if (n_s == 0) return hipSuccess;
    if (hist) {
        const dim3 grid((uint32_t)((n_s + kScatterBlockSamples - 1) / kScatterBlockSamples), (uint32_t)g.n_levels);
        if (table_f16)
            hipLaunchKernelGGL(k_encode_samples_hist<half2_t>, grid, dim3(kScatterBlockSamples), 0, s, g,
                               (const half2_t*)table_f16, ray_obj, t, n_s, S, (float2*)y, *hist);
        else
            hipLaunchKernelGGL(k_encode_samples_hist<float2>, grid, dim3(kScatterBlockSamples), 0, s, g,
                               (const float2*)table, ray_obj, t, n_s, S, (float2*)y, *hist);
        return hipGetLastError();
    }
    if (table_f16)
        hipLaunchKernelGGL(k_encode_samples<half2_t>, enc_grid(n_s, g.n_levels), dim3(kEncBlock), 0, s, g,
                           (const half2_t*)table_f16, ray_obj, t, n_s, S, (float2*)y);
    else
        hipLaunchKernelGGL(k_encode_samples<float2>, enc_grid(n_s, g.n_levels), dim3(kEncBlock), 0, s, g,
                           (const float2*)table, ray_obj, t, n_s, S, (float2*)y);
    return hipGetLastError();
}

hipError_t launch_encode_grid(const GridInfo& g, const float* table, const void* table_f16, int32_t R, int64_t p0,
                              int64_t cnt, float* y, hipStream_t s)
{
    if (cnt == 0) return hipSuccess;
    if (table_f16)
        hipLaunchKernelGGL(k_encode_grid<half2_t>, enc_grid(cnt, g.n_levels), dim3(kEncBlock), 0, s, g,
                           (const half2_t*)table_f16, R, p0, cnt, (float2*)y);
    else
        hipLaunchKernelGGL(k_encode_grid<float2>, enc_grid(cnt, g.n_levels), dim3(kEncBlock), 0, s, g,
                           (const float2*)table, R, p0, cnt, (float2*)y);
    return hipGetLastError();
}

hipError_t launch_density_grid(const float* sc, int64_t n, float* out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_density_grid, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, (const float4*)sc, n, out);
    return hipGetLastError();
}

hipError_t launch_encode_batch_hist(const ObjDev* objs, const ScatterObj* sobjs, int n_obj, int64_t n_items,
                                    const float* params, const void* params_f16, const float* ray_obj, const float* t,
                                    int32_t S, float* y, uint32_t* counts, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    hipLaunchKernelGGL(k_encode_batch_hist, dim3((uint32_t)n_items), dim3(kScatterBlockSamples), 0, s, objs, sobjs,
                       n_obj, params, (const half2_t*)params_f16, ray_obj, t, S, (float2*)y, counts);
    return hipGetLastError();
}


hipError_t launch_encode_points(const GridInfo& g, const float* table, const float* pos, int64_t n,
                                float* features, int32_t* corner_idx, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_encode_points, enc_grid(n, g.n_levels), dim3(kEncBlock), 0, s, g,
                       (const float2*)table, pos, n, (float2*)features, corner_idx);
    return hipGetLastError();
}

}  // namespace prenom

// Hash-table gradient without global atomics: a bucketed scatter-add.
//
// The backward of the encoding adds w_e * dy to the table row of each of the
// 8 cell corners of every (sample, level).  On gfx950 every global FP32
// atomic costs about the same whatever its scope (a device-wide ceiling near
// 2e10 per second), so at 10^9 contributions per step they cannot be issued
// one by one.  Instead the contributions are bucketed by table tile (2^13 rows,
// whose accumulators fill 128 KB of LDS):
//
//   count  : per (sample block, level) an LDS histogram of contributions per
//            tile -> counts[tile][block], and the block's max |dy|
//   scan   : exclusive prefix over blocks (per tile), then over tiles; the
//            tile record ranges are cut into chunks of bounded length, and each
//            tile gets a fixed-point scale 2^e
//   place  : the block recomputes its contributions, sorts them by tile in LDS
//            and writes each tile's run contiguously (coalesced) as records
//            (row within tile: u16, contribution: float2)
//   reduce : a persistent grid takes chunks from a counter; each chunk is
//            accumulated in LDS and added to the gradient rows -- plain
//            read-modify-write when the tile has one chunk (the block owns it),
//            global atomics only for tiles split over several chunks.
//
// The LDS accumulation is 64-bit fixed point (integer LDS atomics run several
// times faster than FP32 ones).  With e chosen so that max|dy| * records * 2^e
// < 2^62, no sum can overflow and each contribution is rounded by at most
// 2^-(e+1), far below FP32 resolution of the result; integer sums do not
// depend on order, so a tile with one chunk gets a bit-reproducible gradient.
//
// Corner rows and weights are computed by the same function as the forward
// encoding, so count and place agree exactly.
#include "common.h"

namespace prenom {
namespace {

constexpr int kTileBits = 13;
constexpr int kTileRows = 1 << kTileBits;
constexpr int kPlaceThreads = 512;
constexpr int kSamplesPerThread = 1;
constexpr int kSamplesPerBlock = kPlaceThreads * kSamplesPerThread;  // 512
constexpr int kRecordsPerBlock = kSamplesPerBlock * 8;
constexpr int kMaxTilesPerLevel = 1 << (24 - kTileBits);  // T <= 2^24
constexpr int kScanThreads = 1024;
constexpr int kReduceThreads = 1024;
constexpr int kReduceUnroll = 8;  // records in flight per thread
constexpr int64_t kChunk = (int64_t)1 << 21;  // records per reduce work item

// Levels with at most this many tiles have most lanes of a wave in the same
// tile; their histogram atomics are combined per wave first.
constexpr int kAggregateTiles = 16;

// Adds 1 to hist[tile] for every active lane and returns the lane's rank
// among the additions to that tile.  Lanes of the wave that share a tile are
// combined into one LDS atomic issued by their first lane (same-address
// atomics of one instruction would otherwise serialise).
__device__ __forceinline__ uint32_t wave_aggregated_add(uint32_t* hist, uint32_t tile)
{
    const int lane = threadIdx.x & 63;
    const uint64_t lane_lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint64_t remaining = __ballot(1);
    uint32_t rank = 0;
    while (remaining) {
        const int leader = __ffsll((unsigned long long)remaining) - 1;
        const uint32_t lt = __shfl(tile, leader);
        const uint64_t mask = __ballot(tile == lt);
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&hist[lt], (uint32_t)__popcll(mask));
        base = __shfl(base, leader);
        if (tile == lt) rank = base + (uint32_t)__popcll(mask & lane_lt);
        remaining &= ~mask;
    }
    return rank;
}

// Feature gradient and corners of one (sample, level); false when dy == 0
// (the sample contributes nothing and is skipped by count and place alike).
__device__ __forceinline__ bool load_contrib(const ScatterArgs& a, int l, int64_t s, float2& d, Corners& c)
{
    d = a.dy[(int64_t)l * a.n_s + s];
    if (d.x == 0.0f && d.y == 0.0f) return false;
    const float* ro = a.ray_obj + 6 * (s / a.S);
    const float ts = a.t[s];
    level_corners(a.grid, l, sample_coord(ts, ro[3], ro[0]), sample_coord(ts, ro[4], ro[1]),
               sample_coord(ts, ro[5], ro[2]), c);
    return true;
}

__global__ __launch_bounds__(kPlaceThreads) void k_scatter_count(ScatterArgs a)
{
    __shared__ uint32_t hist[kMaxTilesPerLevel];
    __shared__ float wmax[kPlaceThreads / 64];
    const int l = blockIdx.y, bx = blockIdx.x;
    const int nt = a.tiles[l];
    for (int i = threadIdx.x; i < nt; i += kPlaceThreads) hist[i] = 0;
    __syncthreads();
    float m = 0.0f;
    for (int k = 0; k < kSamplesPerThread; ++k) {
        const int64_t s = (int64_t)bx * kSamplesPerBlock + k * kPlaceThreads + threadIdx.x;
        if (s >= a.n_s) break;
        float2 d;
        Corners c;
        if (!load_contrib(a, l, s, d, c)) continue;
        m = fmaxf(m, fmaxf(fabsf(d.x), fabsf(d.y)));
        if (nt <= kAggregateTiles) {
#pragma unroll
            for (int e = 0; e < 8; ++e) wave_aggregated_add(hist, c.row[e] >> kTileBits);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) atomicAdd(&hist[c.row[e] >> kTileBits], 1u);
        }
    }
#pragma unroll
    for (int dd = 32; dd >= 1; dd >>= 1) m = fmaxf(m, __shfl_xor(m, dd));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    uint32_t* out = a.counts + (int64_t)a.tile_base[l] * a.n_blocks + bx;
    for (int i = threadIdx.x; i < nt; i += kPlaceThreads) out[(int64_t)i * a.n_blocks] = hist[i];
    if (threadIdx.x == 0) {
        float bm = 0.0f;
        for (int w = 0; w < kPlaceThreads / 64; ++w) bm = fmaxf(bm, wmax[w]);
        a.block_max[(int64_t)l * a.n_blocks + bx] = bm;
    }
}

// Per tile: exclusive prefix of the per-block counts (in place) and the total.
__global__ __launch_bounds__(kScanThreads) void k_scatter_scan_blocks(ScatterArgs a)
{
    __shared__ uint64_t part[kScanThreads];
    const int tile = blockIdx.x;
    uint32_t* row = a.counts + (int64_t)tile * a.n_blocks;
    const int per = (a.n_blocks + kScanThreads - 1) / kScanThreads;
    const int b0 = threadIdx.x * per, b1 = min(b0 + per, a.n_blocks);
    uint64_t sum = 0;
    for (int b = b0; b < b1; ++b) sum += row[b];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {  // inclusive Hillis-Steele scan
        const uint64_t v = threadIdx.x >= d ? part[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint64_t run = part[threadIdx.x] - sum;
    for (int b = b0; b < b1; ++b) {
        const uint32_t c = row[b];
        row[b] = (uint32_t)run;  // offsets within a tile fit 32 bits
        run += c;
    }
    if (threadIdx.x == kScanThreads - 1) a.tile_total[tile] = part[kScanThreads - 1];
}

// Over tiles: record bases, chunk counts and chunk bases, the fixed-point
// exponent of each tile; resets the work counter.
__global__ __launch_bounds__(kScanThreads) void k_scatter_scan_tiles(ScatterArgs a)
{
    __shared__ uint64_t prec[kScanThreads], pchk[kScanThreads];
    __shared__ float lmax[PRENOM_MAX_LEVELS];
    // per-level max |dy| over the blocks
    for (int l = threadIdx.x >> 6; l < a.grid.n_levels; l += kScanThreads / 64) {
        float m = 0.0f;
        for (int b = threadIdx.x & 63; b < a.n_blocks; b += 64) m = fmaxf(m, a.block_max[(int64_t)l * a.n_blocks + b]);
#pragma unroll
        for (int dd = 32; dd >= 1; dd >>= 1) m = fmaxf(m, __shfl_xor(m, dd));
        if ((threadIdx.x & 63) == 0) lmax[l] = m;
    }
    __syncthreads();
    const int n = a.n_tiles;
    const int per = (n + kScanThreads - 1) / kScanThreads;
    const int t0 = threadIdx.x * per, t1 = min(t0 + per, n);
    uint64_t rs = 0, cs = 0;
    for (int t = t0; t < t1; ++t) {
        rs += a.tile_total[t];
        cs += (a.tile_total[t] + kChunk - 1) / kChunk;
    }
    prec[threadIdx.x] = rs;
    pchk[threadIdx.x] = cs;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        const uint64_t v = threadIdx.x >= d ? prec[threadIdx.x - d] : 0;
        const uint64_t w = threadIdx.x >= d ? pchk[threadIdx.x - d] : 0;
        __syncthreads();
        prec[threadIdx.x] += v;
        pchk[threadIdx.x] += w;
        __syncthreads();
    }
    uint64_t r = prec[threadIdx.x] - rs, ck = pchk[threadIdx.x] - cs;
    for (int t = t0; t < t1; ++t) {
        a.tile_start[t] = r;
        a.chunk_start[t] = ck;
        r += a.tile_total[t];
        ck += (a.tile_total[t] + kChunk - 1) / kChunk;
        // largest e with max|dy| * records * 2^e < 2^62 (bound on any row's |sum| * 2^e)
        int l = 0;
        while (l + 1 < a.grid.n_levels && a.tile_base[l + 1] <= t) ++l;
        const double bound = (double)lmax[l] * (double)a.tile_total[t];
        int e = 0;
        if (bound > 0.0) {
            int ex;
            frexp(bound, &ex);  // bound < 2^ex
            e = 62 - ex;
        }
        a.tile_exp[t] = e;
    }
    if (threadIdx.x == kScanThreads - 1) {
        a.tile_start[n] = prec[kScanThreads - 1];
        a.chunk_start[n] = pchk[kScanThreads - 1];
        *a.work_counter = 0;
    }
}

// Dynamic LDS of the place kernel for nt tiles of one level.
__host__ __device__ constexpr size_t place_lds_bytes(int nt)
{
    return (size_t)nt * 8 + (size_t)kRecordsPerBlock * 8 + (size_t)nt * 8 + 16 + (size_t)kRecordsPerBlock * 4;
}

__global__ __launch_bounds__(kPlaceThreads) void k_scatter_place(ScatterArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int nt_lds = a.tiles_max;
    uint64_t* gbase = reinterpret_cast<uint64_t*>(smem);
    float2* s_val = reinterpret_cast<float2*>(gbase + nt_lds);
    uint32_t* hist = reinterpret_cast<uint32_t*>(s_val + kRecordsPerBlock);
    uint32_t* seg = hist + nt_lds;
    uint32_t* p_total = seg + nt_lds;
    uint16_t* s_key = reinterpret_cast<uint16_t*>(p_total + 4);
    uint16_t* s_tile = s_key + kRecordsPerBlock;
    const int l = blockIdx.y, bx = blockIdx.x;
    const int nt = a.tiles[l];
    for (int i = threadIdx.x; i < nt; i += kPlaceThreads) hist[i] = 0;
    __syncthreads();
    // pass 1: rank of each contribution within its tile (LDS atomics)
    uint32_t rank[kSamplesPerThread][8];
    for (int k = 0; k < kSamplesPerThread; ++k) {
        const int64_t s = (int64_t)bx * kSamplesPerBlock + k * kPlaceThreads + threadIdx.x;
        float2 d;
        Corners c;
        if (s >= a.n_s || !load_contrib(a, l, s, d, c)) continue;
        if (nt <= kAggregateTiles) {
#pragma unroll
            for (int e = 0; e < 8; ++e) rank[k][e] = wave_aggregated_add(hist, c.row[e] >> kTileBits);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) rank[k][e] = atomicAdd(&hist[c.row[e] >> kTileBits], 1u);
        }
    }
    __syncthreads();
    // block-local segments: exclusive scan of hist (serial over <= 1024 tiles by one wave)
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        uint32_t carry = 0;
        for (int base = 0; base < nt; base += 64) {
            const int i = base + lane;
            uint32_t v = i < nt ? hist[i] : 0u, incl = v;
#pragma unroll
            for (int dd = 1; dd < 64; dd <<= 1) {
                const uint32_t o = __shfl_up(incl, dd);
                if (lane >= dd) incl += o;
            }
            if (i < nt) seg[i] = carry + incl - v;
            carry += __shfl(incl, 63);
        }
        if (lane == 0) *p_total = carry;
    }
    __syncthreads();
    // global position of record p of tile tt: gbase[tt] + p
    {
        const int tb = a.tile_base[l];
        for (int i = threadIdx.x; i < nt; i += kPlaceThreads)
            gbase[i] = a.tile_start[tb + i] + a.counts[(int64_t)(tb + i) * a.n_blocks + bx] - seg[i];
    }
    // pass 2: recompute and stage the records sorted by tile
    for (int k = 0; k < kSamplesPerThread; ++k) {
        const int64_t s = (int64_t)bx * kSamplesPerBlock + k * kPlaceThreads + threadIdx.x;
        float2 d;
        Corners c;
        if (s >= a.n_s || !load_contrib(a, l, s, d, c)) continue;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint32_t tt = c.row[e] >> kTileBits;
            const uint32_t p = seg[tt] + rank[k][e];
            s_key[p] = (uint16_t)(c.row[e] & (kTileRows - 1));
            s_tile[p] = (uint16_t)tt;
            s_val[p] = make_float2(c.w[e] * d.x, c.w[e] * d.y);
        }
    }
    __syncthreads();
    // write each tile's run to its global range: consecutive threads, consecutive records
    const uint32_t total = *p_total;
    for (uint32_t p = threadIdx.x; p < total; p += kPlaceThreads) {
        const uint64_t dst = gbase[s_tile[p]] + p;
        a.keys[dst] = s_key[p];
        a.vals[dst] = s_val[p];
    }
}

__global__ __launch_bounds__(kReduceThreads) void k_scatter_reduce(ScatterArgs a)
{
    __shared__ unsigned long long acc[2 * kTileRows];  // fixed point: feature 0 rows, then feature 1 rows
    __shared__ int64_t s_chunk;
    const uint64_t n_chunks = a.chunk_start[a.n_tiles];
    for (;;) {
        if (threadIdx.x == 0) s_chunk = (int64_t)atomicAdd(a.work_counter, 1ull);
        __syncthreads();
        const int64_t chunk = s_chunk;
        __syncthreads();
        if ((uint64_t)chunk >= n_chunks) break;
        // tile of this chunk: last t with chunk_start[t] <= chunk
        int lo = 0, hi = a.n_tiles - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.chunk_start[mid] <= (uint64_t)chunk)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int tile = lo;
        int l = 0;
        while (l + 1 < a.grid.n_levels && a.tile_base[l + 1] <= tile) ++l;
        const int tt = tile - a.tile_base[l];
        const int64_t row0 = (int64_t)tt << kTileBits;
        const int n_rows = (int)min((int64_t)kTileRows, a.level_rows[l] - row0);
        const uint64_t k0 = chunk - a.chunk_start[tile];
        const uint64_t r_begin = a.tile_start[tile] + k0 * kChunk;
        const uint64_t r_end = min(r_begin + (uint64_t)kChunk, a.tile_start[tile + 1]);
        const bool owner = (a.chunk_start[tile + 1] - a.chunk_start[tile]) == 1;
        const int ex = a.tile_exp[tile];
        for (int i = threadIdx.x; i < n_rows; i += kReduceThreads) {
            acc[i] = 0ull;
            acc[kTileRows + i] = 0ull;
        }
        __syncthreads();
        // kReduceUnroll independent, coalesced record loads in flight per thread
        for (uint64_t r0 = r_begin; r0 < r_end; r0 += (uint64_t)kReduceThreads * kReduceUnroll) {
            uint32_t key[kReduceUnroll];
            float2 v[kReduceUnroll];
#pragma unroll
            for (int u = 0; u < kReduceUnroll; ++u) {
                const uint64_t r = r0 + (uint64_t)u * kReduceThreads + threadIdx.x;
                const bool ok = r < r_end;
                key[u] = ok ? a.keys[r] : 0u;
                v[u] = ok ? a.vals[r] : make_float2(0.0f, 0.0f);
            }
#pragma unroll
            for (int u = 0; u < kReduceUnroll; ++u) {
                const long long qx = (long long)rintf(ldexpf(v[u].x, ex));
                const long long qy = (long long)rintf(ldexpf(v[u].y, ex));
                if (qx != 0) atomicAdd(&acc[key[u]], (unsigned long long)qx);
                if (qy != 0) atomicAdd(&acc[kTileRows + key[u]], (unsigned long long)qy);
            }
        }
        __syncthreads();
        float2* g = reinterpret_cast<float2*>(a.g_table) + ((int64_t)l << a.grid.log2_table) + row0;
        for (int i = threadIdx.x; i < n_rows; i += kReduceThreads) {
            const long long sx = (long long)acc[i], sy = (long long)acc[kTileRows + i];
            if (sx == 0 && sy == 0) continue;
            const float2 v = make_float2((float)ldexp((double)sx, -ex), (float)ldexp((double)sy, -ex));
            if (owner) {
                float2 o = g[i];
                o.x += v.x;
                o.y += v.y;
                g[i] = o;
            } else {
                atomicAdd(&g[i].x, v.x);
                atomicAdd(&g[i].y, v.y);
            }
        }
        __syncthreads();
    }
}

}  // namespace

ScatterPlan scatter_plan(const GridInfo& g, int64_t n_s)
{
    ScatterPlan p{};
    p.n_blocks = (int)((n_s + kSamplesPerBlock - 1) / kSamplesPerBlock);
    p.n_tiles = 0;
    const int64_t T = (int64_t)1 << g.log2_table;
    for (int l = 0; l < g.n_levels; ++l) {
        const int64_t side = (int64_t)g.res[l] + 1;
        const int64_t rows = ((g.dense_mask >> l) & 1u) ? side * side * side : T;
        p.level_rows[l] = rows;
        p.tiles[l] = (int)((rows + kTileRows - 1) / kTileRows);
        p.tile_base[l] = p.n_tiles;
        p.n_tiles += p.tiles[l];
    }
    p.max_records = n_s * g.n_levels * 8;
    return p;
}

int scatter_max_tiles_per_level() { return kMaxTilesPerLevel; }

hipError_t launch_scatter(const ScatterArgs& a, hipStream_t s)
{
    if (a.n_s == 0) return hipSuccess;
    const dim3 grid((uint32_t)a.n_blocks, (uint32_t)a.grid.n_levels);
    hipLaunchKernelGGL(k_scatter_count, grid, dim3(kPlaceThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scatter_scan_blocks, dim3((uint32_t)a.n_tiles), dim3(kScanThreads), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_scatter_scan_tiles, dim3(1), dim3(kScanThreads), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const size_t place_lds = place_lds_bytes(a.tiles_max);
    if (place_lds > 65536 &&
        (e = hipFuncSetAttribute((const void*)k_scatter_place, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)place_lds)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_scatter_place, grid, dim3(kPlaceThreads), place_lds, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_scatter_reduce, dim3((uint32_t)a.reduce_blocks), dim3(kReduceThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace prenom

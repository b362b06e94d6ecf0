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
//            tile -> counts[tile][block], and the block's max |dy|.  In the
//            single-object training step the forward encoding has written
//            the histograms already (it computes the same corners), so this
//            phase only takes the block maxima of |dy| (k_scatter_dymax)
//   scan   : exclusive prefix over blocks (per tile), then over tiles; the
//            tile record ranges are cut into chunks of bounded length, and each
//            tile gets a fixed-point scale 2^e
//   place  : the block recomputes its contributions, sorts them by tile in LDS
//            and writes each tile's run contiguously (coalesced) as 8-byte
//            records (row within the tile, and the contribution's two
//            features as 22-bit mantissas under one shared exponent)
//   reduce : a persistent grid takes chunks from a counter; each chunk is
//            accumulated in LDS and added to the gradient rows -- plain
//            read-modify-write when the tile has one chunk (the block owns it),
//            global atomics only for tiles split over several chunks.
//
// The LDS accumulation is 64-bit fixed point (integer LDS atomics run several
// times faster than FP32 ones).  With e chosen so that max|dy| * records * 2^e
// < 2^62, no sum can overflow; with max|dy| * 2^e < 2^50 as well, each
// contribution is rounded by at most 2^-(e+1) <= 2^-51 max|dy|, far below FP32
// resolution of the result.  Integer sums do not depend on order, so a tile
// with one chunk gets a bit-reproducible gradient.
//
// A record keeps 21 significant bits of the larger of its two features (an
// FP32 value has 24): each feature is within 2^-21 of the larger one's
// magnitude; the sum over records is then exact up to the fixed-point
// rounding.
//
// Corner rows and weights are computed by the same function as the forward
// encoding, so count and place agree exactly.
//
// The same kernels serve one object (its geometry passed by value) and a
// batch of objects with different grids (geometry in a device table): tiles,
// sample blocks and (object, level) pairs of all objects are numbered
// consecutively, so every phase is one launch for the whole batch.
#include "common.h"

namespace prenom {
namespace {

constexpr int kPlaceThreads = kScatterBlockSamples;
constexpr int kSamplesPerBlock = kPlaceThreads;  // one sample per thread
constexpr int kRecordsPerBlock = kSamplesPerBlock * 8;
constexpr int kScanThreads = 1024;
constexpr int kReduceThreads = 1024;
constexpr int kRun = 8;            // consecutive records per thread and load
constexpr int kRunsPerThread = 3;  // runs in flight per thread
// Records per reduce work item: a power of two between 2^chunk_min_bits and
// 2^kChunkMaxBits, the smallest that gives at most kChunksPerBlock items per
// reduce block (few large items leave blocks idle at the end of a pass; each
// item also zeroes and writes out its whole tile).
constexpr int kChunkMinBits = 18, kChunkMaxBits = 21;
constexpr uint64_t kChunksPerBlock = 4;

// ---------------------------------------------------------------- records
// A record holds the row within the tile (bits 0-12), an exponent offset r
// (EB bits) and the two's-complement mantissas qx, qy (MB bits each); its
// value is (qx, qy) * 2^(E - r - (MB - 1)), E being the level's record
// exponent, and a record whose larger feature lies below 2^(E - 2^EB - 1) (r
// beyond EB bits) is dropped.  Two formats:
//   full:    EB = 7, MB = 22, one 64-bit word (21 significant bits);
//   compact: EB = 5, MB = 15, 48 bits kept as a 32-bit word (bits 0-31) in
//            one array and a 16-bit word (bits 32-47) in another (14
//            significant bits), for FP16 tables.
constexpr int kRecExpBits = 7;
constexpr int kRecMantBits = 22;
constexpr int kRecExpBitsC = 5;
constexpr int kRecMantBitsC = 15;

// Record exponent E of a level whose largest |dy| is lm: a record sums at most
// 8 contributions w dy with 0 <= w <= 1, so |record| <= 8 lm < 2^(E - 1).
__device__ __forceinline__ int level_rec_exp(float lm)
{
    int e = 0;
    frexpf(lm, &e);  // lm < 2^e
    return e + 4;
}

template <int EB, int MB>
__device__ __forceinline__ uint64_t encode_record(float2 v, int E, uint32_t row)
{
    const float m = fmaxf(fabsf(v.x), fabsf(v.y));
    uint64_t rec = row;
    if (m > 0.0f) {
        int k = 0;
        frexpf(m, &k);  // 2^(k-1) <= m < 2^k
        // the larger one can round up to 2^(MB-1), one past the field: it is
        // held at 2^(MB-1) - 1 (an error of one unit in its last place)
        constexpr float kMax = (float)((1u << (MB - 1)) - 1u);
        const float rx = fminf(fmaxf(rintf(ldexpf(v.x, MB - 1 - k)), -kMax), kMax);
        const float ry = fminf(fmaxf(rintf(ldexpf(v.y, MB - 1 - k)), -kMax), kMax);
        const int r = E - k;
        constexpr uint32_t kMant = (1u << MB) - 1u;
        if (r >= 0 && r < (1 << EB))
            rec |= (uint64_t)r << kTileBits | (uint64_t)((uint32_t)(int32_t)rx & kMant) << (kTileBits + EB) |
                   (uint64_t)((uint32_t)(int32_t)ry & kMant) << (kTileBits + EB + MB);
    }
    return rec;
}

// Fields of record word w (format EB, MB): row key, exponent offset, mantissas.
template <int EB, int MB>
__device__ __forceinline__ void decode_record(uint64_t w, uint32_t& key, int& r, long long& qx, long long& qy)
{
    key = (uint32_t)w & (kTileRows - 1);
    r = (int)((w >> kTileBits) & ((1u << EB) - 1u));
    qx = (long long)(w << (64 - kTileBits - EB - MB)) >> (64 - MB);
    qy = (long long)(w << (64 - kTileBits - EB - 2 * MB)) >> (64 - MB);
}

// q * 2^sh rounded to an integer (halves upward), for |q| <= 2^21, sh <= 37.
__device__ __forceinline__ long long scale_mantissa(long long q, int sh)
{
    if (sh >= 0) return q * (1ll << min(sh, 40));  // (the clamp only matters for non-finite gradients)
    const int d = -sh;
    return d > 62 ? 0ll : (q + (1ll << (d - 1))) >> d;
}
static_assert(kTileBits + kRecExpBitsC + 2 * kRecMantBitsC == 48, "compact record fields fill 48 bits");
static_assert(kTileBits + kRecExpBits + 2 * kRecMantBits == 64, "record fields fill one word");


// ---------------------------------------------------------------- object lookup
// Index of the last object whose `field` is <= v (fields ascend with the index).
template <bool kMany, typename F>
__device__ __forceinline__ int last_le(const ScatterArgs& a, int64_t v, F field)
{
    if constexpr (!kMany) {
        return 0;
    } else {
        int lo = 0, hi = a.n_obj - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (field(a.objs[mid]) <= v)
                lo = mid;
            else
                hi = mid - 1;
        }
        return lo;
    }
}

template <bool kMany>
__device__ __forceinline__ const ScatterObj& sobj(const ScatterArgs& a, int i)
{
    if constexpr (kMany)
        return a.objs[i];
    else
        return a.one;
}

template <bool kMany>
__device__ __forceinline__ int obj_of_item(const ScatterArgs& a, int64_t item)
{
    return last_le<kMany>(a, item, [](const ScatterObj& o) { return o.item_off; });
}

template <bool kMany>
__device__ __forceinline__ int obj_of_tile(const ScatterArgs& a, int64_t tile)
{
    return last_le<kMany>(a, tile, [](const ScatterObj& o) { return o.tile_off; });
}

template <bool kMany>
__device__ __forceinline__ int obj_of_level(const ScatterArgs& a, int64_t pair)
{
    return last_le<kMany>(a, pair, [](const ScatterObj& o) { return (int64_t)o.lev_off; });
}

// Level of local tile lt of object o.
__device__ __forceinline__ int level_of_tile(const ScatterObj& o, int lt)
{
    int l = 0;
    while (l + 1 < o.grid.n_levels && o.tile_base[l + 1] <= lt) ++l;
    return l;
}

// Ray of global sample gs (S samples per ray); 32-bit division when it fits.
__device__ __forceinline__ int64_t ray_of_sample(int64_t gs, int S)
{
    return gs < ((int64_t)1 << 32) ? (int64_t)((uint32_t)gs / (uint32_t)S) : gs / S;
}

// Feature gradient and corners of local sample s on level l of object o;
// false when dy == 0 (the sample contributes nothing and is skipped by count
// and place alike).  The gradient, t and the ray are loaded together and the
// corners computed whatever dy is, so the loads are not serialised behind the
// test.
__device__ __forceinline__ bool load_contrib(const ScatterArgs& a, const ScatterObj& o, int l, int64_t s, float2& d,
                                             Corners& c)
{
    const int64_t gs = o.s_begin + s;
    const float* ro = a.ray_obj + 6 * ray_of_sample(gs, a.S);
    d = a.dy[o.dy_off + (int64_t)l * o.n_s + s];
    const float ts = a.t[gs];
    level_corners(o.grid, l, sample_coord(ts, ro[3], ro[0]), sample_coord(ts, ro[4], ro[1]),
                  sample_coord(ts, ro[5], ro[2]), c);
    return d.x != 0.0f || d.y != 0.0f;
}

// Level and sample block of count/place item `rem` of an object (fits 32 bits).
__device__ __forceinline__ void split_item(int64_t rem, int n_blocks, int& l, int& bx)
{
    const uint32_t r = (uint32_t)rem;
    l = (int)(r / (uint32_t)n_blocks);
    bx = (int)(r - (uint32_t)l * (uint32_t)n_blocks);
}

template <bool kMany>
__global__ __launch_bounds__(kPlaceThreads) void k_scatter_count(ScatterArgs a)
{
    __shared__ uint32_t hist[kMaxTilesPerLevel];
    __shared__ float wmax[kPlaceThreads / 64];
    const int64_t item = blockIdx.x;
    const ScatterObj& o = sobj<kMany>(a, obj_of_item<kMany>(a, item));
    int l, bx;
    split_item(item - o.item_off, o.n_blocks, l, bx);
    const int nt = o.tiles[l];
    for (int i = threadIdx.x; i < nt; i += kPlaceThreads) hist[i] = 0;
    __syncthreads();
    float m = 0.0f;
    const int64_t s = (int64_t)bx * kSamplesPerBlock + threadIdx.x;
    float2 d;
    Corners c{};  // lanes past the samples take part in the wave's count with no records
    bool has;
    uint32_t heads = 0xffu;
    if (a.merge_runs) {  // every sample, runs of a repeated corner as one record
        has = s < o.n_s;
        load_contrib(a, o, l, has ? s : o.n_s - 1, d, c);
        heads = run_heads(c, has);
    } else {
        has = s < o.n_s && load_contrib(a, o, l, s, d, c);
    }
    if (a.nonfinite && s < o.n_s && !(isfinite(d.x) && isfinite(d.y))) a.nonfinite[0] = 1;
    if (has) m = fmaxf(fabsf(d.x), fabsf(d.y));
    count_records(hist, c, has ? heads : 0u, nt);
#pragma unroll
    for (int dd = 32; dd >= 1; dd >>= 1) m = fmaxf(m, __shfl_xor(m, dd));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    uint32_t* out = a.counts + o.count_off + (int64_t)o.tile_base[l] * o.n_blocks + bx;
    for (int i = threadIdx.x; i < nt; i += kPlaceThreads) out[(int64_t)i * o.n_blocks] = hist[i];
    if (threadIdx.x == 0) {
        float bm = 0.0f;
        for (int w = 0; w < kPlaceThreads / 64; ++w) bm = fmaxf(bm, wmax[w]);
        a.block_max[o.bmax_off + (int64_t)l * o.n_blocks + bx] = bm;
    }
}

// Max |dy| of each (object, level) over its sample blocks; one block per pair.
// With fwd_counts the histograms exist already: per (level, sample block)
// only the max |dy| that fixes the fixed-point scale.  A workgroup takes
// kDymaxItems consecutive items (consecutive blocks of one level lie next to
// each other in dy), with all their loads in flight at once.
constexpr int kDymaxItems = 8;

template <bool kMany>
__global__ __launch_bounds__(kPlaceThreads) void k_scatter_dymax(ScatterArgs a)
{
    constexpr int kRows = kPlaceThreads / 16;  // 16-lane DPP rows per workgroup
    __shared__ float wmax[kDymaxItems][kRows];
    float m[kDymaxItems];
    bool bad = false;
    // object of the first item by search; the next items follow it (consecutive
    // items belong to the same object or to the ones after it)
    const int64_t item0 = (int64_t)blockIdx.x * kDymaxItems;
    int oi = obj_of_item<kMany>(a, item0 < a.n_items ? item0 : a.n_items - 1);
#pragma unroll
    for (int j = 0; j < kDymaxItems; ++j) {
        const int64_t item = item0 + j;
        m[j] = 0.0f;
        if (item < a.n_items) {
            if constexpr (kMany)
                while (oi + 1 < a.n_obj && a.objs[oi + 1].item_off <= item) ++oi;
            const ScatterObj& o = sobj<kMany>(a, oi);
            int l, bx;
            split_item(item - o.item_off, o.n_blocks, l, bx);
            const int64_t s = (int64_t)bx * kSamplesPerBlock + threadIdx.x;
            if (s < o.n_s) {
                const float2 d = a.dy[o.dy_off + (int64_t)l * o.n_s + s];
                m[j] = fmaxf(fabsf(d.x), fabsf(d.y));
                bad |= !(isfinite(d.x) && isfinite(d.y));
            }
        }
    }
    // a non-finite feature gradient (fmaxf would drop a NaN) marks the step
    // for the loss scaler, which then skips the update
    if (a.nonfinite && bad) a.nonfinite[0] = 1;
    // Row maxima by DPP row shifts: lanes past the row's end read 0, the
    // identity of a maximum of |dy| values; the row's first lane ends with it.
#pragma unroll
    for (int j = 0; j < kDymaxItems; ++j) {
        m[j] = fmaxf(m[j], dpp_f32<0x101>(m[j]));
        m[j] = fmaxf(m[j], dpp_f32<0x102>(m[j]));
        m[j] = fmaxf(m[j], dpp_f32<0x104>(m[j]));
        m[j] = fmaxf(m[j], dpp_f32<0x108>(m[j]));
        if ((threadIdx.x & 15) == 0) wmax[j][threadIdx.x >> 4] = m[j];
    }
    __syncthreads();
    if (threadIdx.x < kDymaxItems) {
        const int64_t item = item0 + threadIdx.x;
        if (item < a.n_items) {
            const ScatterObj& o = sobj<kMany>(a, obj_of_item<kMany>(a, item));
            int l, bx;
            split_item(item - o.item_off, o.n_blocks, l, bx);
            float bm = 0.0f;
            for (int w = 0; w < kRows; ++w) bm = fmaxf(bm, wmax[threadIdx.x][w]);
            a.block_max[o.bmax_off + (int64_t)l * o.n_blocks + bx] = bm;
        }
    }
}

// One workgroup per (object, level) of the pass; a pass has few of them, so
// each takes 16 waves (a maximum does not depend on the order).
constexpr int kLevelMaxThreads = 1024;
template <bool kMany>
__global__ __launch_bounds__(kLevelMaxThreads) void k_scatter_level_max(ScatterArgs a)
{
    __shared__ float red[kLevelMaxThreads / 64];
    const int pair = blockIdx.x;
    const ScatterObj& o = sobj<kMany>(a, obj_of_level<kMany>(a, pair));
    const int l = pair - o.lev_off;
    const float* bm = a.block_max + o.bmax_off + (int64_t)l * o.n_blocks;
    float m = 0.0f;
    for (int b = threadIdx.x; b < o.n_blocks; b += kLevelMaxThreads) m = fmaxf(m, bm[b]);
#pragma unroll
    for (int dd = 32; dd >= 1; dd >>= 1) m = fmaxf(m, __shfl_xor(m, dd));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float r = 0.0f;
        for (int w = 0; w < kLevelMaxThreads / 64; ++w) r = fmaxf(r, red[w]);
        a.level_max[pair] = r;
    }
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t up = __shfl_up(v, d);
        if (lane >= d) v += up;
    }
    return v;
}

// Per tile: exclusive prefix of the per-block counts (into offsets, so the
// forward's histograms survive for another backward) and the total.
// Thread t owns a contiguous run of blocks; the runs' sums are scanned within
// each wave, then across the block's waves.
template <bool kMany>
__global__ __launch_bounds__(kScanThreads) void k_scatter_scan_blocks(ScatterArgs a)
{
    constexpr int kWaves = kScanThreads / 64;
    __shared__ uint64_t wave_tot[kWaves];
    const int64_t tile = blockIdx.x;
    const ScatterObj& o = sobj<kMany>(a, obj_of_tile<kMany>(a, tile));
    const int nb = o.n_blocks;
    const int64_t row0 = o.count_off + (tile - o.tile_off) * nb;
    const uint32_t* row = a.counts + row0;
    uint32_t* orow = a.offsets + row0;
    const int per = (nb + kScanThreads - 1) / kScanThreads;
    const int b0 = min((int)threadIdx.x * per, nb), b1 = min(b0 + per, nb);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t sum = 0;
    for (int b = b0; b < b1; ++b) sum += row[b];
    const uint64_t incl = wave_incl_scan(sum, lane);
    if (lane == 63) wave_tot[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        const uint64_t t = lane < kWaves ? wave_tot[lane] : 0;
        const uint64_t ti = wave_incl_scan(t, lane);
        if (lane < kWaves) wave_tot[lane] = ti - t;  // exclusive over waves
        if (lane == kWaves - 1) a.tile_total[tile] = ti;
    }
    __syncthreads();
    uint64_t run = wave_tot[wave] + incl - sum;
    for (int b = b0; b < b1; ++b) {
        orow[b] = (uint32_t)run;  // offsets within a tile fit 32 bits
        run += row[b];
    }
}

// Over all tiles: record bases, chunk counts and chunk bases, the fixed-point
// exponent of each tile; resets the work counter.
template <bool kMany>
__global__ __launch_bounds__(kScanThreads) void k_scatter_scan_tiles(ScatterArgs a)
{
    __shared__ uint64_t prec[kScanThreads], pchk[kScanThreads];
    const int64_t n = a.n_tiles;
    const int64_t per = (n + kScanThreads - 1) / kScanThreads;
    const int64_t t0 = threadIdx.x * per, t1 = min(t0 + per, n);
    uint64_t rs = 0, cs = 0;
    for (int64_t t = t0; t < t1; ++t) rs += a.tile_total[t];
    prec[threadIdx.x] = rs;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        const uint64_t v = threadIdx.x >= d ? prec[threadIdx.x - d] : 0;
        __syncthreads();
        prec[threadIdx.x] += v;
        __syncthreads();
    }
    // chunk size from the pass's record total
    const uint64_t per_item = prec[kScanThreads - 1] / ((uint64_t)a.reduce_blocks * kChunksPerBlock);
    int cb = min(max(a.chunk_min_bits, kChunkMinBits), kChunkMaxBits);
    while (cb < kChunkMaxBits && ((uint64_t)1 << cb) < per_item) ++cb;
    const uint64_t chunk = (uint64_t)1 << cb;
    for (int64_t t = t0; t < t1; ++t) cs += (a.tile_total[t] + chunk - 1) >> cb;
    pchk[threadIdx.x] = cs;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        const uint64_t w = threadIdx.x >= d ? pchk[threadIdx.x - d] : 0;
        __syncthreads();
        pchk[threadIdx.x] += w;
        __syncthreads();
    }
    uint64_t r = prec[threadIdx.x] - rs, ck = pchk[threadIdx.x] - cs;
    for (int64_t t = t0; t < t1; ++t) {
        a.tile_start[t] = r;
        a.chunk_start[t] = ck;
        r += a.tile_total[t];
        ck += (a.tile_total[t] + chunk - 1) >> cb;
        // largest e with vmax * records * 2^e < 2^62 (bound on any row's
        // |sum| * 2^e) and vmax * 2^e < 2^50 (bound on one record's fixed-point
        // value, so a record's mantissa is shifted by at most 33 bits), vmax
        // the largest record: max|dy|, or 8 max|dy| when repeated corners are
        // merged
        const ScatterObj& o = sobj<kMany>(a, obj_of_tile<kMany>(a, t));
        const int l = level_of_tile(o, (int)(t - o.tile_off));
        // (a merged record sums at most 8 contributions, one per lane of a group)
        const double vmax = (double)a.level_max[o.lev_off + l] * (a.merge_runs ? 8.0 : 1.0);
        const double bound = vmax * (double)a.tile_total[t];
        int e = 0;
        if (bound > 0.0) {
            int ex, evx;
            frexp(bound, &ex);  // bound < 2^ex
            frexp(vmax, &evx);  // vmax < 2^evx
            e = min(62 - ex, 50 - evx);
        }
        a.tile_exp[t] = e;
    }
    if (threadIdx.x == kScanThreads - 1) {
        // Histograms from the forward cannot hold more records than there
        // are corners of samples; if they do (a backward whose workspace
        // holds no forward of these rays), no chunk is handed out and place
        // stops at once.
        const bool ok = !a.fwd_counts || prec[kScanThreads - 1] <= (uint64_t)a.n_records;
        a.tile_start[n] = ok ? prec[kScanThreads - 1] : ~0ull;
        a.chunk_start[n] = ok ? pchk[kScanThreads - 1] : 0ull;
        a.chunk_start[n + 1] = (uint64_t)cb;
        *a.work_counter = 0;
    }
}

// Dynamic LDS of the place kernel for nt tiles of one level, with staged tile
// ids of tile_bytes bytes: record bases, staged records, histogram, block
// segments, the total, staged tile ids.
__host__ __device__ constexpr size_t place_lds_bytes(int nt, int tile_bytes)
{
    return (size_t)nt * 8 + (size_t)kRecordsPerBlock * 8 + (size_t)nt * 8 + 16 + (size_t)kRecordsPerBlock * tile_bytes;
}

// TileT: type of the staged local tile ids (uint8_t when a level has at most
// 256 tiles, which keeps the block's LDS under 40 KB: four blocks per CU).
template <bool kMany, typename TileT>
__global__ __launch_bounds__(kPlaceThreads) void k_scatter_place(ScatterArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int nt_lds = a.tiles_max;
    uint64_t* gbase = reinterpret_cast<uint64_t*>(smem);
    uint64_t* s_rec = gbase + nt_lds;
    uint32_t* hist = reinterpret_cast<uint32_t*>(s_rec + kRecordsPerBlock);
    uint32_t* seg = hist + nt_lds;
    uint32_t* p_total = seg + nt_lds;
    TileT* s_tile = reinterpret_cast<TileT*>(p_total + 4);
    const int64_t item = blockIdx.x;
    const ScatterObj& o = sobj<kMany>(a, obj_of_item<kMany>(a, item));
    int l, bx;
    split_item(item - o.item_off, o.n_blocks, l, bx);
    const int nt = o.tiles[l];
    if (a.fwd_counts && a.tile_start[a.n_tiles] > (uint64_t)a.n_records) return;  // uniform: the scan's verdict
    // Global start of this block's run in the thread's tile (thread i holds
    // tile i; threads past the level's tiles load tile nt - 1 and ignore it).
    // Loaded first, together with the contribution, so the block waits on
    // global memory once.
    const int tb = o.tile_base[l];
    const int own = min((int)threadIdx.x, nt - 1);
    const uint64_t own_start = a.tile_start[o.tile_off + tb + own];
    const uint32_t own_off = a.offsets[o.count_off + (int64_t)(tb + own) * o.n_blocks + bx];
    const int E = level_rec_exp(a.level_max[o.lev_off + l]);
    for (int i = threadIdx.x; i < nt; i += kPlaceThreads) hist[i] = 0;
    __syncthreads();
    // pass 1: rank of each contribution within its tile (LDS atomics)
    const int64_t s = (int64_t)bx * kSamplesPerBlock + threadIdx.x;
    float2 d;
    Corners c;
    bool has;
    uint32_t heads = 0xffu;  // corners that start a record
    float2 val[8];
    if (a.merge_runs) {
        // every sample counted, repeated corners merged as the count (or the
        // forward) did: samples are a prefix of the wave, every lane takes part
        has = s < o.n_s;
        load_contrib(a, o, l, has ? s : o.n_s - 1, d, c);
        heads = run_heads(c, has);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            val[e] = has ? make_float2(c.w[e] * d.x, c.w[e] * d.y) : make_float2(0.0f, 0.0f);
            const bool head = (heads >> e) & 1u;
            if (__ballot(has && !head)) val[e] = run_sum(val[e], head || !has);
        }
    } else {
        has = s < o.n_s && load_contrib(a, o, l, s, d, c);
#pragma unroll
        for (int e = 0; e < 8; ++e) val[e] = make_float2(c.w[e] * d.x, c.w[e] * d.y);
    }
    uint32_t rank[8];
    if (has) {
        if (nt <= kAggregateTiles) {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if ((heads >> e) & 1u) rank[e] = wave_aggregated_add(hist, c.row[e] >> kTileBits);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if ((heads >> e) & 1u) rank[e] = atomicAdd(&hist[c.row[e] >> kTileBits], 1u);
        }
    }
    __syncthreads();
    // block-local segments: exclusive scan of hist (by one wave)
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        uint32_t carry = 0;
        for (int base = 0; base < nt; base += 64) {
            const int i = base + lane;
            uint32_t v = i < nt ? hist[i] : 0u, incl = v;
#pragma unroll
            for (int dd = 1; dd < 64; dd <<= 1) {
                const uint32_t up = __shfl_up(incl, dd);
                if (lane >= dd) incl += up;
            }
            if (i < nt) seg[i] = carry + incl - v;
            carry += __shfl(incl, 63);
        }
        if (lane == 0) *p_total = carry;
    }
    __syncthreads();
    // global position of record p of local tile tt: gbase[tt] + p
    {
        const uint32_t* cnt = a.offsets + o.count_off;
        if ((int)threadIdx.x < nt) gbase[threadIdx.x] = own_start + own_off - seg[threadIdx.x];
        for (int i = threadIdx.x + kPlaceThreads; i < nt; i += kPlaceThreads)
            gbase[i] = a.tile_start[o.tile_off + tb + i] + cnt[(int64_t)(tb + i) * o.n_blocks + bx] - seg[i];
    }
    // pass 2: stage the encoded records sorted by tile (corners kept from pass 1)
    if (has) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            if (!((heads >> e) & 1u)) continue;
            const uint32_t tt = c.row[e] >> kTileBits;
            const uint32_t p = seg[tt] + rank[e];
            s_rec[p] = a.compact ? encode_record<kRecExpBitsC, kRecMantBitsC>(val[e], E, c.row[e] & (kTileRows - 1))
                                 : encode_record<kRecExpBits, kRecMantBits>(val[e], E, c.row[e] & (kTileRows - 1));
            s_tile[p] = (TileT)tt;
        }
    }
    __syncthreads();
    // write each tile's run to its global range: consecutive threads, consecutive records
    // The staging arrays hold kRecordsPerBlock entries, so the LDS reads of
    // several records are issued before the guarded stores.
    const uint32_t total = *p_total;
    constexpr int kPer = kRecordsPerBlock / kPlaceThreads, kHalf = kPer / 2;
#pragma unroll
    for (int h = 0; h < kPer; h += kHalf) {
        if (h * kPlaceThreads >= (int)total) break;
        uint32_t tt[kHalf];
        uint64_t rec[kHalf];
#pragma unroll
        for (int k = 0; k < kHalf; ++k) {
            const uint32_t p = threadIdx.x + (h + k) * kPlaceThreads;
            tt[k] = s_tile[p];
            rec[k] = s_rec[p];
        }
#pragma unroll
        for (int k = 0; k < kHalf; ++k) {
            const uint32_t p = threadIdx.x + (h + k) * kPlaceThreads;
            const uint64_t dst = gbase[min(tt[k], (uint32_t)nt - 1u)] + p;
            if (p < total && dst < (uint64_t)a.n_records) {
                if (a.compact) {
                    reinterpret_cast<uint32_t*>(a.recs)[dst] = (uint32_t)rec[k];
                    reinterpret_cast<uint16_t*>(reinterpret_cast<uint32_t*>(a.recs) + a.n_records)[dst] =
                        (uint16_t)(rec[k] >> 32);
                } else {
                    a.recs[dst] = rec[k];
                }
            }
        }
    }
}

template <bool kMany, bool kCompact>
__global__ __launch_bounds__(kReduceThreads) void k_scatter_reduce(ScatterArgs a)
{
    constexpr int EB = kCompact ? kRecExpBitsC : kRecExpBits, MB = kCompact ? kRecMantBitsC : kRecMantBits;
    // a run's words: four 16-byte loads of 64-bit records, or two of 32-bit
    // low words and one of 16-bit high words
    constexpr int kLoads = kCompact ? 3 : kRun / 2;
    __shared__ unsigned long long acc[2 * kTileRows];  // fixed point: feature 0 rows, then feature 1 rows
    __shared__ int64_t s_chunk;
    const uint64_t n_chunks = a.chunk_start[a.n_tiles];
    const int cb = (int)a.chunk_start[a.n_tiles + 1];
    for (;;) {
        if (threadIdx.x == 0) s_chunk = (int64_t)atomicAdd(a.work_counter, 1ull);
        __syncthreads();
        const int64_t chunk = s_chunk;
        __syncthreads();
        if ((uint64_t)chunk >= n_chunks) break;
        // tile of this chunk: last t with chunk_start[t] <= chunk
        int64_t lo = 0, hi = a.n_tiles - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (a.chunk_start[mid] <= (uint64_t)chunk)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int64_t tile = lo;
        const ScatterObj& o = sobj<kMany>(a, obj_of_tile<kMany>(a, tile));
        const int lt = (int)(tile - o.tile_off);
        const int l = level_of_tile(o, lt);
        const int tt = lt - o.tile_base[l];
        const int64_t row0 = (int64_t)tt << kTileBits;
        const int n_rows = (int)min((int64_t)kTileRows, o.level_rows[l] - row0);
        const uint64_t k0 = chunk - a.chunk_start[tile];
        const uint64_t r_begin = a.tile_start[tile] + (k0 << cb);
        const uint64_t r_end = min(r_begin + ((uint64_t)1 << cb), a.tile_start[tile + 1]);
        const bool owner = (a.chunk_start[tile + 1] - a.chunk_start[tile]) == 1;
        const int ex = a.tile_exp[tile];
        // a record (qx, qy, r) is worth (qx, qy) 2^(E - r - (MB - 1)); in fixed
        // point at 2^ex that is (qx, qy) 2^(sh0 - r)
        const int sh0 = level_rec_exp(a.level_max[o.lev_off + l]) - (MB - 1) + ex;
        for (int i = threadIdx.x; i < n_rows; i += kReduceThreads) {
            acc[i] = 0ull;
            acc[kTileRows + i] = 0ull;
        }
        __syncthreads();
        // Each thread takes runs of kRun consecutive records (four 16-byte
        // loads; runs start at multiples of kRun, so the loads are aligned and
        // stay inside the record array, whose length is a multiple of kRun).
        // Records of a run outside [r_begin, r_end) add zero.  Consecutive
        // records often carry the same row (neighbouring samples of one ray on
        // a coarse level); such repeats are summed in registers first, so one
        // LDS atomic per row and run is issued instead of one per record.
        const uint64_t q_begin = r_begin / kRun, q_end = (r_end + kRun - 1) / kRun;
        for (uint64_t q0 = q_begin + threadIdx.x; q0 < q_end; q0 += (uint64_t)kReduceThreads * kRunsPerThread) {
            uint4 rw[kRunsPerThread][kLoads];
#pragma unroll
            for (int u = 0; u < kRunsPerThread; ++u) {
                const uint64_t q = q0 + (uint64_t)u * kReduceThreads;
                const uint64_t qc = q < q_end ? q : q_begin;
                if constexpr (kCompact) {
                    const uint32_t* lo = reinterpret_cast<const uint32_t*>(a.recs);
                    const uint16_t* hi = reinterpret_cast<const uint16_t*>(lo + a.n_records);
                    rw[u][0] = reinterpret_cast<const uint4*>(lo + qc * kRun)[0];
                    rw[u][1] = reinterpret_cast<const uint4*>(lo + qc * kRun)[1];
                    rw[u][2] = reinterpret_cast<const uint4*>(hi + qc * kRun)[0];
                } else {
                    const uint4* rp = reinterpret_cast<const uint4*>(a.recs + qc * kRun);
#pragma unroll
                    for (int i = 0; i < kRun / 2; ++i) rw[u][i] = rp[i];
                }
            }
#pragma unroll
            for (int u = 0; u < kRunsPerThread; ++u) {
                const uint64_t q = q0 + (uint64_t)u * kReduceThreads;
                const uint64_t rec0 = q * kRun;
                uint32_t key[kRun];
                long long sx[kRun], sy[kRun];
#pragma unroll
                for (int i = 0; i < kRun; ++i) {
                    uint32_t lo, hi;
                    if constexpr (kCompact) {
                        const uint4& l4 = rw[u][i >> 2];
                        lo = (i & 3) == 0 ? l4.x : (i & 3) == 1 ? l4.y : (i & 3) == 2 ? l4.z : l4.w;
                        const uint4& h4 = rw[u][2];
                        const uint32_t hw = (i >> 1) == 0 ? h4.x : (i >> 1) == 1 ? h4.y : (i >> 1) == 2 ? h4.z : h4.w;
                        hi = (i & 1) ? hw >> 16 : hw & 0xffffu;
                    } else {
                        lo = (i & 1) ? rw[u][i >> 1].z : rw[u][i >> 1].x;
                        hi = (i & 1) ? rw[u][i >> 1].w : rw[u][i >> 1].y;
                    }
                    int r;
                    long long qx, qy;
                    decode_record<EB, MB>((uint64_t)hi << 32 | lo, key[i], r, qx, qy);
                    const int sh = sh0 - r;
                    const bool ok = q < q_end && rec0 + i >= r_begin && rec0 + i < r_end;
                    sx[i] = ok ? scale_mantissa(qx, sh) : 0ll;
                    sy[i] = ok ? scale_mantissa(qy, sh) : 0ll;
                }
#pragma unroll
                for (int i = 1; i < kRun; ++i) {
                    if (key[i] == key[i - 1]) {
                        sx[i] += sx[i - 1];
                        sy[i] += sy[i - 1];
                        sx[i - 1] = 0;
                        sy[i - 1] = 0;
                    }
                }
#pragma unroll
                for (int i = 0; i < kRun; ++i) {
                    if (sx[i] != 0) atomicAdd(&acc[key[i]], (unsigned long long)sx[i]);
                    if (sy[i] != 0) atomicAdd(&acc[kTileRows + key[i]], (unsigned long long)sy[i]);
                }
            }
        }
        __syncthreads();
        float2* g = reinterpret_cast<float2*>(a.g_table + o.g_off) + ((int64_t)l << o.grid.log2_table) + row0;
        for (int i = threadIdx.x; i < n_rows; i += kReduceThreads) {
            const long long sx = (long long)acc[i], sy = (long long)acc[kTileRows + i];
            if (sx == 0 && sy == 0) continue;
            const float2 v = make_float2((float)ldexp((double)sx, -ex), (float)ldexp((double)sy, -ex));
            if (owner) {
                float2 w = g[i];
                w.x += v.x;
                w.y += v.y;
                g[i] = w;
            } else {
                atomicAdd(&g[i].x, v.x);
                atomicAdd(&g[i].y, v.y);
            }
        }
        __syncthreads();
    }
}

template <bool kMany>
hipError_t scatter_phase_impl(const ScatterArgs& a, int phase, hipStream_t s)
{
    switch (phase) {
        case 0:
            if (a.fwd_counts)
                hipLaunchKernelGGL(k_scatter_dymax<kMany>, dim3((uint32_t)((a.n_items + kDymaxItems - 1) / kDymaxItems)),
                                   dim3(kPlaceThreads), 0, s, a);
            else
                hipLaunchKernelGGL(k_scatter_count<kMany>, dim3((uint32_t)a.n_items), dim3(kPlaceThreads), 0, s, a);
            break;
        case 1:
            hipLaunchKernelGGL(k_scatter_level_max<kMany>, dim3((uint32_t)a.n_levels_total), dim3(kLevelMaxThreads), 0, s,
                               a);
            break;
        case 2:
            hipLaunchKernelGGL(k_scatter_scan_blocks<kMany>, dim3((uint32_t)a.n_tiles), dim3(kScanThreads), 0, s, a);
            break;
        case 3:
            hipLaunchKernelGGL(k_scatter_scan_tiles<kMany>, dim3(1), dim3(kScanThreads), 0, s, a);
            break;
        case 4: {
            const bool narrow = a.tiles_max <= 256;
            const size_t place_lds = place_lds_bytes(a.tiles_max, narrow ? 1 : 2);
            const void* fn = narrow ? (const void*)k_scatter_place<kMany, uint8_t> : (const void*)k_scatter_place<kMany, uint16_t>;
            hipError_t e;
            if (place_lds > 65536 &&
                (e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)place_lds)) != hipSuccess)
                return e;
            if (narrow)
                hipLaunchKernelGGL((k_scatter_place<kMany, uint8_t>), dim3((uint32_t)a.n_items), dim3(kPlaceThreads),
                                   place_lds, s, a);
            else
                hipLaunchKernelGGL((k_scatter_place<kMany, uint16_t>), dim3((uint32_t)a.n_items), dim3(kPlaceThreads),
                                   place_lds, s, a);
            break;
        }
        case 5:
            if (a.compact)
                hipLaunchKernelGGL((k_scatter_reduce<kMany, true>), dim3((uint32_t)a.reduce_blocks),
                                   dim3(kReduceThreads), 0, s, a);
            else
                hipLaunchKernelGGL((k_scatter_reduce<kMany, false>), dim3((uint32_t)a.reduce_blocks),
                                   dim3(kReduceThreads), 0, s, a);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

ScatterObj scatter_obj(const GridInfo& g, int64_t n_s)
{
    ScatterObj o{};
    o.grid = g;
    o.n_s = n_s;
    o.n_blocks = (int32_t)((n_s + kSamplesPerBlock - 1) / kSamplesPerBlock);
    o.n_tiles = 0;
    const int64_t T = (int64_t)1 << g.log2_table;
    for (int l = 0; l < g.n_levels; ++l) {
        const int64_t side = (int64_t)g.res[l] + 1;
        const int64_t rows = ((g.dense_mask >> l) & 1u) ? side * side * side : T;
        o.level_rows[l] = rows;
        o.tiles[l] = (int32_t)((rows + kTileRows - 1) / kTileRows);
        o.tile_base[l] = o.n_tiles;
        o.n_tiles += o.tiles[l];
    }
    return o;
}

int64_t scatter_items(const ScatterObj& o) { return (int64_t)o.grid.n_levels * o.n_blocks; }

// A multiple of kRun: the reduce reads whole aligned runs.
int64_t scatter_records(const ScatterObj& o) { return o.n_s * o.grid.n_levels * 8; }
static_assert(8 % kRun == 0, "record arrays must hold whole runs");

int scatter_max_tiles_per_level() { return kMaxTilesPerLevel; }

int scatter_tiles_max(const ScatterObj& o)
{
    int m = 1;
    for (int l = 0; l < o.grid.n_levels; ++l) m = o.tiles[l] > m ? o.tiles[l] : m;
    return m;
}

const char* const kScatterPhaseNames[kScatterPhases] = {"k_scatter_count",      "k_scatter_level_max",
                                                        "k_scatter_scan_blocks", "k_scatter_scan_tiles",
                                                        "k_scatter_place",      "k_scatter_reduce"};

hipError_t launch_scatter_phase(const ScatterArgs& a, int phase, hipStream_t s)
{
    if (a.n_items == 0) return hipSuccess;
    return a.n_obj == 1 && a.objs == nullptr ? scatter_phase_impl<false>(a, phase, s)
                                             : scatter_phase_impl<true>(a, phase, s);
}

}  // namespace prenom

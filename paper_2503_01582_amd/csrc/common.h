// Internal declarations shared by the HIP translation units of libprenom.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "prenom.h"

namespace prenom {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// Level table of a hash grid, passed by value to kernels.
struct GridInfo {
    int32_t res[PRENOM_MAX_LEVELS];
    uint32_t dense_mask;  // bit l set: level l stored 1:1 ((N_l+1)^3 <= T)
    int32_t n_levels;
    int32_t log2_table;
};

// Table row of lattice vertex (vx, vy, vz) on one level: 1:1 on dense levels,
// otherwise the XOR-of-primes spatial hash of the multiresolution hash
// encoding (Mueller et al. 2022) reduced modulo 2^32 and masked to T.
__device__ __forceinline__ uint32_t corner_row(bool dense, uint32_t side, uint32_t log2T, uint32_t vx,
                                               uint32_t vy, uint32_t vz)
{
    if (dense) return vx + side * (vy + side * vz);
    return (vx ^ (vy * 2654435761u) ^ (vz * 805459861u)) & ((1u << log2T) - 1u);
}

// Cell of x on a lattice of resolution N: c = min(floor(x N), N - 1) of the
// exact product, and the local coordinate f = x N - c rounded to FP32.  In
// FP32: N < 2^20 is exact, and rounding x N to nearest never takes it below
// an integer it reaches, so floor of the rounded product is the exact floor
// or one above it; fma(x, N, -c) is the exact x N - c rounded once, so its
// sign tells which, and after the clamp it is f itself.
__device__ __forceinline__ void lattice_cell(float x, int N, uint32_t& c, float& f)
{
    const float Nf = (float)N;
    float cf = floorf(x * Nf);
    if (fmaf(x, Nf, -cf) < 0.0f) cf -= 1.0f;
    cf = fminf(fmaxf(cf, 0.0f), (float)(N - 1));
    c = (uint32_t)cf;
    f = fmaf(x, Nf, -cf);
}

// The 8 cell corners of x on level l: table rows and trilinear weights
// (corner e = (e & 1, e >> 1 & 1, e >> 2 & 1)).  Used by the forward encoding
// and by both passes of the scatter, so all of them agree bit for bit.
struct Corners {
    uint32_t row[8];
    float w[8];
};

// Sample position in the object frame: clamp(fmaf(t, d, o), 0, 1).
__device__ __forceinline__ float sample_coord(float t, float d, float o)
{
    return fminf(fmaxf(fmaf(t, d, o), 0.0f), 1.0f);
}

__device__ __forceinline__ void level_corners(const GridInfo& g, int l, float x0, float x1, float x2, Corners& c)
{
    const int N = g.res[l];
    const bool dense = (g.dense_mask >> l) & 1u;
    const uint32_t side = (uint32_t)N + 1u;
    uint32_t cx, cy, cz;
    float fx, fy, fz;
    lattice_cell(x0, N, cx, fx);
    lattice_cell(x1, N, cy, fy);
    lattice_cell(x2, N, cz, fz);
    // Rows of the 8 corners from two products per level (corner_row of each
    // corner, strength-reduced): (c + 1) P = c P + P modulo 2^32 for the hash,
    // and the 1:1 row of a corner is the cell's row plus 1, side or side^2.
    uint32_t r0 = 0, ry = 0, rz = 0, hy[2] = {0, 0}, hz[2] = {0, 0};
    if (dense) {
        r0 = cx + side * (cy + side * cz);
        ry = side;
        rz = side * side;
    } else {
        hy[0] = cy * 2654435761u;
        hy[1] = hy[0] + 2654435761u;
        hz[0] = cz * 805459861u;
        hz[1] = hz[0] + 805459861u;
    }
    const uint32_t mask = (1u << g.log2_table) - 1u;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const uint32_t ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
        c.row[e] = dense ? r0 + ex + (ey ? ry : 0u) + (ez ? rz : 0u) : ((cx + ex) ^ hy[ey] ^ hz[ez]) & mask;
        c.w[e] = (ex ? fx : 1.0f - fx) * (ey ? fy : 1.0f - fy) * (ez ? fz : 1.0f - fz);
    }
}

// ------------------------------------------------------------------ table tiles
// The hash-table gradient buckets contributions by table tile (2^13 rows),
// per (level, block of kScatterBlockSamples samples).  The training forward
// writes the same per-block tile histograms as it encodes (TileHist).
constexpr int kTileBits = 13;
constexpr int kTileRows = 1 << kTileBits;
constexpr int kMaxTilesPerLevel = 1 << (24 - kTileBits);  // T <= 2^24
constexpr int kScatterBlockSamples = 512;
// Place combines the rank atomics of a wave per tile first on levels of at
// most this many tiles, where most lanes of a wave share a tile.  With more
// tiles the leader rounds cost more vector instructions than the LDS
// serialisation of same-address atomics they save, dense levels included
// (48-object place on gfx950: 17.2 ms aggregating up to 16 tiles, 16.3 ms
// up to 4 hashed or 16 dense, 15.7 ms up to 2).
constexpr int kAggregateTiles = 2;

// Adds 1 to hist[tile] for every active lane and returns the lane's rank
// among the additions to that tile.  Lanes of the wave that share the tile of
// the first remaining lane are combined into one LDS atomic issued by that
// lane (same-address atomics of one instruction would otherwise serialise);
// after kAggregateRounds such rounds the lanes left use plain LDS atomics, so
// a wave spread over many tiles does not pay one round per tile.  Every slot
// comes from an atomic on the same counter, so ranks are distinct whichever
// way a lane takes.
constexpr int kAggregateRounds = 2;

__device__ __forceinline__ uint32_t wave_aggregated_add(uint32_t* hist, uint32_t tile)
{
    const int lane = threadIdx.x & 63;
    const uint64_t lane_lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint64_t remaining = __ballot(1);
    uint32_t rank = 0;
    bool placed = false;
#pragma unroll
    for (int round = 0; round < kAggregateRounds; ++round) {
        if (remaining == 0) break;
        const int leader = __ffsll((unsigned long long)remaining) - 1;
        const uint32_t lt = __shfl(tile, leader);
        const uint64_t mask = __ballot(tile == lt);
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&hist[lt], (uint32_t)__popcll(mask));
        base = __shfl(base, leader);
        if (tile == lt) {
            rank = base + (uint32_t)__popcll(mask & lane_lt);
            placed = true;
        }
        remaining &= ~mask;
    }
    if (!placed) rank = atomicAdd(&hist[tile], 1u);
    return rank;
}

// Lane exchange within a row of 16 lanes (DPP): kCtrl = 0x100 + n (row_shl:
// lane i reads lane i + n, 0 past the row end) or 0x110 + n (row_shr: lane i
// reads lane i - n, 0 before the row start).  All lanes must be active.
template <int kCtrl>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, 0xf, 0xf, true);
}

template <int kCtrl>
__device__ __forceinline__ float dpp_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, 0xf, 0xf, true));
}

// Tile histogram of the wave's records on a level of at most 16 tiles, for
// counting only (no ranks): bit e of `heads` marks corner e as a record.  Each
// lane counts its records per tile in the 4-bit fields of a 64-bit word (at
// most 8 per tile), the fields are widened to bytes and summed over each row
// of 16 lanes by four DPP additions (mirror, half mirror, two quad swaps:
// every lane ends with the row's sums, at most 128 per tile), and lane i of
// each row adds the row's count of tile i.  About 90 instructions per wave,
// against about 35 per corner for wave_aggregated_add.  Every lane of the wave
// must call it (lanes without records pass heads = 0).
__device__ __forceinline__ void wave_count_tiles16(uint32_t* hist, const uint32_t row[8], uint32_t heads, int nt)
{
    uint64_t p = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const uint32_t t = row[e] >> kTileBits;  // < 16 for every row of the level
        p += (uint64_t)((heads >> e) & 1u) << ((4u * t) & 63u);
    }
    const uint32_t lo = (uint32_t)p, hi = (uint32_t)(p >> 32);
    // v[k]: tile b sits in byte (b >> 1) & 3 of v[(b & 1) * 2 + (b >> 3)]
    uint32_t v[4] = {lo & 0x0f0f0f0fu, hi & 0x0f0f0f0fu, (lo >> 4) & 0x0f0f0f0fu, (hi >> 4) & 0x0f0f0f0fu};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] += dpp_u32<0x140>(v[k]);  // row_mirror: lane i + lane 15 - i
        v[k] += dpp_u32<0x141>(v[k]);  // row_half_mirror
        v[k] += dpp_u32<0x1b>(v[k]);   // quad_perm [3, 2, 1, 0]
        v[k] += dpp_u32<0xb1>(v[k]);   // quad_perm [1, 0, 3, 2]
    }
    const uint32_t b = threadIdx.x & 15u;
    const uint32_t k = (b & 1u) * 2u + (b >> 3);
    const uint32_t w = k == 0 ? v[0] : k == 1 ? v[1] : k == 2 ? v[2] : v[3];
    const uint32_t cnt = (w >> (8u * ((b >> 1) & 3u))) & 0xffu;
    if ((int)b < nt && cnt != 0u) atomicAdd(&hist[b], cnt);
}

// Adds the lane's records (bit e of heads: corner e) to a block's LDS tile
// histogram of a level of nt tiles.  Every lane of the wave must call it.
__device__ __forceinline__ void count_records(uint32_t* hist, const Corners& c, uint32_t heads, int nt)
{
    if (nt <= 16) {
        wave_count_tiles16(hist, c.row, heads, nt);
        return;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e)
        if ((heads >> e) & 1u) atomicAdd(&hist[c.row[e] >> kTileBits], 1u);
}

// Merging repeated corners.  Consecutive samples of a ray often share a cell
// on the coarser levels, so the same corner row repeats on neighbouring
// lanes; such a run becomes one record (the sum of its contributions).  Runs
// stay inside groups of 8 lanes.  Bit e of the result is set when the lane's
// corner e starts a run: the lane holds a sample and is the first of its
// group of 8, or lane - 1's corner e has another row.  Lanes with samples
// must form a prefix of the wave (then lane - 1 holds one whenever the lane
// does).  Every lane of the wave must call it.
__device__ __forceinline__ uint32_t run_heads(const Corners& c, bool has)
{
    const bool first = (threadIdx.x & 7) == 0;
    uint32_t m = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const uint32_t prev = dpp_u32<0x111>(c.row[e]);
        if (has && (first || prev != c.row[e])) m |= 1u << e;
    }
    return m;
}

// Per lane that starts a run (boundary set): the sum of v over its run (the
// lane and the following lanes of its group of 8 up to the next boundary); a
// segmented suffix scan in three steps, in a fixed order.  Lanes without a
// sample pass v = 0 and boundary = true.  Every lane of the wave must call it.
__device__ __forceinline__ float2 run_sum(float2 v, bool boundary)
{
    const int g = threadIdx.x & 7;
    const int lane = threadIdx.x & 63;
    const uint64_t B = __ballot(boundary);
    // lane + 1 .. lane + d continue this lane's run (they lie in its group)
    const bool c1 = g + 1 < 8 && ((B >> (lane + 1)) & 1ull) == 0;
    const bool c2 = g + 2 < 8 && ((B >> (lane + 1)) & 3ull) == 0;
    const bool c4 = g + 4 < 8 && ((B >> (lane + 1)) & 15ull) == 0;
    float ox = dpp_f32<0x101>(v.x), oy = dpp_f32<0x101>(v.y);
    if (c1) { v.x += ox; v.y += oy; }
    ox = dpp_f32<0x102>(v.x);
    oy = dpp_f32<0x102>(v.y);
    if (c2) { v.x += ox; v.y += oy; }
    ox = dpp_f32<0x104>(v.x);
    oy = dpp_f32<0x104>(v.y);
    if (c4) { v.x += ox; v.y += oy; }
    return v;
}

// Tile histograms of one object: counts[(tile_base[l] + i) * n_blocks + b]
// = records (runs of repeated corners, run_heads) of sample block b of level
// l in tile i of that level.
struct TileHist {
    uint32_t* counts;
    int32_t n_blocks;
    int32_t pad_;
    int32_t tiles[PRENOM_MAX_LEVELS];
    int32_t tile_base[PRENOM_MAX_LEVELS];
};

// ------------------------------------------------------------------ batches
// Device descriptor of one object of a batch (offsets index the batch's
// concatenated arrays; objects own consecutive rays).
struct ObjDev {
    GridInfo grid;
    int32_t table_dtype;  // PRENOM_F32 or PRENOM_F16 (read the FP16 parameter copy)
    int32_t prior_res;
    int32_t pad_[2];
    int64_t param_off;    // floats: first parameter (the tables) of the object
    int64_t ray_begin, n_rays;
    int64_t y_off;        // floats: the object's features [L][n_s][2] (and their gradient)
    const float* prior;   // [R^3] or null (uniform sampling)
    double A[12];         // world -> object frame
};

// Object of a batch that holds ray `ray` (objects are contiguous in rays).
__device__ __forceinline__ int find_object(const ObjDev* objs, int n_obj, int64_t ray)
{
    int lo = 0, hi = n_obj - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (objs[mid].ray_begin <= ray)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------------------ launches
// Every launcher returns hipSuccess or the launch error.

struct SampleArgs {
    int32_t n_coarse, n_fine, include_coarse, use_prior;
    double eps, near_t, far_t;
    double A[12];
    const float* prior;
    int32_t R;
    const float* rays_o;
    const float* rays_d;
    const float* xi;
    int64_t n;
    float* ray_obj;
    float* t;
    float* dt;
    int32_t* bins;
    uint8_t* flags;
};
hipError_t launch_sample(const SampleArgs& a, hipStream_t s);
hipError_t launch_sample_batch(const SampleArgs& a, const ObjDev* objs, int n_obj, hipStream_t s);

// Encoding of the grid vertices p0 .. p0 + cnt - 1 of the R^3 grid, vertex
// p = (k R + j) R + i at (i, j, k) / (R - 1): features [L][cnt][2]; and the
// density column of head outputs sc [n][4] into out [n].
hipError_t launch_encode_grid(const GridInfo& g, const float* table, const void* table_f16, int32_t R, int64_t p0,
                              int64_t cnt, float* y, hipStream_t s);
hipError_t launch_density_grid(const float* sc, int64_t n, float* out, hipStream_t s);

// Encoding of explicit positions: features [L][n][2], optional corner rows.
hipError_t launch_encode_points(const GridInfo& g, const float* table, const float* pos, int64_t n,
                                float* features, int32_t* corner_idx, hipStream_t s);

struct ScatterObj;
// Encoding of the rendered samples of every object of a batch, which also
// writes the tile histograms of its hash-table gradient: one block per
// scatter item (object, level, sample block) of sobjs, counts laid out as the
// scatter reads them; FP16 tables come from params_f16.
hipError_t launch_encode_batch_hist(const ObjDev* objs, const ScatterObj* sobjs, int n_obj, int64_t n_items,
                                    const float* params, const void* params_f16, const float* ray_obj, const float* t,
                                    int32_t S, float* y, uint32_t* counts, hipStream_t s);

// Encoding of the rendered samples (positions from rays and t); reads the
// FP16 table copy when table_f16 is not null, the FP32 tables otherwise.
// hist (or null): also write the tile histograms of every (level, block of
// kScatterBlockSamples samples), counting every sample, for the backward.
hipError_t launch_encode_samples(const GridInfo& g, const float* table, const void* table_f16,
                                 const float* ray_obj, const float* t, int64_t n_rays, int32_t S, float* y,
                                 hipStream_t s, const TileHist* hist = nullptr);

// Bucketed scatter-add of the feature gradients into the table gradient.
// Geometry of one object's scatter: its table tiles and sample blocks, and
// where its pieces sit in the (possibly batched) arrays.
struct ScatterObj {
    GridInfo grid;
    int32_t n_blocks;  // sample blocks per level
    int32_t n_tiles;   // table tiles over the object's levels
    int32_t lev_off;   // first (object, level) entry of level_max
    int32_t pad_;
    int32_t tiles[PRENOM_MAX_LEVELS];
    int32_t tile_base[PRENOM_MAX_LEVELS];
    int64_t level_rows[PRENOM_MAX_LEVELS];
    int64_t n_s;        // samples
    int64_t s_begin;    // first sample in the per-sample arrays (t; ray = sample / S)
    int64_t dy_off;     // float2 index of the object's dy [L][n_s]
    int64_t g_off;      // float index of the object's table gradient
    int64_t tile_off;   // first tile in the per-tile arrays
    int64_t count_off;  // first entry of its counts [n_tiles][n_blocks]
    int64_t bmax_off;   // first entry of its block_max [L][n_blocks]
    int64_t item_off;   // first (level, sample block) item of the count and place grids
};
// Fills the geometry of one object (offsets within the batch are left 0).
ScatterObj scatter_obj(const GridInfo& g, int64_t n_s);
int64_t scatter_items(const ScatterObj& o);      // L * n_blocks
int64_t scatter_records(const ScatterObj& o);    // n_s * L * 8
int scatter_max_tiles_per_level();
int scatter_tiles_max(const ScatterObj& o);      // max tiles of one level

struct ScatterArgs {
    int32_t S;
    int32_t n_obj;              // 1: `one` holds the object; else `objs` (device) holds n_obj of them
    int32_t tiles_max;          // max tiles of one level over all objects
    int32_t reduce_blocks;
    int64_t n_tiles;            // over all objects
    int64_t n_items;            // (object, level, sample block) items of count and place
    int32_t n_levels_total;     // (object, level) pairs
    int32_t pad_;
    ScatterObj one;
    const ScatterObj* objs;
    const float* ray_obj;
    const float* t;
    const float2* dy;
    float* g_table;
    uint32_t* counts;       // per object [n_tiles][n_blocks], read only after the first phase
    uint32_t* offsets;      // same layout: per block, its first record within the tile
    float* block_max;       // per object [L][n_blocks] max |dy| per sample block
    float* level_max;       // [n_levels_total]
    int32_t* tile_exp;      // [n_tiles] fixed-point exponent
    uint64_t* tile_total;   // [n_tiles]
    uint64_t* tile_start;   // [n_tiles + 1]
    uint64_t* chunk_start;  // [n_tiles + 2]: chunk bases, their total, the chunk size's log2
    unsigned long long* work_counter;
    uint64_t* recs;         // [records] packed records (scatter.hip: row, shared exponent, two mantissas); 8 bytes each
    int64_t n_records;      // length of recs
    int32_t* nonfinite;     // set to 1 when a dy entry is not finite (loss scaling), or null
    // 1: counts were written by the training forward (TileHist); the first
    // phase then only takes the per-block max |dy|, and the scan checks the
    // histograms hold at most n_records (else place and reduce do nothing).
    // 0: the first phase counts.
    int32_t fwd_counts;
    // 1: every sample counted, a corner repeating the previous lane's row
    // joining its record (run_heads; the rule the forward's histograms
    // follow).  0: one record per corner of every sample whose dy is not zero.
    int32_t merge_runs;
    // log2 of the smallest reduce work item in records (18..21; the scan picks
    // a size from the pass's records).  A tile longer than one item is summed
    // by several workgroups whose FP32 partials meet in atomics, in an order
    // that can change the last bits; 21 keeps most tiles to one item.
    int32_t chunk_min_bits;
    // 1: compact records (15-bit mantissas, 48 bits: 32-bit words at recs,
    // then n_records 16-bit words), for FP16 tables; 0: 64-bit records.
    int32_t compact;
};
// The scatter runs as kScatterPhases dependent kernels, launched in order
// (phase 0 .. kScatterPhases - 1): count (or, with fwd_counts, the block
// maxima of |dy| alone), per-level max, scan over blocks, scan over tiles,
// place, reduce.
constexpr int kScatterPhases = 6;
extern const char* const kScatterPhaseNames[kScatterPhases];
hipError_t launch_scatter_phase(const ScatterArgs& a, int phase, hipStream_t s);

// MLP: forward writes (sigma, r, g, b) per sample; backward recomputes the
// activations, writes dy and per-wave partial weight gradients.
struct MlpShape {
    int32_t in_dim, width, hidden, dtype;
};
bool mlp_supported(const MlpShape& m);

// One block's share of a batched MLP launch: tiles [tile_begin, tile_end) of
// one object.  w_off (floats) locates the object's MLP weights in the batch
// parameters, y_off (floats) its features (level-major [L][n_s][2]), s_off
// (samples) its first sample in the per-sample arrays, a_off (floats) its
// stored activations and deltas when the MLP is 128 wide.
struct MlpWork {
    int64_t w_off, y_off, s_off, n_s;
    int64_t tile_begin, tile_end;
    int64_t a_off;
    int64_t bmax_off;   // the object's [L][n_blocks] maxima of |dy| (scatter blocks), written by the backward
    int64_t n_sblocks;  // its scatter blocks (kScatterBlockSamples samples each)
};

// The 128-wide MLP stores its hidden activations in the forward and runs its
// backward as a chain kernel (deltas, dy) and a weight-gradient kernel; the
// two buffers hold act[D][n_s][W] and delta[D][n_s][W], FP32 in the FP32
// form and already rounded to the MFMA type (16 bits) in the reduced form,
// where they only ever enter the matrix cores rounded (and the ReLU masks
// only need their sign).
constexpr int kWideWidth = 128;
inline int64_t mlp_act_floats(const MlpShape& m, int64_t n_s)
{
    if (m.width < kWideWidth) return 0;
    // FP32: activations and deltas; 16-bit: both in the MFMA type (whole 16-sample
    // tiles), plus the ReLU mask words
    const int64_t n_sp = (n_s + 15) / 16 * 16;
    return m.dtype == PRENOM_F32 ? 2 * (int64_t)m.hidden * n_s * m.width
                                 : (int64_t)m.hidden * n_sp * (m.width + m.width / 32);
}
int mlp_bwd_waves(int64_t n_samples);  // partial-gradient slots (one per block) the bwd writes
// act: activation/delta buffer of mlp_act_floats floats (128-wide MLPs; else unused)
hipError_t launch_mlp_fwd(const MlpShape& m, const float* w, const float* y, int64_t n_s, float* sc, float* act,
                          hipStream_t s);
hipError_t launch_mlp_bwd(const MlpShape& m, const float* w, const float* y, const float* dout, const float* sc,
                          int64_t n_s, float* dy, float* partial, float* act, hipStream_t s);
hipError_t launch_mlp_fwd_lp(const MlpShape& m, const float* w, const float* y, int64_t n_s, float* sc, float* act,
                             hipStream_t s);
hipError_t launch_mlp_bwd_lp(const MlpShape& m, const float* w, const float* y, const float* dout, const float* sc,
                             int64_t n_s, float* dy, float* partial, float* act, hipStream_t s);
hipError_t launch_mlp_fwd_batch(const MlpShape& m, const MlpWork* work, int n_blocks, const float* params,
                                const float* y, float* sc, float* act, hipStream_t s);
// Batched backward: besides dy and the partial weight gradients, every work
// item writes its maxima of |dy| into block_max (MlpWork::bmax_off) and sets
// *nonfinite (when not null) on a non-finite dy; work items start at a
// multiple of kScatterBlockSamples / 16 tiles and span at most 1024 tiles.
hipError_t launch_mlp_bwd_batch(const MlpShape& m, const MlpWork* work, int n_blocks, const float* params,
                                const float* y, const float* dout, const float* sc, float* dy, float* partial,
                                int64_t slot_stride, float* act, float* block_max, int32_t* nonfinite,
                                hipStream_t s);
hipError_t launch_mlp_fwd_lp_batch(const MlpShape& m, const MlpWork* work, int n_blocks, const float* params,
                                   const float* y, float* sc, float* act, hipStream_t s);
hipError_t launch_mlp_bwd_lp_batch(const MlpShape& m, const MlpWork* work, int n_blocks, const float* params,
                                   const float* y, const float* dout, const float* sc, float* dy, float* partial,
                                   int64_t slot_stride, float* act, float* block_max, int32_t* nonfinite,
                                   hipStream_t s);
hipError_t launch_reduce_partials(const float* partial, int n_slots, int64_t n_mlp, float* g_mlp,
                                  hipStream_t s);

// Per object of a batch: where its backward partials sit and where its MLP
// gradient goes.  mlp_begin is the prefix of n_mlp over the objects.
struct MlpRed {
    int64_t mlp_begin, n_mlp;
    int64_t partial_off;  // floats
    int64_t n_slots;      // partials (each n_mlp floats, consecutive)
    int64_t g_off;        // floats: the object's MLP gradient in the batch gradient
};
hipError_t launch_reduce_partials_batch(const MlpRed* reds, int n_obj, int64_t n_mlp_total, const float* partial,
                                        float* grads, hipStream_t s);

// Compositing and loss.
struct CompositeArgs {
    int64_t n_rays;
    int64_t norm_rays;    // single object: rays the loss is averaged over (0: n_rays), for calls over a part of them
    int32_t S;
    int32_t loss_mode;
    float lambda_d, lambda_sigma;
    const float* sc;      // [n_s][4]
    const float* t;       // [n_rays][S]
    const float* dt;      // [n_rays][S]
    const uint8_t* flags;
    const float* bg;      // [n][3] or null
    const float* tgt_rgb; // [n][3] or null
    const float* tgt_depth;
    const uint8_t* mask;
    float* rgb;           // fwd outputs, or null (then only ray_state is written)
    float* depth;
    float* opacity;
    float* ray_state;     // [n][8]: rgb(3), depth, T_S, sigma sum, -, -
    double* loss_partial; // [blocks]
    const ObjDev* objs;   // batch: per-object loss normalisation (n = the object's rays), or null
    int32_t n_obj;
    double* ray_loss;     // batch fwd: [n_rays] loss term of each ray
    const float* d_rgb;   // bwd only
    const float* d_depth;
    const float* d_opacity;
    const float* loss_scale;  // bwd: device scalar multiplying the upstream gradient, or null
    float* dout;          // bwd: [n_s][4] (dsigma, dr, dg, db)
};
int composite_loss_blocks(int64_t n_rays);
int composite_rays_per_block();  // rays of one compositing block (its loss partial)
hipError_t launch_composite_fwd(const CompositeArgs& a, hipStream_t s);
hipError_t launch_loss_finalize(const double* partial, int n_blocks, float* loss, hipStream_t s);
hipError_t launch_composite_bwd(const CompositeArgs& a, hipStream_t s);
// loss[o] = sum of ray_loss over the rays of object o (FP64), one block per object.
hipError_t launch_loss_objects(const ObjDev* objs, int n_obj, const double* ray_loss, float* loss, hipStream_t s);

struct AdamArgs {
    float* p;
    float* g;
    float* m;
    float* v;
    int64_t n;
    float lr, beta1, beta2, eps, inv_c1, inv_c2;
    void* table_f16;         // FP16 copy of the first n_table entries, or null
    int64_t n_table;
    float* loss_scale;       // null: plain Adam
    int32_t* scaler_state;   // [2] non-finite flag, finite steps since the last scale change
    int32_t growth_interval;
    int64_t* step_dev;       // non-null: bias corrections from this device step counter, which is
                             // advanced after every applied (not skipped) step
};
hipError_t launch_adam(const AdamArgs& a, hipStream_t s);
// Plain gradient descent p -= lr g on the same arguments (m, v, beta1, beta2,
// eps and the bias corrections unused).
hipError_t launch_sgd(const AdamArgs& a, hipStream_t s);
hipError_t launch_to_f16(const float* src, void* dst, int64_t n, hipStream_t s);

// Reptile's outer update over n_tasks parameter vectors trained from theta:
// theta += beta * mean_b(task_b - theta), then every task slot (and its FP16
// copy, and its Adam moments, when given) restarts from the new theta.
struct ReptileArgs {
    float* theta;
    float* tasks;            // task b at tasks + b * stride
    float* m;                // Adam moments in the task layout, or null
    float* v;
    void* tasks_f16;         // FP16 copy in the task layout (its first n_f16 entries), or null
    int64_t* step;           // device step counter reset to 0, or null
    int64_t n, stride;       // stride a multiple of 4
    int64_t n_f16;
    int32_t n_tasks;
    float beta;
};
hipError_t launch_reptile(const ReptileArgs& a, hipStream_t s);

// Trilinear, vertex-aligned lookup of a density grid F [R][R][R] (x fastest;
// value F[i] at i/(R-1)), each coordinate clamped to [0, 1] (NaN to 0); FP64
// without contraction, the sampler's prior lookup (Eq. (4)) and the canonical
// yaw score (Eq. (3)).
__device__ inline double prior_at(const float* __restrict__ F, int R, const double xin[3])
{
#pragma clang fp contract(off)
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

// Canonical yaw search (Eq. (3)); workspace: per (yaw, chunk) extents and sums.
struct YawArgs {
    const float* pts;   // [n][3]
    int64_t n;
    const float* F;     // [R][R][R]
    int32_t R, K;
    int64_t n_chunks;
    double* part_ext;   // [K][n_chunks][6]: min xyz, max xyz
    double* part_sum;   // [K][n_chunks]
    double* scores;     // [K]
    double* extents;    // [K][3]
    double* centers;    // [K][3]
    int32_t* best;
};
int64_t yaw_chunks(int64_t n);
hipError_t launch_canonical_yaw(const YawArgs& a, hipStream_t s);

}  // namespace prenom

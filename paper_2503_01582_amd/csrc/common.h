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
// exact product (an FP32 x times an integer below 2^20 is exact in FP64), and
// the local coordinate f = x N - c rounded to FP32.
__device__ __forceinline__ void lattice_cell(float x, int N, uint32_t& c, float& f)
{
    const double g = (double)x * (double)N;
    int ci = (int)floor(g);
    ci = ci > N - 1 ? N - 1 : ci;
    ci = ci < 0 ? 0 : ci;
    c = (uint32_t)ci;
    f = (float)(g - (double)ci);
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
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const uint32_t ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
        c.row[e] = corner_row(dense, side, (uint32_t)g.log2_table, cx + ex, cy + ey, cz + ez);
        c.w[e] = (ex ? fx : 1.0f - fx) * (ey ? fy : 1.0f - fy) * (ez ? fz : 1.0f - fz);
    }
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

// Encoding of explicit positions: features [L][n][2], optional corner rows.
hipError_t launch_encode_points(const GridInfo& g, const float* table, const float* pos, int64_t n,
                                float* features, int32_t* corner_idx, hipStream_t s);

// Encoding of the rendered samples (positions from rays and t); reads the
// FP16 table copy when table_f16 is not null, the FP32 tables otherwise.
hipError_t launch_encode_samples(const GridInfo& g, const float* table, const void* table_f16,
                                 const float* ray_obj, const float* t, int64_t n_rays, int32_t S, float* y,
                                 hipStream_t s);

// Bucketed scatter-add of the feature gradients into the table gradient.
struct ScatterPlan {
    int32_t n_blocks;  // sample blocks per level
    int32_t n_tiles;   // table tiles over all levels
    int32_t tiles[PRENOM_MAX_LEVELS];
    int32_t tile_base[PRENOM_MAX_LEVELS];
    int64_t level_rows[PRENOM_MAX_LEVELS];
    int64_t max_records;  // n_s * L * 8
};
ScatterPlan scatter_plan(const GridInfo& g, int64_t n_s);
int scatter_max_tiles_per_level();

struct ScatterArgs {
    GridInfo grid;
    int64_t n_s;
    int32_t S;
    int32_t n_blocks, n_tiles, reduce_blocks;
    int32_t tiles_max;  // max tiles of one level
    int32_t tiles[PRENOM_MAX_LEVELS];
    int32_t tile_base[PRENOM_MAX_LEVELS];
    int64_t level_rows[PRENOM_MAX_LEVELS];
    const float* ray_obj;
    const float* t;
    const float2* dy;
    float* g_table;
    uint32_t* counts;       // [n_tiles][n_blocks]
    float* block_max;       // [L][n_blocks] max |dy| per sample block
    int32_t* tile_exp;      // [n_tiles] fixed-point exponent
    uint64_t* tile_total;   // [n_tiles]
    uint64_t* tile_start;   // [n_tiles + 1]
    uint64_t* chunk_start;  // [n_tiles + 1]
    unsigned long long* work_counter;
    uint16_t* keys;         // [max_records]
    float2* vals;           // [max_records]
};
hipError_t launch_scatter(const ScatterArgs& a, hipStream_t s);

// MLP: forward writes (sigma, r, g, b) per sample; backward recomputes the
// activations, writes dy and per-wave partial weight gradients.
struct MlpShape {
    int32_t in_dim, width, hidden, dtype;
};
bool mlp_supported(const MlpShape& m);
int mlp_bwd_waves(int64_t n_samples);  // partial-gradient slots (one per block) the bwd writes
hipError_t launch_mlp_fwd(const MlpShape& m, const float* w, const float* y, int64_t n_s, float* sc,
                          hipStream_t s);
hipError_t launch_mlp_bwd(const MlpShape& m, const float* w, const float* y, const float* dout,
                          int64_t n_s, float* dy, float* partial, hipStream_t s);
hipError_t launch_mlp_fwd_lp(const MlpShape& m, const float* w, const float* y, int64_t n_s, float* sc,
                             hipStream_t s);
hipError_t launch_mlp_bwd_lp(const MlpShape& m, const float* w, const float* y, const float* dout, int64_t n_s,
                             float* dy, float* partial, hipStream_t s);
hipError_t launch_reduce_partials(const float* partial, int n_slots, int64_t n_mlp, float* g_mlp,
                                  hipStream_t s);

// Compositing and loss.
struct CompositeArgs {
    int64_t n_rays;
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
    const float* d_rgb;   // bwd only
    const float* d_depth;
    const float* d_opacity;
    const float* loss_scale;  // bwd: device scalar multiplying the upstream gradient, or null
    float* dout;          // bwd: [n_s][4] (dsigma, dr, dg, db)
};
int composite_loss_blocks(int64_t n_rays);
hipError_t launch_composite_fwd(const CompositeArgs& a, hipStream_t s);
hipError_t launch_loss_finalize(const double* partial, int n_blocks, float* loss, hipStream_t s);
hipError_t launch_composite_bwd(const CompositeArgs& a, hipStream_t s);

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
};
hipError_t launch_adam(const AdamArgs& a, hipStream_t s);
hipError_t launch_to_f16(const float* src, void* dst, int64_t n, hipStream_t s);

}  // namespace prenom

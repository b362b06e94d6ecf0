/*
 * prenom.h -- C ABI of the MI355X (gfx950) per-object NeRF training step of
 * PRENOM (arXiv 2503.01582, Sec. III-B "Online Object Mapping").
 *
 * One training iteration of one object NeRF is
 *
 *   prenom_sample      prior-based probabilistic ray sampling   Sec. III-B, Eq. (4)-(6)
 *   prenom_render_fwd  hash encoding + MLP + volume rendering   Sec. III-B, Eq. (7)
 *                      + losses                                 Eq. (8)-(9)
 *   prenom_render_bwd  the adjoint of render_fwd (parameter gradients)
 *   prenom_adam_step   Adam on every parameter                  Sec. III-B, last paragraph
 *
 * Conventions for every call
 *   - Array arguments are DEVICE pointers owned by the caller.  The library
 *     never allocates, frees or synchronises inside these calls; each call only
 *     enqueues kernels on `stream` (a hipStream_t; NULL = the null stream) and
 *     returns.  Structs are passed by HOST pointer and read before return.
 *   - Arguments are validated on the host before anything is launched; on any
 *     error status nothing is enqueued.  Launch failures return
 *     PRENOM_ERR_HIP.  prenom_last_error() gives a message for the calling
 *     thread's last non-OK status.  No call aborts or exits.
 *   - Layouts are row-major and densely packed.  FP32 unless stated.
 *   - Thread safety: calls on different streams with disjoint outputs and
 *     workspaces may run concurrently.
 */
#ifndef PRENOM_H
#define PRENOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PRENOM_MAX_LEVELS 32
#define PRENOM_N_OUT 4 /* head outputs: density logit + 3 colour logits */

typedef enum prenom_status {
    PRENOM_OK = 0,
    PRENOM_ERR_INVALID_ARG = 1, /* NULL where required, out-of-range scalar */
    PRENOM_ERR_SHAPE = 2,       /* sizes inconsistent with each other       */
    PRENOM_ERR_UNSUPPORTED = 3, /* architecture not compiled into the lib   */
    PRENOM_ERR_WORKSPACE = 4,   /* workspace smaller than required          */
    PRENOM_ERR_HIP = 5          /* a HIP launch failed                      */
} prenom_status;

/* Element types of the reduced-precision forms. */
typedef enum prenom_dtype { PRENOM_F32 = 0, PRENOM_BF16 = 1, PRENOM_F16 = 2 } prenom_dtype;

/* Per-ray flags written by prenom_sample. */
enum {
    PRENOM_FLAG_MISS = 1,    /* ray does not meet the object box: no samples  */
    PRENOM_FLAG_ESCAPED = 2, /* prior mass below epsilon: uniform draws       */
    PRENOM_FLAG_UNIFORM = 4  /* no prior used (uniform mode or no prior grid) */
};

/* Architecture alpha (Sec. III and III-A): a multi-resolution hash grid with
 * n_levels levels of 2^log2_table entries of n_features features each, and a
 * bias-free MLP: mlp_hidden ReLU layers of width mlp_width, then a linear
 * 4-output head (density = exp(o0), colour = sigmoid(o1..3)).
 * resolution[l] is the lattice resolution N_l of level l (the caller computes
 * floor(N_min * b^l)).  A level is stored 1:1 when (N_l+1)^3 <= 2^log2_table,
 * and through the XOR-of-primes spatial hash otherwise.
 * mlp_dtype: element type of the MLP matrix products (PRENOM_F32, or
 * PRENOM_BF16 / PRENOM_F16 operands with FP32 accumulation; weights stay FP32
 * masters).  table_dtype: PRENOM_F32, or PRENOM_F16 when the forward gathers
 * read the FP16 copy model->table_lp (gradients accumulate in FP32 always).
 * Supported: n_features = 2; n_levels in {8, 12, 16}; mlp_width in {32, 64, 128};
 * mlp_hidden in {1, 2}; log2_table in [10, 24]; 2 <= N_l < 2^20. */
typedef struct prenom_arch {
    int32_t n_levels;
    int32_t log2_table;
    int32_t n_features;
    int32_t resolution[PRENOM_MAX_LEVELS];
    int32_t mlp_width;
    int32_t mlp_hidden;
    int32_t mlp_dtype;
    int32_t table_dtype;
} prenom_arch;

/* One object's NeRF.  Four device arrays of prenom_param_count(&arch) floats:
 * parameters, their gradients (accumulated with += by prenom_render_bwd,
 * zeroed by prenom_adam_step after use; the caller zeroes them once at
 * allocation), and Adam's first and second moments.
 * Parameter layout: hash tables [L][T][F], then W_1 [W][L*F],
 * W_2..W_D [W][W], W_out [4][W].
 * table_lp: FP16 copy of the tables ([L][T][F] halves), required when
 *   arch.table_dtype == PRENOM_F16; prenom_adam_step keeps it in step with the
 *   masters and prenom_refresh_lowp (re)writes it.
 * loss_scale: device scalar multiplying the upstream gradient inside
 *   render_bwd (NULL = 1).  scaler_state: device int32[2] = {non-finite
 *   gradient seen, finite steps since the scale last changed}, required with
 *   loss_scale, zeroed by the caller once.  With them prenom_adam_step
 *   unscales the gradient, skips the update when any entry is not finite and
 *   halves the scale, and doubles it after growth_interval finite steps. */
typedef struct prenom_model {
    prenom_arch arch;
    float* params;
    float* grads;
    float* adam_m;
    float* adam_v;
    void* table_lp;
    float* loss_scale;
    int32_t* scaler_state;
} prenom_model;

int64_t prenom_param_count(const prenom_arch* arch);       /* -1 if invalid */
int64_t prenom_table_param_count(const prenom_arch* arch); /* L * T * F   */

/* ------------------------------------------------------------------------
 * prenom_sample -- Sec. III-B "Probabilistic Ray Sampling", Eq. (4)-(6).
 *
 * Each world ray (rays_o, rays_d: [n_rays][3], unit direction) is moved into
 * the object frame with world_to_obj (row-major 3x4 affine onto NOCS [0,1]^3),
 * clipped to the unit box and [near_t, far_t].  n_coarse points at the bin
 * midpoints give sigma_i = F(x_i) (trilinear, vertex-aligned: F[i] at
 * i/(R-1)), delta_i = bin length in NOCS units, the termination mass of
 * Eq. (5) and the CDF of Eq. (6).  n_fine stratified draws
 * u_k = (k + xi_k)/n_fine (xi: [n_rays][n_fine], each in (0,1)) are inverted:
 * bin b_k = first i with CDF_{i+1} >= u_k, linear inside the bin.  A ray whose
 * total mass 1 - exp(-sum sigma delta) is below eps escapes to the uniform
 * draws t_k = t_n + u_k (t_f - t_n) (Sec. III-B, escape rule).  The whole
 * decision chain runs in FP64, so bins do not depend on FP32 rounding.
 *
 * Outputs (S = n_fine + (include_coarse ? n_coarse : 0)):
 *   ray_obj [n_rays][6]  object-frame origin and direction (FP32)
 *   t       [n_rays][S]  sorted sample distances (world units along the ray)
 *   dt      [n_rays][S]  delta_j = (t_{j+1} - t_j) |d_obj|, last: (t_f - t_S-1)|d_obj|
 *   bins    [n_rays][n_fine]  int32 CDF bin of each draw, -1 when uniform
 *   flags   [n_rays]     uint8 PRENOM_FLAG_*; missed rays get t = dt = 0
 * prior: device [R][R][R] (x fastest), R >= 2, or NULL (uniform draws).
 * n_coarse in [1, 256] unless uniform_only; n_fine in [1, 256].
 * ---------------------------------------------------------------------- */
typedef struct prenom_sample_cfg {
    int32_t n_coarse;
    int32_t n_fine;
    int32_t include_coarse; /* also render the n_coarse midpoints (sorted merge) */
    int32_t uniform_only;   /* ignore the prior: stratified uniform draws        */
    float eps;              /* escape threshold                                  */
    float near_t, far_t;
    float world_to_obj[12];
    const float* prior;
    int32_t prior_res;
} prenom_sample_cfg;

prenom_status prenom_sample(const prenom_sample_cfg* cfg, const float* rays_o, const float* rays_d,
                            const float* xi, int64_t n_rays, float* ray_obj, float* t, float* dt,
                            int32_t* bins, uint8_t* flags, void* stream);

/* ------------------------------------------------------------------------
 * Rendering configuration.  loss_mode 0: mean squared errors,
 *   L = 1/(3n) sum_k |C^_k - C_k|^2 + lambda_d/n sum_{mask} (D^_k - D_k)^2
 *       + lambda_sigma/n sum_{!mask} sum_j sigma_kj
 * loss_mode 1: the norms of Eq. (8) combined by Eq. (9),
 *   L = sum_k |C^_k - C_k|_2 + lambda_d sum_{mask} |D^_k - D_k|
 *       + lambda_sigma sum_{!mask} sum_j |sigma_kj|
 * where C_k is tgt_rgb (for background rays: the background colour, the
 * random colour of Eq. (8)).
 * ---------------------------------------------------------------------- */
typedef struct prenom_render_cfg {
    int32_t n_samples; /* S, 1..256 */
    int32_t loss_mode;
    float lambda_d;
    float lambda_sigma;
    int32_t recompute; /* 0: render_bwd reads what render_fwd stored in the workspace
                          (per-sample features, head outputs, per-ray results);
                          1: both calls run pass by pass over chunks of about 2^21
                          samples and render_bwd recomputes each pass's features,
                          head outputs and per-ray results, so the workspace holds
                          one pass (not the batch) and need not survive between
                          the two calls (activations are not kept) */
} prenom_render_cfg;

/* Bytes of device workspace render_fwd/render_bwd need for this batch, in the
 * stored (recompute = 0) or the recompute (1) form; 0 on invalid input. */
size_t prenom_workspace_size(const prenom_arch* arch, int64_t n_rays, int32_t n_samples, int32_t recompute);

/* ------------------------------------------------------------------------
 * prenom_render_fwd -- Sec. III-B "Volume Rendering", Eq. (7)-(9).
 *
 * Sample positions x_j = clamp(fmaf(t_j, d, o), 0, 1) (o, d from ray_obj) are
 * hash-encoded (Mueller et al. 2022, used in Sec. III-B "Object-level
 * NeRFs"), fed through the MLP, and composited:
 *   alpha_j = 1 - exp(-sigma_j delta_j), T_j = exp(-sum_{i<j} sigma_i delta_i),
 *   rgb = sum_j T_j alpha_j c_j + T_S bg, depth = sum_j T_j alpha_j t_j,
 *   opacity = sum_j T_j alpha_j.
 * Missed rays (flags & MISS) give rgb = bg, depth = opacity = 0.
 * Inputs: ray_obj [n][6], t, dt [n][S], flags [n] as from prenom_sample;
 *   bg [n][3] or NULL (black); targets tgt_rgb [n][3], tgt_depth [n],
 *   mask [n] (uint8, 1 = object ray) may all be NULL (no loss).
 * Outputs: rgb [n][3], depth [n], opacity [n]; loss [1] (device scalar, or
 *   NULL); sample_out [n][S][4] = (sigma, r, g, b) per sample, or NULL.
 * workspace: >= prenom_workspace_size(arch, n, S, cfg->recompute) bytes,
 *   256-byte aligned.  In the stored form it also
 *   receives the per-tile histograms of the hash-table gradient's records
 *   (per level and block of 512 samples: one per corner of every sample,
 *   a corner that repeats the previous sample's row joining its record)
 *   that the backward's table-gradient scatter starts from.  Unless cfg->recompute is set, it
 *   carries the per-sample features and per-ray results that
 *   prenom_render_bwd reads: pass the same workspace and unchanged inputs to
 *   the matching bwd call.
 * ---------------------------------------------------------------------- */
prenom_status prenom_render_fwd(const prenom_model* model, const prenom_render_cfg* cfg,
                                const float* ray_obj, const float* t, const float* dt,
                                const uint8_t* flags, int64_t n_rays, const float* bg,
                                const float* tgt_rgb, const float* tgt_depth, const uint8_t* mask,
                                float* rgb, float* depth, float* opacity, float* loss,
                                float* sample_out, void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * prenom_render_bwd -- gradient of the rendering path (Sec. III-B, last
 * paragraph: the loss of Eq. (9) is back-propagated to the NeRF parameters).
 * Adds dL/dparams to model->grads.  With d_rgb [n][3] given (d_depth [n]
 * and d_opacity [n] optional), the gradient is that of
 * sum(d_rgb*rgb + d_depth*depth + d_opacity*opacity), the vector-Jacobian
 * product an outer autograd needs; with d_rgb == NULL it is the gradient of
 * the fused loss of render_fwd (targets required).
 * Without cfg->recompute it must follow render_fwd on the same stream with the
 * same workspace and inputs; with it, only the inputs must match.  The
 * backward leaves what the forward wrote unchanged, so several backward calls
 * (for instance with different upstream gradients) may follow one forward.  A call
 * that breaks this gives a wrong gradient but stays within its arrays: the
 * scatter checks that the forward's histograms hold no more records than
 * there are corners of samples, else it adds nothing to the table gradient,
 * and every record it writes or reads is bounded by the workspace's record
 * arrays.
 * The table gradient is accumulated per 2^13-row tile in 64-bit fixed point
 * (order independent); tiles that receive more than 2^21 contributions are
 * split and their partial sums added with FP32 atomics, so only those may
 * differ in the last bits between runs.
 * ---------------------------------------------------------------------- */
prenom_status prenom_render_bwd(const prenom_model* model, const prenom_render_cfg* cfg,
                                const float* ray_obj, const float* t, const float* dt,
                                const uint8_t* flags, int64_t n_rays, const float* bg,
                                const float* tgt_rgb, const float* tgt_depth, const uint8_t* mask,
                                const float* d_rgb, const float* d_depth, const float* d_opacity,
                                void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * prenom_adam_step -- Adam (Sec. III-B, last paragraph) on every parameter:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps)
 * then zeroes the gradients.  step >= 1 is the 1-based iteration count.
 * ---------------------------------------------------------------------- */
typedef struct prenom_adam_cfg {
    float lr, beta1, beta2, eps;
    int64_t step;
    int32_t growth_interval; /* loss scaling: finite steps before the scale doubles (0 = never) */
} prenom_adam_cfg;

prenom_status prenom_adam_step(const prenom_model* model, const prenom_adam_cfg* cfg, void* stream);

/* Rewrites model->table_lp (FP16) from the FP32 tables, rounding to nearest. */
prenom_status prenom_refresh_lowp(const prenom_model* model, void* stream);

/* ------------------------------------------------------------------------
 * prenom_prior_refresh -- the prior density grid recomputed from the NeRF.
 * The category prior is the NeRF's density output over a cubic grid of
 * resolution R (Sec. III-A, "Normalized mesh generation"); during online
 * mapping it is recomputed from the object's current NeRF every m
 * iterations so that sampling converges on the object even from an
 * imprecise pose (Sec. III-B, "Probabilistic Ray Sampling"; m = 50 in
 * Sec. IV-A).
 * prior_out [R][R][R] (x fastest, the layout prenom_sample reads) receives
 *   sigma = exp(o_0) at the vertices (i, j, k) / (R - 1) of the object
 *   frame, each coordinate rounded from FP64 to FP32 like a sample position;
 *   the forward reads the FP16 table copy when table_dtype is FP16.
 * R in [2, PRENOM_MAX_PRIOR_RES]; workspace: >=
 *   prenom_prior_refresh_workspace_size(arch, R) bytes (0 for an invalid
 *   arch or R), 256-byte aligned, contents not preserved; the grid is
 *   processed in chunks of at most 2^21 vertices, so the workspace stays
 *   near (4 L F + 16) * 2^21 bytes (L levels, F features) whatever R is.  Errors:
 *   PRENOM_ERR_SHAPE (R), PRENOM_ERR_INVALID_ARG, PRENOM_ERR_WORKSPACE,
 *   PRENOM_ERR_UNSUPPORTED, checked before any launch.  Asynchronous on
 *   stream; model->grads is not touched.
 * ---------------------------------------------------------------------- */
#define PRENOM_MAX_PRIOR_RES 512
size_t prenom_prior_refresh_workspace_size(const prenom_arch* arch, int32_t R);
prenom_status prenom_prior_refresh(const prenom_model* model, int32_t R, float* prior_out, void* workspace,
                                   size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * prenom_prior_refresh_noalloc -- prenom_prior_refresh for callers that
 * cannot allocate device memory (code under HIP graph capture, tight mapping
 * loops, harnesses that forbid hipMalloc).  Same arguments, result and errors
 * as prenom_prior_refresh, without the workspace: the per-vertex features
 * and head outputs of each chunk live in a fixed array of
 * PRENOM_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends.  The grid is processed in chunks sized to that
 * array (any R in [2, PRENOM_MAX_PRIOR_RES]); an architecture whose features
 * of 1024 vertices do not fit returns PRENOM_ERR_WORKSPACE before any launch.
 * Nothing is allocated or freed: the array's device address is looked up
 * once per device, on the first call with that device current (make that
 * first call outside graph capture).  Every call on a GPU shares that GPU's
 * array, so calls that overlap on one GPU (different streams without
 * ordering) race; calls on one stream are ordered and safe.
 * ---------------------------------------------------------------------- */
#define PRENOM_NOALLOC_SCRATCH_BYTES (((size_t)16) << 20)
size_t prenom_noalloc_scratch_bytes(void);
prenom_status prenom_prior_refresh_noalloc(const prenom_model* model, int32_t R, float* prior_out, void* stream);

/* ------------------------------------------------------------------------
 * prenom_encode -- the hash encoding alone (Sec. III-B "Object-level NeRFs"):
 * pos [n][3] in [0,1]^3 -> features [L][n][F] (level-major); corner_idx
 * [L][n][8] (int32 table row of each cell corner, corner e = (e&1, e>>1&1,
 * e>>2&1)) or NULL.  table: [L][T][F], 16-byte aligned (rows are read in
 * aligned pairs); features 8-byte aligned; otherwise PRENOM_ERR_INVALID_ARG.
 * ---------------------------------------------------------------------- */
prenom_status prenom_encode(const prenom_arch* arch, const float* table, const float* pos, int64_t n,
                            float* features, int32_t* corner_idx, void* stream);

/* ------------------------------------------------------------------------
 * prenom_canonical_yaw -- the object's yaw in the category's canonical frame
 * (Sec. III-B, "Object State Canonicalization", Eq. (3)).  Objects stand on
 * the ground (z up), so only the yaw is searched: for each of the n_yaw
 * yaws gamma_k = 2 pi k / n_yaw the cloud is turned about z, P_k = Rz(gamma_k) P,
 * normalised into the unit cube by its extents,
 *   Pn = (P_k - C_k) / S_k + 1/2   (S_k = max - min, C_k = (max + min) / 2
 *                                   per axis; an axis with S_k = 0 maps to 1/2),
 * and scored by the sum over its points of the prior's trilinear density
 * (the lookup of prenom_sample).  best = the first k of largest score.
 *   points  [n_points][3] device FP32, in the object's frame (any origin).
 *   prior   [prior_res]^3 device FP32 density grid (x fastest).
 *   scores  [n_yaw], extents and centers [n_yaw][3]: device FP64 outputs.
 *   best    device int32.
 * FP64 arithmetic; sums in a fixed order (results do not depend on
 * scheduling).  1 <= n_points <= PRENOM_MAX_YAW_POINTS, 1 <= n_yaw <=
 * PRENOM_MAX_YAWS, 2 <= prior_res <= PRENOM_MAX_PRIOR_RES; workspace: >=
 * prenom_canonical_yaw_workspace_size bytes (0 for invalid sizes), 256-byte
 * aligned.  Errors: PRENOM_ERR_SHAPE, PRENOM_ERR_INVALID_ARG,
 * PRENOM_ERR_WORKSPACE, checked before any launch.
 * ---------------------------------------------------------------------- */
#define PRENOM_MAX_YAWS 4096
#define PRENOM_MAX_YAW_POINTS (((int64_t)1) << 28)
size_t prenom_canonical_yaw_workspace_size(int64_t n_points, int32_t n_yaw);
prenom_status prenom_canonical_yaw(const float* points, int64_t n_points, const float* prior, int32_t prior_res,
                                   int32_t n_yaw, double* scores, double* extents, double* centers, int32_t* best,
                                   void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Batched training of many objects (Fig. 1 and Sec. IV-A: every object NeRF
 * of the map trains concurrently, each with its own category architecture
 * alpha, prior and pose).  Where the method gives each object its own host
 * thread, a batch runs the step of all its objects with one launch per
 * phase (the MLP: one launch per distinct MLP shape), so objects with few
 * rays share the GPU with large ones.  The arithmetic of every object is that
 * of the single-object calls above, with the loss of each object averaged
 * over its own rays; the optimisation of each object is independent.
 *
 * Rays of the batch are the objects' rays in object order: object i owns
 * rays [sum_{j<i} n_rays_j, sum_{j<=i} n_rays_j) of every per-ray array.
 * Parameters of the batch are one device array per kind (params, grads,
 * adam_m, adam_v) of prenom_batch_param_count floats; object i's parameters
 * (layout as in prenom_model) start at prenom_batch_param_offset(i), a
 * multiple of 64 floats.
 * ---------------------------------------------------------------------- */

/* Per-object part of a batch. */
typedef struct prenom_object {
    prenom_arch arch;
    int64_t n_rays;          /* rays of this object in the batch (>= 0)              */
    const float* prior;      /* device [R^3] prior grid of prenom_sample, or NULL:   */
    int32_t prior_res;       /*   uniform sampling for this object                   */
    float world_to_obj[12];  /* row-major 3x4 world -> NOCS affine, as in prenom_sample */
} prenom_object;

/* Tile shape of the batched MLP launches for one MLP shape (chosen by an
 * autotuner; shapes without an entry use defaults).  fwd_tiles: 16-sample
 * tiles per forward block, a multiple of 4 in [4, 4096]; bwd_tiles: per
 * backward block (each writes one partial weight gradient and the maxima of
 * |dy| of its 512-sample blocks, which the table gradient's fixed-point scale
 * needs), a multiple of 32 in [32, 1024]. */
typedef struct prenom_mlp_tiles {
    int32_t in_dim, width, hidden, dtype;
    int32_t fwd_tiles, bwd_tiles;
} prenom_mlp_tiles;

/* A batch: host arrays `objects` and `tiles` are read during each call.
 * params_lp: device FP16 copy of the whole parameter array, required when an
 *   object has table_dtype PRENOM_F16 (prenom_batch_adam_step keeps it in step).
 * loss_scale / scaler_state: as in prenom_model, shared by the batch (a
 *   non-finite gradient anywhere skips the update of every object).
 * step: device int64 Adam step counter or NULL.  With it the bias corrections
 *   use *step + 1 and the counter advances on the device after each applied
 *   update, so a captured step graph can be replayed without host arguments
 *   (the caller zeroes it once).
 * record_budget: bytes of hash-table gradient records one scatter pass may
 *   hold, 0 for PRENOM_RECORD_BUDGET.  The backward's scatter (Eq. (3)'s
 *   table gradient) runs over groups of consecutive whole objects whose
 *   worst-case records (64 bytes per sample and level) fit the budget; an
 *   object above it is a group of its own.  The workspace holds the largest
 *   group's records, so a smaller budget trades a smaller workspace for more
 *   launches (six per group); the gradients do not depend on the grouping. */
#define PRENOM_RECORD_BUDGET ((int64_t)4 << 30)
typedef struct prenom_batch {
    int32_t n_objects;
    const prenom_object* objects;
    int32_t n_tiles;
    const prenom_mlp_tiles* tiles;
    float* params;
    float* grads;
    float* adam_m;
    float* adam_v;
    void* params_lp;
    float* loss_scale;
    int32_t* scaler_state;
    int64_t* step;
    int64_t record_budget;
} prenom_batch;

#define PRENOM_MAX_OBJECTS 4096

/* Floats of each parameter array of the batch, and object i's first one
 * (-1 on invalid input). */
int64_t prenom_batch_param_count(const prenom_object* objects, int32_t n_objects);
int64_t prenom_batch_param_offset(const prenom_object* objects, int32_t n_objects, int32_t i);

/* Workspace bytes of the batched calls for n_samples samples per ray (0 on
 * invalid input).  The workspace holds the batch's device descriptors and
 * every intermediate of the step. */
size_t prenom_batch_workspace_size(const prenom_batch* batch, int32_t n_samples);

/* Writes the batch's device descriptors into the workspace (copies from host
 * memory, then waits for `stream`).  Every other batched call checks that the
 * workspace was prepared for the same objects, tile shapes and n_samples and
 * fails with PRENOM_ERR_WORKSPACE otherwise.  Call it again whenever the
 * objects change (new ray counts, priors or poses). */
prenom_status prenom_batch_prepare(const prenom_batch* batch, int32_t n_samples, void* workspace, size_t ws_bytes,
                                   void* stream);

/* prenom_sample for every object at once: cfg's sampling counts, eps and
 * near/far apply to all objects; its prior, prior_res and world_to_obj are
 * ignored (each object supplies its own; uniform_only forces uniform draws
 * for all).  Arrays as in prenom_sample over all rays of the batch. */
prenom_status prenom_batch_sample(const prenom_batch* batch, const prenom_sample_cfg* cfg, const float* rays_o,
                                  const float* rays_d, const float* xi, float* ray_obj, float* t, float* dt,
                                  int32_t* bins, uint8_t* flags, void* workspace, size_t ws_bytes, void* stream);

/* prenom_render_fwd for every object at once.  loss: device float[n_objects]
 * (object i's loss of Eq. (8)/(9), averaged over its rays) or NULL. */
prenom_status prenom_batch_render_fwd(const prenom_batch* batch, const prenom_render_cfg* cfg, const float* ray_obj,
                                      const float* t, const float* dt, const uint8_t* flags, const float* bg,
                                      const float* tgt_rgb, const float* tgt_depth, const uint8_t* mask, float* rgb,
                                      float* depth, float* opacity, float* loss, void* workspace, size_t ws_bytes,
                                      void* stream);

/* prenom_render_bwd for every object at once: accumulates every object's
 * gradient of its own loss (or of the upstream d_rgb / d_depth / d_opacity)
 * into batch->grads. */
prenom_status prenom_batch_render_bwd(const prenom_batch* batch, const prenom_render_cfg* cfg, const float* ray_obj,
                                      const float* t, const float* dt, const uint8_t* flags, const float* bg,
                                      const float* tgt_rgb, const float* tgt_depth, const uint8_t* mask,
                                      const float* d_rgb, const float* d_depth, const float* d_opacity,
                                      void* workspace, size_t ws_bytes, void* stream);

/* prenom_adam_step over the whole parameter array of the batch (one launch).
 * With batch->step set, cfg->step is ignored. */
prenom_status prenom_batch_adam_step(const prenom_batch* batch, const prenom_adam_cfg* cfg, void* stream);

/* Rewrites batch->params_lp (FP16, every parameter) from batch->params. */
prenom_status prenom_batch_refresh_lowp(const prenom_batch* batch, void* stream);

/* ------------------------------------------------------------------------
 * Meta-learning of the initial parameters (Sec. III-A, "Meta-learning",
 * Eq. (1)-(2), Reptile).  A task is one object instance of a category,
 * trained from the meta-parameters theta for q inner iterations of plain
 * gradient descent (Eq. (1)); theta then moves towards the result (Eq. (2)).
 * Tasks trained from the same theta can run together as the objects of one
 * batch; the outer update then takes the mean of their differences.
 * ---------------------------------------------------------------------- */
typedef struct prenom_sgd_cfg {
    float lr;                /* eta of Eq. (1), finite, >= 0 */
    int32_t growth_interval; /* loss scaling as in prenom_adam_cfg */
} prenom_sgd_cfg;

/* Eq. (1): params -= lr * grads (unscaled by *loss_scale when the model has
 * one; the whole update skipped after a non-finite gradient), then zeroes
 * the gradients; rewrites the FP16 table copy when table_dtype is FP16.  No
 * moments are read or written.  Errors as prenom_adam_step. */
prenom_status prenom_sgd_step(const prenom_model* model, const prenom_sgd_cfg* cfg, void* stream);

/* prenom_sgd_step over the whole parameter array of a batch; batch->step,
 * when set, counts the applied steps; adam_m / adam_v are not used. */
prenom_status prenom_batch_sgd_step(const prenom_batch* batch, const prenom_sgd_cfg* cfg, void* stream);

/* Eq. (2) over n_tasks >= 1 tasks trained from theta:
 *   theta += beta * (1 / n_tasks) * sum_b (task_b - theta)
 * (n_tasks = 1: theta + beta (theta^(q) - theta), Eq. (2) itself), then
 * every task slot is reset to the new theta for the next meta-iteration:
 * task_b <- theta; its FP16 copy's first n_lp entries <- theta rounded to
 * nearest (tasks_lp, or NULL); its Adam moments <- 0 (adam_m and adam_v,
 * both or neither); *step <- 0 (a device step counter, or NULL).
 *   theta   [n_params] device FP32, 16-byte aligned; must not overlap a task.
 *   tasks   device FP32, task b at tasks + b * task_stride, 16-byte aligned;
 *           task_stride >= n_params and a multiple of 4 (the batch layout
 *           of prenom_batch_param_offset when every object has the same
 *           architecture).
 *   adam_m, adam_v: in the task layout, 16-byte aligned.
 *   tasks_lp: FP16 in the task layout (in halves), 8-byte aligned;
 *           0 <= n_lp <= n_params.
 * n_tasks in [1, PRENOM_MAX_OBJECTS]; beta finite.  Errors: PRENOM_ERR_SHAPE,
 * PRENOM_ERR_INVALID_ARG, checked before any launch.  One launch; tasks
 * are read and written in place, so calls on the same tasks must not
 * overlap. */
prenom_status prenom_reptile_update(float* theta, float* tasks, int64_t n_params, int32_t n_tasks,
                                    int64_t task_stride, float beta, float* adam_m, float* adam_v, void* tasks_lp,
                                    int64_t n_lp, int64_t* step, void* stream);

/* ------------------------------------------------------------------------
 * Kernel timing (instrumentation, not part of the method).  Between
 * prenom_profile_begin() and prenom_profile_end(), every kernel the library
 * launches is bracketed by a pair of HIP events on its stream.
 * prenom_profile_end waits for those events and returns, per kernel name,
 * the number of launches and their summed duration in milliseconds
 * (up to `capacity` entries; *n_kernels receives the number written).
 * The events are created on first use and reused; nothing else allocates.
 * ---------------------------------------------------------------------- */
typedef struct prenom_kernel_time {
    char name[48];
    int64_t launches;
    double total_ms;
} prenom_kernel_time;

prenom_status prenom_profile_begin(void);
prenom_status prenom_profile_end(prenom_kernel_time* out, int32_t capacity, int32_t* n_kernels);

const char* prenom_status_string(prenom_status s);
const char* prenom_last_error(void);
const char* prenom_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PRENOM_H */

// C ABI of libprenom: argument validation, workspace layout and the launch
// sequence of each call.  Host code only; every kernel lives in its own unit.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "api_util.h"
#include "common.h"

namespace prenom {
namespace host {

namespace {
thread_local char g_last_error[512] = "";

struct ProfRecord {
    const char* name;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRecord> g_prof_records;
std::vector<hipEvent_t> g_event_pool;
size_t g_pool_used = 0;

hipEvent_t pool_event()
{
    if (g_pool_used == g_event_pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        g_event_pool.push_back(e);
    }
    return g_event_pool[g_pool_used++];
}
}  // namespace

prenom_status fail(prenom_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return st;
}

prenom_status hip_status(hipError_t e, const char* what)
{
    if (e == hipSuccess) return PRENOM_OK;
    return fail(PRENOM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

const char* last_error() { return g_last_error; }

bool prof_events(hipEvent_t* a, hipEvent_t* b)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return false;
    *a = pool_event();
    *b = pool_event();
    return *a && *b;
}

void prof_record(const char* name, hipEvent_t a, hipEvent_t b)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_records.push_back({name, a, b});
}

// Compute units of the current device (persistent grids size to it).
int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 256;
    return cus;
}

// Shape rules an architecture must satisfy (independent of what is compiled).
prenom_status check_arch(const prenom_arch* a)
{
    if (!a) return fail(PRENOM_ERR_INVALID_ARG, "arch is NULL");
    if (a->n_levels < 1 || a->n_levels > PRENOM_MAX_LEVELS)
        return fail(PRENOM_ERR_INVALID_ARG, "n_levels %d outside [1, %d]", a->n_levels, PRENOM_MAX_LEVELS);
    if (a->log2_table < 10 || a->log2_table > 24)
        return fail(PRENOM_ERR_INVALID_ARG, "log2_table %d outside [10, 24]", a->log2_table);
    if (a->n_features != 2) return fail(PRENOM_ERR_UNSUPPORTED, "n_features %d (only 2)", a->n_features);
    for (int l = 0; l < a->n_levels; ++l)
        if (a->resolution[l] < 2 || a->resolution[l] >= (1 << 20))
            return fail(PRENOM_ERR_INVALID_ARG, "resolution[%d] = %d outside [2, 2^20)", l, a->resolution[l]);
    if (a->mlp_width < 16 || a->mlp_width % 16 || a->mlp_hidden < 1 || a->mlp_hidden > 4)
        return fail(PRENOM_ERR_INVALID_ARG, "mlp %d x %d", a->mlp_width, a->mlp_hidden);
    if (a->mlp_dtype != PRENOM_F32 && a->mlp_dtype != PRENOM_BF16 && a->mlp_dtype != PRENOM_F16)
        return fail(PRENOM_ERR_INVALID_ARG, "mlp_dtype %d", a->mlp_dtype);
    if (a->table_dtype != PRENOM_F32 && a->table_dtype != PRENOM_F16)
        return fail(PRENOM_ERR_INVALID_ARG, "table_dtype %d (FP32 or FP16)", a->table_dtype);
    return PRENOM_OK;
}

MlpShape mlp_shape(const prenom_arch* a)
{
    return MlpShape{a->n_levels * a->n_features, a->mlp_width, a->mlp_hidden, a->mlp_dtype};
}

hipError_t mlp_fwd_any(const MlpShape& m, const float* w, const float* y, int64_t n_s, float* sc, float* act,
                       hipStream_t s)
{
    return m.dtype == PRENOM_F32 ? launch_mlp_fwd(m, w, y, n_s, sc, act, s) : launch_mlp_fwd_lp(m, w, y, n_s, sc, act, s);
}

hipError_t mlp_bwd_any(const MlpShape& m, const float* w, const float* y, const float* dout, const float* sc,
                       int64_t n_s, float* dy, float* partial, float* act, hipStream_t s)
{
    return m.dtype == PRENOM_F32 ? launch_mlp_bwd(m, w, y, dout, sc, n_s, dy, partial, act, s)
                                 : launch_mlp_bwd_lp(m, w, y, dout, sc, n_s, dy, partial, act, s);
}

prenom_status check_supported(const prenom_arch* a)
{
    const prenom_status st = check_arch(a);
    if (st != PRENOM_OK) return st;
    const MlpShape m = mlp_shape(a);
    if (!mlp_supported(m))
        return fail(PRENOM_ERR_UNSUPPORTED, "MLP in=%d width=%d hidden=%d is not compiled into this library",
                    m.in_dim, m.width, m.hidden);
    return PRENOM_OK;
}

int64_t table_params(const prenom_arch* a) { return ((int64_t)a->n_levels << a->log2_table) * a->n_features; }

int64_t mlp_params(const prenom_arch* a)
{
    const int64_t in = (int64_t)a->n_levels * a->n_features, W = a->mlp_width;
    return W * in + (int64_t)(a->mlp_hidden - 1) * W * W + (int64_t)PRENOM_N_OUT * W;
}

GridInfo grid_info(const prenom_arch* a)
{
    GridInfo g{};
    g.n_levels = a->n_levels;
    g.log2_table = a->log2_table;
    g.dense_mask = 0;
    const int64_t T = (int64_t)1 << a->log2_table;
    for (int l = 0; l < a->n_levels; ++l) {
        g.res[l] = a->resolution[l];
        const int64_t side = (int64_t)a->resolution[l] + 1;
        if (side * side * side <= T) g.dense_mask |= 1u << l;
    }
    return g;
}

prenom_status check_sample_cfg(const prenom_sample_cfg* cfg, bool need_prior_fields)
{
    if (!cfg) return fail(PRENOM_ERR_INVALID_ARG, "cfg is NULL");
    if (cfg->n_fine < 1 || cfg->n_fine > 256) return fail(PRENOM_ERR_SHAPE, "n_fine %d outside [1, 256]", cfg->n_fine);
    if (cfg->n_coarse < 0 || cfg->n_coarse > 256) return fail(PRENOM_ERR_SHAPE, "n_coarse %d outside [0, 256]", cfg->n_coarse);
    const bool use_prior = need_prior_fields ? (!cfg->uniform_only && cfg->prior != nullptr) : !cfg->uniform_only;
    if ((use_prior || cfg->include_coarse) && cfg->n_coarse < 1)
        return fail(PRENOM_ERR_SHAPE, "n_coarse must be >= 1 with a prior or include_coarse");
    if (need_prior_fields && use_prior && cfg->prior_res < 2) return fail(PRENOM_ERR_SHAPE, "prior_res %d < 2", cfg->prior_res);
    if (!(cfg->eps >= 0.0f)) return fail(PRENOM_ERR_INVALID_ARG, "eps must be >= 0");
    if (!(cfg->near_t <= cfg->far_t)) return fail(PRENOM_ERR_INVALID_ARG, "near_t > far_t");
    if (need_prior_fields)
        for (int i = 0; i < 12; ++i)
            if (!std::isfinite(cfg->world_to_obj[i])) return fail(PRENOM_ERR_INVALID_ARG, "world_to_obj not finite");
    return PRENOM_OK;
}

prenom_status check_render_cfg(const prenom_render_cfg* cfg)
{
    if (!cfg) return fail(PRENOM_ERR_INVALID_ARG, "cfg is NULL");
    if (cfg->n_samples < 1 || cfg->n_samples > 256)
        return fail(PRENOM_ERR_SHAPE, "n_samples %d outside [1, 256]", cfg->n_samples);
    if (cfg->loss_mode != 0 && cfg->loss_mode != 1) return fail(PRENOM_ERR_INVALID_ARG, "loss_mode %d", cfg->loss_mode);
    if (cfg->recompute != 0 && cfg->recompute != 1) return fail(PRENOM_ERR_INVALID_ARG, "recompute %d", cfg->recompute);
    if (!(cfg->lambda_d >= 0.0f) || !(cfg->lambda_sigma >= 0.0f))
        return fail(PRENOM_ERR_INVALID_ARG, "negative or NaN loss weight");
    return PRENOM_OK;
}

prenom_status check_model(const prenom_model* m, bool need_grads)
{
    if (!m) return fail(PRENOM_ERR_INVALID_ARG, "model is NULL");
    const prenom_status st = check_supported(&m->arch);
    if (st != PRENOM_OK) return st;
    if (!m->params || !aligned(m->params, 16)) return fail(PRENOM_ERR_INVALID_ARG, "params NULL or not 16-byte aligned");
    if (need_grads && (!m->grads || !aligned(m->grads, 16)))
        return fail(PRENOM_ERR_INVALID_ARG, "grads NULL or not 16-byte aligned");
    if (m->arch.table_dtype == PRENOM_F16 && (!m->table_lp || !aligned(m->table_lp, 8)))
        return fail(PRENOM_ERR_INVALID_ARG, "table_dtype FP16 needs an 8-byte aligned table_lp");
    if (m->loss_scale && !m->scaler_state) return fail(PRENOM_ERR_INVALID_ARG, "loss_scale needs scaler_state");
    return PRENOM_OK;
}

prenom_status prior_refresh_chunks(const prenom_model* model, int32_t R, float* prior_out, float* y, float* sc,
                                   int64_t chunk, hipStream_t s)
{
    const prenom_arch* a = &model->arch;
    const int64_t n = (int64_t)R * R * R;
    const void* tlp = a->table_dtype == PRENOM_F16 ? model->table_lp : nullptr;
    for (int64_t p0 = 0; p0 < n; p0 += chunk) {
        const int64_t cnt = n - p0 < chunk ? n - p0 : chunk;
        PRENOM_LAUNCH("k_encode_grid", s, launch_encode_grid(grid_info(a), model->params, tlp, R, p0, cnt, y, s));
        PRENOM_LAUNCH("k_mlp_fwd", s,
                      mlp_fwd_any(mlp_shape(a), model->params + table_params(a), y, cnt, sc, nullptr, s));
        PRENOM_LAUNCH("k_density_grid", s, launch_density_grid(sc, cnt, prior_out + p0, s));
    }
    return PRENOM_OK;
}

}  // namespace host
}  // namespace prenom

namespace {

using namespace prenom;
using namespace prenom::host;


struct WsLayout {
    size_t y, sc, dout, dy, ray_state, loss_partial, mlp_partial, act;
    size_t counts, offsets, block_max, level_max, tile_exp, tile_total, tile_start, chunk_start, work_counter, recs, total;
    int n_loss_blocks, n_mlp_slots;
    ScatterObj plan;
};

// Rays per pass of the recompute form: about 2^21 samples, a multiple of the
// compositing kernels' rays per block (so each pass's loss partials continue
// those of the pass before).
constexpr int64_t kRecomputeSamples = int64_t(1) << 21;

int64_t recompute_chunk_rays(int32_t S)
{
    const int64_t rpb = composite_rays_per_block();
    const int64_t c = kRecomputeSamples / S / rpb * rpb;
    return c < rpb ? rpb : c;
}

// Rays whose per-sample buffers the workspace holds at once: all of them, or
// one pass of the recompute form.
int64_t buffered_rays(int64_t n_rays, int32_t S, bool recompute)
{
    if (!recompute) return n_rays;
    const int64_t c = recompute_chunk_rays(S);
    return n_rays < c ? n_rays : c;
}

WsLayout ws_layout(const prenom_arch* a, int64_t n_rays_all, int32_t S, bool recompute)
{
    WsLayout w{};
    const int64_t n_rays = buffered_rays(n_rays_all, S, recompute);
    const size_t n_s = (size_t)n_rays * (size_t)S, L = (size_t)a->n_levels;
    size_t off = 0;
    w.y = off;
    off = align_up(off + L * n_s * 2 * sizeof(float));
    w.sc = off;
    off = align_up(off + n_s * 4 * sizeof(float));
    w.dout = off;
    off = align_up(off + n_s * 4 * sizeof(float));
    w.dy = off;
    off = align_up(off + L * n_s * 2 * sizeof(float));
    w.ray_state = off;
    off = align_up(off + (size_t)n_rays * 8 * sizeof(float));
    w.n_loss_blocks = composite_loss_blocks(n_rays_all);
    w.loss_partial = off;
    off = align_up(off + (size_t)(w.n_loss_blocks > 0 ? w.n_loss_blocks : 1) * sizeof(double));
    w.n_mlp_slots = mlp_bwd_waves((int64_t)n_s);
    w.mlp_partial = off;
    off = align_up(off + (size_t)w.n_mlp_slots * (size_t)mlp_params(a) * sizeof(float));
    w.act = off;
    off = align_up(off + (size_t)mlp_act_floats(mlp_shape(a), (int64_t)n_s) * sizeof(float));
    w.plan = scatter_obj(grid_info(a), (int64_t)n_s);
    const size_t nt = (size_t)w.plan.n_tiles;
    w.counts = off;
    off = align_up(off + nt * (size_t)w.plan.n_blocks * sizeof(uint32_t));
    w.offsets = off;
    off = align_up(off + nt * (size_t)w.plan.n_blocks * sizeof(uint32_t));
    w.block_max = off;
    off = align_up(off + (size_t)a->n_levels * (size_t)w.plan.n_blocks * sizeof(float));
    w.level_max = off;
    off = align_up(off + (size_t)a->n_levels * sizeof(float));
    w.tile_exp = off;
    off = align_up(off + nt * sizeof(int32_t));
    w.tile_total = off;
    off = align_up(off + nt * sizeof(uint64_t));
    w.tile_start = off;
    off = align_up(off + (nt + 1) * sizeof(uint64_t));
    w.chunk_start = off;
    off = align_up(off + (nt + 2) * sizeof(uint64_t));
    w.work_counter = off;
    off = align_up(off + sizeof(uint64_t));
    w.recs = off;
    off = align_up(off + (size_t)scatter_records(w.plan) * sizeof(uint64_t));
    w.total = off;
    return w;
}


prenom_status check_render(const prenom_model* model, const prenom_render_cfg* cfg, const float* ray_obj,
                           const float* t, const float* dt, const uint8_t* flags, int64_t n_rays, void* ws,
                           size_t ws_bytes, bool need_grads)
{
    prenom_status st = check_model(model, need_grads);
    if (st != PRENOM_OK) return st;
    st = check_render_cfg(cfg);
    if (st != PRENOM_OK) return st;
    if (n_rays < 0) return fail(PRENOM_ERR_SHAPE, "n_rays < 0");
    if ((double)n_rays * cfg->n_samples > 536870912.0) return fail(PRENOM_ERR_SHAPE, "n_rays * n_samples > 2^29");
    if (n_rays > 0 && (!ray_obj || !t || !dt || !flags))
        return fail(PRENOM_ERR_INVALID_ARG, "ray_obj, t, dt and flags are required");
    const WsLayout w = ws_layout(&model->arch, n_rays, cfg->n_samples, cfg->recompute != 0);
    if (!ws || !aligned(ws, kAlign)) return fail(PRENOM_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    if (ws_bytes < w.total)
        return fail(PRENOM_ERR_WORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, w.total);
    return PRENOM_OK;
}

// Workspace of prenom_prior_refresh, for one chunk of at most kPriorChunk
// vertices: features [L][chunk][2], then head outputs [chunk][4].
constexpr int64_t kPriorChunk = int64_t(1) << 21;

size_t prior_refresh_ws(const prenom_arch* a, int32_t R, size_t* sc_off)
{
    const int64_t n = (int64_t)R * R * R;
    const int64_t c = n < kPriorChunk ? n : kPriorChunk;
    const size_t y = align_up((size_t)c * a->n_levels * a->n_features * sizeof(float));
    if (sc_off) *sc_off = y;
    return y + align_up((size_t)c * 4 * sizeof(float));
}

// Tile histograms of the training forward, in the workspace's scatter counts,
// laid out for the scatter plan of the samples encoded.
TileHist tile_hist(const WsLayout& w, const ScatterObj& plan, void* workspace)
{
    TileHist h{};
    h.counts = at<uint32_t>(workspace, w.counts);
    h.n_blocks = plan.n_blocks;
    for (int l = 0; l < plan.grid.n_levels; ++l) {
        h.tiles[l] = plan.tiles[l];
        h.tile_base[l] = plan.tile_base[l];
    }
    return h;
}

}  // namespace

extern "C" {

int64_t prenom_param_count(const prenom_arch* arch)
{
    if (check_arch(arch) != PRENOM_OK) return -1;
    return table_params(arch) + mlp_params(arch);
}

int64_t prenom_table_param_count(const prenom_arch* arch)
{
    if (check_arch(arch) != PRENOM_OK) return -1;
    return table_params(arch);
}

size_t prenom_workspace_size(const prenom_arch* arch, int64_t n_rays, int32_t n_samples, int32_t recompute)
{
    if (check_arch(arch) != PRENOM_OK || n_rays < 0 || n_samples < 1 || (recompute != 0 && recompute != 1)) return 0;
    return ws_layout(arch, n_rays, n_samples, recompute != 0).total;
}

size_t prenom_prior_refresh_workspace_size(const prenom_arch* arch, int32_t R)
{
    if (check_arch(arch) != PRENOM_OK || R < 2 || R > PRENOM_MAX_PRIOR_RES) return 0;
    return prior_refresh_ws(arch, R, nullptr);
}

prenom_status prenom_prior_refresh(const prenom_model* model, int32_t R, float* prior_out, void* workspace,
                                   size_t ws_bytes, void* stream)
{
    prenom_status st = check_model(model, false);
    if (st != PRENOM_OK) return st;
    if (R < 2 || R > PRENOM_MAX_PRIOR_RES) return fail(PRENOM_ERR_SHAPE, "R %d outside [2, %d]", R, PRENOM_MAX_PRIOR_RES);
    if (!prior_out) return fail(PRENOM_ERR_INVALID_ARG, "prior_out is NULL");
    const prenom_arch* a = &model->arch;
    size_t sc_off = 0;
    const size_t need = prior_refresh_ws(a, R, &sc_off);
    if (!workspace || !aligned(workspace, kAlign)) return fail(PRENOM_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    if (ws_bytes < need) return fail(PRENOM_ERR_WORKSPACE, "workspace %zu bytes < %zu", ws_bytes, need);
    return prior_refresh_chunks(model, R, prior_out, at<float>(workspace, 0), at<float>(workspace, sc_off), kPriorChunk,
                                (hipStream_t)stream);
}

prenom_status prenom_sample(const prenom_sample_cfg* cfg, const float* rays_o, const float* rays_d, const float* xi,
                            int64_t n_rays, float* ray_obj, float* t, float* dt, int32_t* bins, uint8_t* flags,
                            void* stream)
{
    prenom_status st = check_sample_cfg(cfg, true);
    if (st != PRENOM_OK) return st;
    if (n_rays < 0) return fail(PRENOM_ERR_SHAPE, "n_rays < 0");
    const bool use_prior = !cfg->uniform_only && cfg->prior != nullptr;
    if (n_rays > 0 && (!rays_o || !rays_d || !xi || !ray_obj || !t || !dt || !bins || !flags))
        return fail(PRENOM_ERR_INVALID_ARG, "NULL array argument");
    SampleArgs a{};
    a.n_coarse = cfg->n_coarse;
    a.n_fine = cfg->n_fine;
    a.include_coarse = cfg->include_coarse ? 1 : 0;
    a.use_prior = use_prior ? 1 : 0;
    a.eps = (double)cfg->eps;
    a.near_t = (double)cfg->near_t;
    a.far_t = (double)cfg->far_t;
    for (int i = 0; i < 12; ++i) a.A[i] = (double)cfg->world_to_obj[i];
    a.prior = cfg->prior;
    a.R = cfg->prior_res;
    a.rays_o = rays_o;
    a.rays_d = rays_d;
    a.xi = xi;
    a.n = n_rays;
    a.ray_obj = ray_obj;
    a.t = t;
    a.dt = dt;
    a.bins = bins;
    a.flags = flags;
    PRENOM_LAUNCH("k_sample", (hipStream_t)stream, launch_sample(a, (hipStream_t)stream));
    return PRENOM_OK;
}

prenom_status prenom_render_fwd(const prenom_model* model, const prenom_render_cfg* cfg, const float* ray_obj,
                                const float* t, const float* dt, const uint8_t* flags, int64_t n_rays, const float* bg,
                                const float* tgt_rgb, const float* tgt_depth, const uint8_t* mask, float* rgb,
                                float* depth, float* opacity, float* loss, float* sample_out, void* workspace,
                                size_t ws_bytes, void* stream)
{
    prenom_status st = check_render(model, cfg, ray_obj, t, dt, flags, n_rays, workspace, ws_bytes, false);
    if (st != PRENOM_OK) return st;
    if (n_rays > 0 && (!rgb || !depth || !opacity)) return fail(PRENOM_ERR_INVALID_ARG, "rgb, depth, opacity required");
    if (loss && !tgt_rgb && n_rays > 0) return fail(PRENOM_ERR_INVALID_ARG, "loss requested without tgt_rgb");
    hipStream_t s = (hipStream_t)stream;
    const prenom_arch* a = &model->arch;
    const bool recompute = cfg->recompute != 0;
    const int32_t S = cfg->n_samples;
    const WsLayout w = ws_layout(a, n_rays, S, recompute);
    const GridInfo g = grid_info(a);
    const MlpShape m = mlp_shape(a);
    float* y = at<float>(workspace, w.y);
    float* sc = at<float>(workspace, w.sc);
    const void* tlp = a->table_dtype == PRENOM_F16 ? model->table_lp : nullptr;
    double* loss_partial = loss ? at<double>(workspace, w.loss_partial) : nullptr;
    // The stored form runs once over all rays and keeps features, head outputs
    // and per-ray results (and the scatter's histograms) for render_bwd; the
    // recompute form runs pass by pass over chunks of rays and keeps nothing.
    const int64_t chunk = recompute ? recompute_chunk_rays(S) : (n_rays > 0 ? n_rays : 1);
    for (int64_t r0 = 0; r0 < n_rays; r0 += chunk) {
        const int64_t nr = n_rays - r0 < chunk ? n_rays - r0 : chunk;
        const int64_t n_s = nr * S;
        const ScatterObj plan = scatter_obj(g, n_s);
        const TileHist h = tile_hist(w, plan, workspace);
        PRENOM_LAUNCH("k_encode_fwd", s,
                      launch_encode_samples(g, model->params, tlp, ray_obj + 6 * r0, t + S * r0, nr, S, y, s,
                                            recompute ? nullptr : &h));
        PRENOM_LAUNCH("k_mlp_fwd", s,
                      mlp_fwd_any(m, model->params + table_params(a), y, n_s, sc, at<float>(workspace, w.act), s));
        CompositeArgs c{};
        c.n_rays = nr;
        c.norm_rays = n_rays;
        c.S = S;
        c.loss_mode = cfg->loss_mode;
        c.lambda_d = cfg->lambda_d;
        c.lambda_sigma = cfg->lambda_sigma;
        c.sc = sc;
        c.t = t + S * r0;
        c.dt = dt + S * r0;
        c.flags = flags + r0;
        c.bg = bg ? bg + 3 * r0 : nullptr;
        c.tgt_rgb = tgt_rgb ? tgt_rgb + 3 * r0 : nullptr;
        c.tgt_depth = tgt_depth ? tgt_depth + r0 : nullptr;
        c.mask = mask ? mask + r0 : nullptr;
        c.rgb = rgb + 3 * r0;
        c.depth = depth + r0;
        c.opacity = opacity + r0;
        c.ray_state = at<float>(workspace, w.ray_state);
        c.loss_partial = loss_partial ? loss_partial + r0 / composite_rays_per_block() : nullptr;
        PRENOM_LAUNCH("k_composite_fwd", s, launch_composite_fwd(c, s));
        if (sample_out && n_s > 0)
            PRENOM_TRY_HIP(hipMemcpyAsync(sample_out + 4 * S * r0, sc, (size_t)n_s * 4 * sizeof(float),
                                          hipMemcpyDeviceToDevice, s),
                           "copy sample_out");
    }
    if (loss) PRENOM_LAUNCH("k_loss_finalize", s, launch_loss_finalize(loss_partial, w.n_loss_blocks, loss, s));
    return PRENOM_OK;
}

prenom_status prenom_render_bwd(const prenom_model* model, const prenom_render_cfg* cfg, const float* ray_obj,
                                const float* t, const float* dt, const uint8_t* flags, int64_t n_rays, const float* bg,
                                const float* tgt_rgb, const float* tgt_depth, const uint8_t* mask, const float* d_rgb,
                                const float* d_depth, const float* d_opacity, void* workspace, size_t ws_bytes,
                                void* stream)
{
    prenom_status st = check_render(model, cfg, ray_obj, t, dt, flags, n_rays, workspace, ws_bytes, true);
    if (st != PRENOM_OK) return st;
    if (!d_rgb && !tgt_rgb && n_rays > 0)
        return fail(PRENOM_ERR_INVALID_ARG, "either d_rgb or the loss targets are required");
    hipStream_t s = (hipStream_t)stream;
    const prenom_arch* a = &model->arch;
    const bool recompute = cfg->recompute != 0;
    const int32_t S = cfg->n_samples;
    const WsLayout w = ws_layout(a, n_rays, S, recompute);
    const GridInfo g = grid_info(a);
    const MlpShape m = mlp_shape(a);
    const void* tlp = a->table_dtype == PRENOM_F16 ? model->table_lp : nullptr;
    const int64_t chunk = recompute ? recompute_chunk_rays(S) : (n_rays > 0 ? n_rays : 1);
    for (int64_t r0 = 0; r0 < n_rays; r0 += chunk) {
        const int64_t nr = n_rays - r0 < chunk ? n_rays - r0 : chunk;
        const int64_t n_s = nr * S;
        const ScatterObj plan = scatter_obj(g, n_s);
        const float* ro = ray_obj + 6 * r0;
        const float* tc = t + S * r0;
        CompositeArgs c{};
        c.n_rays = nr;
        c.norm_rays = n_rays;
        c.S = S;
        c.loss_mode = cfg->loss_mode;
        c.lambda_d = cfg->lambda_d;
        c.lambda_sigma = cfg->lambda_sigma;
        c.sc = at<float>(workspace, w.sc);
        c.t = tc;
        c.dt = dt + S * r0;
        c.flags = flags + r0;
        c.bg = bg ? bg + 3 * r0 : nullptr;
        c.tgt_rgb = tgt_rgb ? tgt_rgb + 3 * r0 : nullptr;
        c.tgt_depth = tgt_depth ? tgt_depth + r0 : nullptr;
        c.mask = mask ? mask + r0 : nullptr;
        c.ray_state = at<float>(workspace, w.ray_state);
        if (recompute) {
            // rebuild this pass's features, head outputs and per-ray results
            // (and the scatter's tile histograms) as render_fwd would have left them
            const TileHist h = tile_hist(w, plan, workspace);
            PRENOM_LAUNCH("k_encode_fwd", s,
                          launch_encode_samples(g, model->params, tlp, ro, tc, nr, S, at<float>(workspace, w.y), s, &h));
            PRENOM_LAUNCH("k_mlp_fwd", s, mlp_fwd_any(m, model->params + table_params(a), at<float>(workspace, w.y),
                                                      n_s, at<float>(workspace, w.sc), at<float>(workspace, w.act), s));
            CompositeArgs f = c;
            f.tgt_rgb = nullptr;  // per-ray results only, no loss
            PRENOM_LAUNCH("k_composite_fwd", s, launch_composite_fwd(f, s));
        }
        c.d_rgb = d_rgb ? d_rgb + 3 * r0 : nullptr;
        c.d_depth = d_depth ? d_depth + r0 : nullptr;
        c.d_opacity = d_opacity ? d_opacity + r0 : nullptr;
        c.loss_scale = model->loss_scale;
        c.dout = at<float>(workspace, w.dout);
        PRENOM_LAUNCH("k_composite_bwd", s, launch_composite_bwd(c, s));
        float* partial = at<float>(workspace, w.mlp_partial);
        float* dy = at<float>(workspace, w.dy);
        PRENOM_LAUNCH("k_mlp_bwd", s,
                      mlp_bwd_any(m, model->params + table_params(a), at<float>(workspace, w.y), c.dout,
                                  at<float>(workspace, w.sc), n_s, dy, partial, at<float>(workspace, w.act), s));
        if (n_s > 0)
            PRENOM_LAUNCH("k_reduce_partials", s,
                          launch_reduce_partials(partial, mlp_bwd_waves(n_s), mlp_params(a),
                                                 model->grads + table_params(a), s));
        ScatterArgs sa{};
        sa.S = S;
        sa.n_obj = 1;
        sa.one = plan;
        sa.objs = nullptr;
        sa.tiles_max = scatter_tiles_max(plan);
        sa.reduce_blocks = device_cus();
        sa.n_tiles = plan.n_tiles;
        sa.n_items = scatter_items(plan);
        sa.n_levels_total = a->n_levels;
        sa.ray_obj = ro;
        sa.t = tc;
        sa.dy = reinterpret_cast<const float2*>(dy);
        sa.g_table = model->grads;
        sa.counts = at<uint32_t>(workspace, w.counts);
        sa.offsets = at<uint32_t>(workspace, w.offsets);
        sa.block_max = at<float>(workspace, w.block_max);
        sa.level_max = at<float>(workspace, w.level_max);
        sa.tile_exp = at<int32_t>(workspace, w.tile_exp);
        sa.tile_total = at<uint64_t>(workspace, w.tile_total);
        sa.tile_start = at<uint64_t>(workspace, w.tile_start);
        sa.chunk_start = at<uint64_t>(workspace, w.chunk_start);
        sa.work_counter = at<unsigned long long>(workspace, w.work_counter);
        sa.recs = at<uint64_t>(workspace, w.recs);
        sa.n_records = scatter_records(plan);
        sa.nonfinite = model->loss_scale ? model->scaler_state : nullptr;
        sa.fwd_counts = 1;  // render_fwd (or the recompute above) wrote the tile histograms
        sa.merge_runs = 1;
        sa.chunk_min_bits = 21;  // one pass over one object: items of 2^21 records keep the CUs busy
        sa.compact = a->table_dtype == PRENOM_F16;
        for (int ph = 0; ph < kScatterPhases; ++ph)
            PRENOM_LAUNCH(ph == 0 ? "k_scatter_dymax" : kScatterPhaseNames[ph], s, launch_scatter_phase(sa, ph, s));
    }
    return PRENOM_OK;
}

prenom_status prenom_adam_step(const prenom_model* model, const prenom_adam_cfg* cfg, void* stream)
{
    prenom_status st = check_model(model, true);
    if (st != PRENOM_OK) return st;
    if (!cfg) return fail(PRENOM_ERR_INVALID_ARG, "cfg is NULL");
    if (cfg->step < 1) return fail(PRENOM_ERR_INVALID_ARG, "step must be >= 1");
    if (cfg->growth_interval < 0) return fail(PRENOM_ERR_INVALID_ARG, "growth_interval < 0");
    if (!model->adam_m || !model->adam_v || !aligned(model->adam_m, 16) || !aligned(model->adam_v, 16))
        return fail(PRENOM_ERR_INVALID_ARG, "adam moments NULL or not 16-byte aligned");
    if (!(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f && cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f && cfg->lr >= 0.0f &&
          cfg->eps >= 0.0f))
        return fail(PRENOM_ERR_INVALID_ARG, "Adam hyper-parameters out of range");
    AdamArgs a{};
    a.p = model->params;
    a.g = model->grads;
    a.m = model->adam_m;
    a.v = model->adam_v;
    a.n = table_params(&model->arch) + mlp_params(&model->arch);
    a.lr = cfg->lr;
    a.beta1 = cfg->beta1;
    a.beta2 = cfg->beta2;
    a.eps = cfg->eps;
    a.inv_c1 = (float)(1.0 / (1.0 - std::pow((double)cfg->beta1, (double)cfg->step)));
    a.inv_c2 = (float)(1.0 / (1.0 - std::pow((double)cfg->beta2, (double)cfg->step)));
    a.table_f16 = model->arch.table_dtype == PRENOM_F16 ? model->table_lp : nullptr;
    a.n_table = table_params(&model->arch);
    a.loss_scale = model->loss_scale;
    a.scaler_state = model->scaler_state;
    a.growth_interval = cfg->growth_interval;
    PRENOM_LAUNCH("k_adam", (hipStream_t)stream, launch_adam(a, (hipStream_t)stream));
    return PRENOM_OK;
}

prenom_status prenom_sgd_step(const prenom_model* model, const prenom_sgd_cfg* cfg, void* stream)
{
    prenom_status st = check_model(model, true);
    if (st != PRENOM_OK) return st;
    if (!cfg) return fail(PRENOM_ERR_INVALID_ARG, "cfg is NULL");
    if (!(cfg->lr >= 0.0f && std::isfinite(cfg->lr))) return fail(PRENOM_ERR_INVALID_ARG, "lr must be finite and >= 0");
    if (cfg->growth_interval < 0) return fail(PRENOM_ERR_INVALID_ARG, "growth_interval < 0");
    AdamArgs a{};
    a.p = model->params;
    a.g = model->grads;
    a.n = table_params(&model->arch) + mlp_params(&model->arch);
    a.lr = cfg->lr;
    a.table_f16 = model->arch.table_dtype == PRENOM_F16 ? model->table_lp : nullptr;
    a.n_table = table_params(&model->arch);
    a.loss_scale = model->loss_scale;
    a.scaler_state = model->scaler_state;
    a.growth_interval = cfg->growth_interval;
    PRENOM_LAUNCH("k_sgd", (hipStream_t)stream, launch_sgd(a, (hipStream_t)stream));
    return PRENOM_OK;
}

prenom_status prenom_reptile_update(float* theta, float* tasks, int64_t n_params, int32_t n_tasks, int64_t task_stride,
                                    float beta, float* adam_m, float* adam_v, void* tasks_lp, int64_t n_lp,
                                    int64_t* step, void* stream)
{
    if (n_params < 0) return fail(PRENOM_ERR_SHAPE, "n_params < 0");
    if (n_tasks < 1 || n_tasks > PRENOM_MAX_OBJECTS)
        return fail(PRENOM_ERR_SHAPE, "n_tasks %d outside [1, %d]", n_tasks, PRENOM_MAX_OBJECTS);
    if (task_stride < n_params || task_stride % 4 != 0)
        return fail(PRENOM_ERR_SHAPE, "task_stride %lld must be >= n_params and a multiple of 4", (long long)task_stride);
    if (!std::isfinite(beta)) return fail(PRENOM_ERR_INVALID_ARG, "beta is not finite");
    if ((adam_m == nullptr) != (adam_v == nullptr)) return fail(PRENOM_ERR_INVALID_ARG, "adam_m and adam_v: both or neither");
    if (tasks_lp && (n_lp < 0 || n_lp > n_params)) return fail(PRENOM_ERR_SHAPE, "n_lp outside [0, n_params]");
    if (n_params > 0) {
        if (!theta || !tasks || !aligned(theta, 16) || !aligned(tasks, 16))
            return fail(PRENOM_ERR_INVALID_ARG, "theta / tasks NULL or not 16-byte aligned");
        if ((adam_m && (!aligned(adam_m, 16) || !aligned(adam_v, 16))) || (tasks_lp && !aligned(tasks_lp, 8)))
            return fail(PRENOM_ERR_INVALID_ARG, "adam moments not 16-byte or tasks_lp not 8-byte aligned");
        const uintptr_t t0 = (uintptr_t)tasks, t1 = (uintptr_t)(tasks + (int64_t)(n_tasks - 1) * task_stride + n_params);
        const uintptr_t h0 = (uintptr_t)theta, h1 = (uintptr_t)(theta + n_params);
        if (h0 < t1 && t0 < h1) return fail(PRENOM_ERR_INVALID_ARG, "theta overlaps the task slots");
    }
    ReptileArgs a{};
    a.theta = theta;
    a.tasks = tasks;
    a.m = adam_m;
    a.v = adam_v;
    a.tasks_f16 = tasks_lp;
    a.n_f16 = tasks_lp ? n_lp : 0;
    a.step = step;
    a.n = n_params;
    a.stride = task_stride;
    a.n_tasks = n_tasks;
    a.beta = beta;
    PRENOM_LAUNCH("k_reptile", (hipStream_t)stream, launch_reptile(a, (hipStream_t)stream));
    return PRENOM_OK;
}

size_t prenom_canonical_yaw_workspace_size(int64_t n_points, int32_t n_yaw)
{
    if (n_points < 1 || n_points > PRENOM_MAX_YAW_POINTS || n_yaw < 1 || n_yaw > PRENOM_MAX_YAWS) return 0;
    return align_up((size_t)n_yaw * (size_t)yaw_chunks(n_points) * 7 * sizeof(double));
}

prenom_status prenom_canonical_yaw(const float* points, int64_t n_points, const float* prior, int32_t prior_res,
                                   int32_t n_yaw, double* scores, double* extents, double* centers, int32_t* best,
                                   void* workspace, size_t ws_bytes, void* stream)
{
    if (n_points < 1 || n_points > PRENOM_MAX_YAW_POINTS)
        return fail(PRENOM_ERR_SHAPE, "n_points %lld outside [1, %lld]", (long long)n_points,
                    (long long)PRENOM_MAX_YAW_POINTS);
    if (n_yaw < 1 || n_yaw > PRENOM_MAX_YAWS) return fail(PRENOM_ERR_SHAPE, "n_yaw %d outside [1, %d]", n_yaw, PRENOM_MAX_YAWS);
    if (prior_res < 2 || prior_res > PRENOM_MAX_PRIOR_RES)
        return fail(PRENOM_ERR_SHAPE, "prior_res %d outside [2, %d]", prior_res, PRENOM_MAX_PRIOR_RES);
    if (!points || !prior || !scores || !extents || !centers || !best)
        return fail(PRENOM_ERR_INVALID_ARG, "NULL array argument");
    const int64_t C = yaw_chunks(n_points);
    const size_t need = prenom_canonical_yaw_workspace_size(n_points, n_yaw);
    if (!workspace || !aligned(workspace, kAlign)) return fail(PRENOM_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    if (ws_bytes < need) return fail(PRENOM_ERR_WORKSPACE, "workspace %zu bytes < %zu", ws_bytes, need);
    YawArgs a{};
    a.pts = points;
    a.n = n_points;
    a.F = prior;
    a.R = prior_res;
    a.K = n_yaw;
    a.n_chunks = C;
    a.part_ext = at<double>(workspace, 0);
    a.part_sum = a.part_ext + (int64_t)n_yaw * C * 6;
    a.scores = scores;
    a.extents = extents;
    a.centers = centers;
    a.best = best;
    PRENOM_LAUNCH("k_canonical_yaw", (hipStream_t)stream, launch_canonical_yaw(a, (hipStream_t)stream));
    return PRENOM_OK;
}

prenom_status prenom_refresh_lowp(const prenom_model* model, void* stream)
{
    prenom_status st = check_model(model, false);
    if (st != PRENOM_OK) return st;
    if (model->arch.table_dtype != PRENOM_F16) return PRENOM_OK;
    PRENOM_LAUNCH("k_to_f16", (hipStream_t)stream,
                  launch_to_f16(model->params, model->table_lp, table_params(&model->arch), (hipStream_t)stream));
    return PRENOM_OK;
}

prenom_status prenom_encode(const prenom_arch* arch, const float* table, const float* pos, int64_t n, float* features,
                            int32_t* corner_idx, void* stream)
{
    prenom_status st = check_arch(arch);
    if (st != PRENOM_OK) return st;
    if (n < 0 || n >= (int64_t)1 << 31) return fail(PRENOM_ERR_SHAPE, "n outside [0, 2^31)");
    if (n > 0 && (!table || !pos || !features)) return fail(PRENOM_ERR_INVALID_ARG, "NULL array argument");
    if (table && !aligned(table, 16)) return fail(PRENOM_ERR_INVALID_ARG, "table not 16-byte aligned");
    if (features && !aligned(features, 8)) return fail(PRENOM_ERR_INVALID_ARG, "features not 8-byte aligned");
    PRENOM_LAUNCH("k_encode_points", (hipStream_t)stream,
                  launch_encode_points(grid_info(arch), table, pos, n, features, corner_idx, (hipStream_t)stream));
    return PRENOM_OK;
}

prenom_status prenom_profile_begin(void)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = true;
    g_prof_records.clear();
    g_pool_used = 0;
    return PRENOM_OK;
}

prenom_status prenom_profile_end(prenom_kernel_time* out, int32_t capacity, int32_t* n_kernels)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = false;
    int32_t n = 0;
    for (const ProfRecord& r : g_prof_records) {
        PRENOM_TRY_HIP(hipEventSynchronize(r.b), "hipEventSynchronize");
        float ms = 0.0f;
        PRENOM_TRY_HIP(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
        int32_t k = 0;
        while (k < n && std::strncmp(out[k].name, r.name, sizeof(out[k].name)) != 0) ++k;
        if (k == n) {
            if (!out || n >= capacity) continue;
            std::memset(out[k].name, 0, sizeof(out[k].name));
            std::strncpy(out[k].name, r.name, sizeof(out[k].name) - 1);
            out[k].launches = 0;
            out[k].total_ms = 0.0;
            ++n;
        }
        out[k].launches += 1;
        out[k].total_ms += (double)ms;
    }
    g_prof_records.clear();
    g_pool_used = 0;
    if (n_kernels) *n_kernels = n;
    return PRENOM_OK;
}

const char* prenom_status_string(prenom_status s)
{
    switch (s) {
        case PRENOM_OK: return "ok";
        case PRENOM_ERR_INVALID_ARG: return "invalid argument";
        case PRENOM_ERR_SHAPE: return "inconsistent shape";
        case PRENOM_ERR_UNSUPPORTED: return "unsupported architecture";
        case PRENOM_ERR_WORKSPACE: return "workspace too small";
        case PRENOM_ERR_HIP: return "HIP error";
    }
    return "unknown status";
}

const char* prenom_last_error(void) { return g_last_error; }

const char* prenom_version(void) { return "prenom-mi355x 0.1 (gfx950)"; }

}  // extern "C"

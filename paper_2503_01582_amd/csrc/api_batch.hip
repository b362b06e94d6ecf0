// C ABI of the batched multi-object step: the batch plan (device descriptors,
// MLP shape groups, scatter geometry, workspace layout) and the launch
// sequence of each call.  Host code only.
//
// Every phase is one launch over all objects (sampler, encoding, compositing,
// loss, MLP-gradient reduction, the five scatter kernels, Adam); the MLP is
// one launch per distinct MLP shape, since the shape fixes the kernel's
// registers and LDS.  The plan is a pure function of the objects, the tile
// shapes and S, so the calls need no host-device traffic and a step can be
// captured in a graph once prenom_batch_prepare has run.
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "api_util.h"
#include "common.h"

namespace {

using namespace prenom;
using namespace prenom::host;

constexpr int64_t kParamAlign = 64;  // floats: each object's parameters start 256-byte aligned
constexpr int kDefaultFwdTiles = 128;
constexpr int kDefaultBwdTiles = 1024;

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

int64_t obj_params(const prenom_arch* a) { return table_params(a) + mlp_params(a); }

struct Group {
    MlpShape shape;
    int fwd_tiles, bwd_tiles;
    int64_t fwd_first, n_fwd;  // work items in the forward / backward lists
    int64_t bwd_first, n_bwd;
    int64_t partial_off;       // floats
};

// One pass of the table-gradient scatter: consecutive whole objects
// [first, first + count), with their scatter geometry re-based so the pass's
// items, tiles and levels count from 0 (counts, block maxima, dy and the
// gradient keep the batch's offsets).
struct ScatterGroup {
    int first = 0, count = 0;
    int64_t n_items = 0, n_tiles = 0, records = 0;
    int32_t n_levels = 0;
};

struct Plan {
    int n_obj = 0, S = 0;
    std::vector<ObjDev> dev;
    std::vector<ScatterObj> sc;
    std::vector<ScatterObj> sc_pass;  // sc re-based per scatter group
    std::vector<ScatterGroup> sgroups;
    std::vector<MlpRed> red;
    std::vector<MlpWork> fwd, bwd;
    std::vector<Group> groups;
    int64_t n_rays = 0, n_params = 0, n_mlp_total = 0, n_tiles = 0, n_items = 0, records = 0;
    int64_t y_floats = 0, partial_floats = 0, counts = 0, bmax = 0, act_floats = 0;
    int32_t n_levels_total = 0, tiles_max = 1;
    bool any_f16_table = false, all_f16_table = true;
    // workspace offsets (bytes)
    size_t o_dev, o_sc, o_sc_pass, o_red, o_fwd, o_bwd;
    size_t y, sc_out, dout, dy, ray_state, ray_loss, partial, act, cnt, offs, block_max, level_max, tile_exp, tile_total,
        tile_start, chunk_start, work_counter, recs, total;
    uint64_t fingerprint = 0;
};

uint64_t fnv(uint64_t h, const void* p, size_t n)
{
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
    return h;
}

// Tile shape of the batched MLP launches for shape m.
void tiles_for(const prenom_batch* b, const MlpShape& m, int& fwd, int& bwd)
{
    fwd = kDefaultFwdTiles;
    bwd = kDefaultBwdTiles;
    for (int i = 0; i < b->n_tiles; ++i) {
        const prenom_mlp_tiles& t = b->tiles[i];
        if (t.in_dim == m.in_dim && t.width == m.width && t.hidden == m.hidden && t.dtype == m.dtype) {
            if (t.fwd_tiles > 0) fwd = t.fwd_tiles;
            if (t.bwd_tiles > 0) bwd = t.bwd_tiles;
        }
    }
}

prenom_status check_objects(const prenom_object* objs, int32_t n)
{
    if (n < 1 || n > PRENOM_MAX_OBJECTS) return fail(PRENOM_ERR_INVALID_ARG, "n_objects %d outside [1, %d]", n, PRENOM_MAX_OBJECTS);
    if (!objs) return fail(PRENOM_ERR_INVALID_ARG, "objects is NULL");
    for (int i = 0; i < n; ++i) {
        const prenom_status st = check_supported(&objs[i].arch);
        if (st != PRENOM_OK) return fail(st, "object %d: %s", i, last_error());
        if (objs[i].n_rays < 0) return fail(PRENOM_ERR_SHAPE, "object %d: n_rays < 0", i);
        if (objs[i].prior && objs[i].prior_res < 2) return fail(PRENOM_ERR_SHAPE, "object %d: prior_res < 2", i);
        for (int k = 0; k < 12; ++k)
            if (!std::isfinite(objs[i].world_to_obj[k]))
                return fail(PRENOM_ERR_INVALID_ARG, "object %d: world_to_obj not finite", i);
    }
    return PRENOM_OK;
}

prenom_status build_plan(const prenom_batch* b, int32_t S, Plan& p)
{
    if (!b) return fail(PRENOM_ERR_INVALID_ARG, "batch is NULL");
    prenom_status st = check_objects(b->objects, b->n_objects);
    if (st != PRENOM_OK) return st;
    if (S < 1 || S > 256) return fail(PRENOM_ERR_SHAPE, "n_samples %d outside [1, 256]", S);
    if (b->n_tiles < 0 || (b->n_tiles > 0 && !b->tiles)) return fail(PRENOM_ERR_INVALID_ARG, "tiles");
    if (b->record_budget < 0) return fail(PRENOM_ERR_INVALID_ARG, "record_budget < 0");
    for (int i = 0; i < b->n_tiles; ++i) {
        const prenom_mlp_tiles& t = b->tiles[i];
        if (t.fwd_tiles != 0 && (t.fwd_tiles < 4 || t.fwd_tiles > 4096 || t.fwd_tiles % 4))
            return fail(PRENOM_ERR_INVALID_ARG, "tiles[%d].fwd_tiles %d", i, t.fwd_tiles);
        if (t.bwd_tiles != 0 && (t.bwd_tiles < 32 || t.bwd_tiles > 1024 || t.bwd_tiles % 32))
            return fail(PRENOM_ERR_INVALID_ARG, "tiles[%d].bwd_tiles %d", i, t.bwd_tiles);
    }
    const int n = b->n_objects;
    p = Plan{};
    p.n_obj = n;
    p.S = S;
    p.dev.resize(n);
    p.sc.resize(n);
    p.red.resize(n);
    uint64_t h = 1469598103934665603ull;
    h = fnv(h, &n, sizeof n);
    h = fnv(h, &S, sizeof S);

    int64_t ray = 0, param = 0, yoff = 0, tile = 0, item = 0, cnt = 0, bmax = 0, mlp = 0;
    int32_t lev = 0;
    for (int i = 0; i < n; ++i) {
        const prenom_object& o = b->objects[i];
        const prenom_arch* a = &o.arch;
        h = fnv(h, a, sizeof *a);
        h = fnv(h, &o.n_rays, sizeof o.n_rays);
        h = fnv(h, &o.prior, sizeof o.prior);
        h = fnv(h, &o.prior_res, sizeof o.prior_res);
        h = fnv(h, o.world_to_obj, sizeof o.world_to_obj);
        const int64_t n_s = o.n_rays * S;
        ObjDev& d = p.dev[i];
        d = ObjDev{};
        d.grid = grid_info(a);
        d.table_dtype = a->table_dtype;
        d.prior_res = o.prior ? o.prior_res : 0;
        d.param_off = param;
        d.ray_begin = ray;
        d.n_rays = o.n_rays;
        d.y_off = yoff;
        d.prior = o.prior;
        for (int k = 0; k < 12; ++k) d.A[k] = (double)o.world_to_obj[k];
        p.any_f16_table = p.any_f16_table || a->table_dtype == PRENOM_F16;
        p.all_f16_table = p.all_f16_table && a->table_dtype == PRENOM_F16;

        ScatterObj& so = p.sc[i];
        so = scatter_obj(d.grid, n_s);
        so.lev_off = lev;
        so.s_begin = ray * S;
        so.dy_off = yoff / 2;
        so.g_off = param;
        so.tile_off = tile;
        so.count_off = cnt;
        so.bmax_off = bmax;
        so.item_off = item;
        p.tiles_max = scatter_tiles_max(so) > p.tiles_max ? scatter_tiles_max(so) : p.tiles_max;

        MlpRed& r = p.red[i];
        r.mlp_begin = mlp;
        r.n_mlp = mlp_params(a);
        r.g_off = param + table_params(a);

        ray += o.n_rays;
        param += round_up(obj_params(a), kParamAlign);
        yoff += (int64_t)a->n_levels * n_s * 2;
        tile += so.n_tiles;
        item += scatter_items(so);
        cnt += (int64_t)so.n_tiles * so.n_blocks;
        bmax += (int64_t)a->n_levels * so.n_blocks;
        lev += a->n_levels;
        mlp += r.n_mlp;
    }
    if ((double)ray * S > 536870912.0) return fail(PRENOM_ERR_SHAPE, "batch rays * n_samples > 2^29");
    p.n_rays = ray;
    p.n_params = param;
    p.y_floats = yoff;
    p.n_tiles = tile;
    p.n_items = item;
    p.counts = cnt;
    p.bmax = bmax;
    p.n_levels_total = lev;
    p.n_mlp_total = mlp;
    if (item >= ((int64_t)1 << 31) || tile >= ((int64_t)1 << 31))
        return fail(PRENOM_ERR_SHAPE, "batch grid too large");

    // scatter passes: greedy runs of whole objects within the record budget
    const int64_t budget = (b->record_budget > 0 ? b->record_budget : PRENOM_RECORD_BUDGET) / (int64_t)sizeof(uint64_t);
    h = fnv(h, &budget, sizeof budget);
    p.sc_pass = p.sc;
    p.records = 0;
    for (int i = 0; i < n;) {
        ScatterGroup g{};
        g.first = i;
        do {
            ScatterObj& lo = p.sc_pass[i];
            lo.item_off = g.n_items;
            lo.tile_off = g.n_tiles;
            lo.lev_off = g.n_levels;
            g.n_items += scatter_items(p.sc[i]);
            g.n_tiles += p.sc[i].n_tiles;
            g.n_levels += p.sc[i].grid.n_levels;
            g.records += scatter_records(p.sc[i]);
            ++i;
        } while (i < n && g.records + scatter_records(p.sc[i]) <= budget);
        g.count = i - g.first;
        p.records = g.records > p.records ? g.records : p.records;
        p.sgroups.push_back(g);
    }

    // MLP groups, in order of first appearance; work items object by object
    for (int i = 0; i < n; ++i) {
        const MlpShape m = mlp_shape(&b->objects[i].arch);
        bool found = false;
        for (const Group& g : p.groups)
            found = found || (g.shape.in_dim == m.in_dim && g.shape.width == m.width && g.shape.hidden == m.hidden &&
                              g.shape.dtype == m.dtype);
        if (found) continue;
        Group g{};
        g.shape = m;
        tiles_for(b, m, g.fwd_tiles, g.bwd_tiles);
        p.groups.push_back(g);
    }
    int64_t partial = 0, act = 0;
    for (Group& g : p.groups) {
        g.fwd_first = (int64_t)p.fwd.size();
        g.bwd_first = (int64_t)p.bwd.size();
        g.partial_off = partial;
        for (int i = 0; i < n; ++i) {
            const prenom_arch* a = &b->objects[i].arch;
            const MlpShape m = mlp_shape(a);
            if (!(m.in_dim == g.shape.in_dim && m.width == g.shape.width && m.hidden == g.shape.hidden &&
                  m.dtype == g.shape.dtype))
                continue;
            const int64_t n_s = b->objects[i].n_rays * S, n_t = (n_s + 15) / 16;
            MlpWork w{};
            w.w_off = p.dev[i].param_off + table_params(a);
            w.y_off = p.dev[i].y_off;
            w.s_off = p.dev[i].ray_begin * S;
            w.n_s = n_s;
            w.a_off = act;
            w.bmax_off = p.sc[i].bmax_off;
            w.n_sblocks = p.sc[i].n_blocks;
            act += mlp_act_floats(m, n_s);
            for (int64_t t0 = 0; t0 < n_t; t0 += g.fwd_tiles) {
                w.tile_begin = t0;
                w.tile_end = t0 + g.fwd_tiles < n_t ? t0 + g.fwd_tiles : n_t;
                p.fwd.push_back(w);
            }
            const int64_t first_slot = (int64_t)p.bwd.size() - g.bwd_first;
            for (int64_t t0 = 0; t0 < n_t; t0 += g.bwd_tiles) {
                w.tile_begin = t0;
                w.tile_end = t0 + g.bwd_tiles < n_t ? t0 + g.bwd_tiles : n_t;
                p.bwd.push_back(w);
            }
            MlpRed& r = p.red[i];
            r.n_slots = (int64_t)p.bwd.size() - g.bwd_first - first_slot;
            r.partial_off = partial + first_slot * r.n_mlp;
        }
        g.n_fwd = (int64_t)p.fwd.size() - g.fwd_first;
        g.n_bwd = (int64_t)p.bwd.size() - g.bwd_first;
        const int64_t n_mlp = mlp_params_of(g.shape);
        partial += g.n_bwd * n_mlp;
        if (g.n_fwd >= ((int64_t)1 << 31) || g.n_bwd >= ((int64_t)1 << 31))
            return fail(PRENOM_ERR_SHAPE, "MLP grid too large");
    }
    p.partial_floats = partial;
    p.act_floats = act;
    for (int i = 0; i < b->n_tiles; ++i) h = fnv(h, &b->tiles[i], sizeof b->tiles[i]);
    p.fingerprint = h;

    // workspace layout
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + (bytes ? bytes : 1));
        return o;
    };
    const size_t n_s = (size_t)p.n_rays * (size_t)S;
    p.o_dev = take(sizeof(ObjDev) * n);
    p.o_sc = take(sizeof(ScatterObj) * n);
    p.o_sc_pass = take(sizeof(ScatterObj) * n);
    p.o_red = take(sizeof(MlpRed) * n);
    p.o_fwd = take(sizeof(MlpWork) * p.fwd.size());
    p.o_bwd = take(sizeof(MlpWork) * p.bwd.size());
    p.y = take(sizeof(float) * (size_t)p.y_floats);
    p.sc_out = take(sizeof(float) * 4 * n_s);
    p.dout = take(sizeof(float) * 4 * n_s);
    p.dy = take(sizeof(float) * (size_t)p.y_floats);
    p.ray_state = take(sizeof(float) * 8 * (size_t)p.n_rays);
    p.ray_loss = take(sizeof(double) * (size_t)p.n_rays);
    p.partial = take(sizeof(float) * (size_t)p.partial_floats);
    p.act = take(sizeof(float) * (size_t)p.act_floats);
    p.cnt = take(sizeof(uint32_t) * (size_t)p.counts);
    p.offs = take(sizeof(uint32_t) * (size_t)p.counts);
    p.block_max = take(sizeof(float) * (size_t)p.bmax);
    p.level_max = take(sizeof(float) * (size_t)p.n_levels_total);
    p.tile_exp = take(sizeof(int32_t) * (size_t)p.n_tiles);
    p.tile_total = take(sizeof(uint64_t) * (size_t)p.n_tiles);
    p.tile_start = take(sizeof(uint64_t) * (size_t)(p.n_tiles + 1));
    p.chunk_start = take(sizeof(uint64_t) * (size_t)(p.n_tiles + 2));
    p.work_counter = take(sizeof(uint64_t));
    p.recs = take(sizeof(uint64_t) * (size_t)p.records);
    p.total = off;
    return PRENOM_OK;
}

// Workspaces prepared by prenom_batch_prepare, with the plan fingerprint.
std::mutex g_prep_mu;
std::map<const void*, uint64_t> g_prepared;

prenom_status check_prepared(const Plan& p, void* ws, size_t ws_bytes)
{
    if (!ws || !aligned(ws, kAlign)) return fail(PRENOM_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    if (ws_bytes < p.total) return fail(PRENOM_ERR_WORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, p.total);
    std::lock_guard<std::mutex> lk(g_prep_mu);
    auto it = g_prepared.find(ws);
    if (it == g_prepared.end() || it->second != p.fingerprint)
        return fail(PRENOM_ERR_WORKSPACE, "workspace not prepared for this batch (call prenom_batch_prepare)");
    return PRENOM_OK;
}

prenom_status check_params(const prenom_batch* b, const Plan& p, bool need_grads)
{
    if (!b->params || !aligned(b->params, 256)) return fail(PRENOM_ERR_INVALID_ARG, "params NULL or not 256-byte aligned");
    if (need_grads && (!b->grads || !aligned(b->grads, 256)))
        return fail(PRENOM_ERR_INVALID_ARG, "grads NULL or not 256-byte aligned");
    if (p.any_f16_table && (!b->params_lp || !aligned(b->params_lp, 128)))
        return fail(PRENOM_ERR_INVALID_ARG, "an FP16 table needs a 128-byte aligned params_lp");
    if (b->loss_scale && !b->scaler_state) return fail(PRENOM_ERR_INVALID_ARG, "loss_scale needs scaler_state");
    return PRENOM_OK;
}

// Scatter of group g's objects; the per-tile and per-level arrays are reused
// from their start by every pass.
ScatterArgs scatter_args(const Plan& p, const ScatterGroup& g, void* ws, const float* ray_obj, const float* t,
                         float* grads, int32_t* nonfinite)
{
    ScatterArgs sa{};
    sa.S = p.S;
    sa.n_obj = g.count;
    sa.objs = at<ScatterObj>(ws, p.o_sc_pass) + g.first;
    sa.tiles_max = p.tiles_max;
    sa.reduce_blocks = device_cus();
    sa.n_tiles = g.n_tiles;
    sa.n_items = g.n_items;
    sa.n_levels_total = g.n_levels;
    sa.ray_obj = ray_obj;
    sa.t = t;
    sa.dy = at<const float2>(ws, p.dy);
    sa.g_table = grads;
    sa.counts = at<uint32_t>(ws, p.cnt);
    sa.offsets = at<uint32_t>(ws, p.offs);
    sa.block_max = at<float>(ws, p.block_max);
    sa.level_max = at<float>(ws, p.level_max);
    sa.tile_exp = at<int32_t>(ws, p.tile_exp);
    sa.tile_total = at<uint64_t>(ws, p.tile_total);
    sa.tile_start = at<uint64_t>(ws, p.tile_start);
    sa.chunk_start = at<uint64_t>(ws, p.chunk_start);
    sa.work_counter = at<unsigned long long>(ws, p.work_counter);
    sa.recs = at<uint64_t>(ws, p.recs);
    sa.n_records = p.records;
    sa.nonfinite = nonfinite;
    sa.fwd_counts = 1;  // fwd_features (render_fwd, or the recompute in render_bwd) wrote the histograms
    sa.merge_runs = 1;
    sa.chunk_min_bits = 18;  // a pass of a few objects needs smaller items to fill the CUs
    sa.compact = p.all_f16_table;
    return sa;
}

// Encoding + MLP forward of every object: features and head outputs in the workspace.
prenom_status fwd_features(const prenom_batch* b, const Plan& p, const float* ray_obj, const float* t, void* ws,
                           hipStream_t s)
{
    const ObjDev* dev = at<const ObjDev>(ws, p.o_dev);
    float* y = at<float>(ws, p.y);
    // the encoding also writes the tile histograms the backward's scatter starts from
    PRENOM_LAUNCH("k_encode_fwd", s,
                  launch_encode_batch_hist(dev, at<const ScatterObj>(ws, p.o_sc), p.n_obj, p.n_items, b->params,
                                           p.any_f16_table ? b->params_lp : nullptr, ray_obj, t, p.S, y,
                                           at<uint32_t>(ws, p.cnt), s));
    for (const Group& g : p.groups) {
        const MlpWork* work = at<const MlpWork>(ws, p.o_fwd) + g.fwd_first;
        float* sc = at<float>(ws, p.sc_out);
        PRENOM_LAUNCH("k_mlp_fwd", s,
                      g.shape.dtype == PRENOM_F32
                          ? launch_mlp_fwd_batch(g.shape, work, (int)g.n_fwd, b->params, y, sc, at<float>(ws, p.act), s)
                          : launch_mlp_fwd_lp_batch(g.shape, work, (int)g.n_fwd, b->params, y, sc, at<float>(ws, p.act),
                                                    s));
    }
    return PRENOM_OK;
}

CompositeArgs composite_args(const prenom_render_cfg* cfg, const Plan& p, void* ws, const float* t, const float* dt,
                             const uint8_t* flags, const float* bg)
{
    CompositeArgs c{};
    c.n_rays = p.n_rays;
    c.S = p.S;
    c.loss_mode = cfg->loss_mode;
    c.lambda_d = cfg->lambda_d;
    c.lambda_sigma = cfg->lambda_sigma;
    c.sc = at<float>(ws, p.sc_out);
    c.t = t;
    c.dt = dt;
    c.flags = flags;
    c.bg = bg;
    c.ray_state = at<float>(ws, p.ray_state);
    c.objs = at<const ObjDev>(ws, p.o_dev);
    c.n_obj = p.n_obj;
    return c;
}

prenom_status check_ray_arrays(const Plan& p, const float* ray_obj, const float* t, const float* dt,
                               const uint8_t* flags)
{
    if (p.n_rays > 0 && (!ray_obj || !t || !dt || !flags))
        return fail(PRENOM_ERR_INVALID_ARG, "ray_obj, t, dt and flags are required");
    return PRENOM_OK;
}

}  // namespace

namespace prenom {
namespace host {
int64_t mlp_params_of(const MlpShape& m)
{
    return (int64_t)m.width * m.in_dim + (int64_t)(m.hidden - 1) * m.width * m.width + (int64_t)PRENOM_N_OUT * m.width;
}
}  // namespace host
}  // namespace prenom

extern "C" {

int64_t prenom_batch_param_count(const prenom_object* objects, int32_t n_objects)
{
    if (check_objects(objects, n_objects) != PRENOM_OK) return -1;
    int64_t n = 0;
    for (int i = 0; i < n_objects; ++i) n += round_up(obj_params(&objects[i].arch), kParamAlign);
    return n;
}

int64_t prenom_batch_param_offset(const prenom_object* objects, int32_t n_objects, int32_t i)
{
    if (check_objects(objects, n_objects) != PRENOM_OK || i < 0 || i >= n_objects) return -1;
    int64_t n = 0;
    for (int k = 0; k < i; ++k) n += round_up(obj_params(&objects[k].arch), kParamAlign);
    return n;
}

size_t prenom_batch_workspace_size(const prenom_batch* batch, int32_t n_samples)
{
    Plan p;
    if (build_plan(batch, n_samples, p) != PRENOM_OK) return 0;
    return p.total;
}

prenom_status prenom_batch_prepare(const prenom_batch* batch, int32_t n_samples, void* workspace, size_t ws_bytes,
                                   void* stream)
{
    Plan p;
    prenom_status st = build_plan(batch, n_samples, p);
    if (st != PRENOM_OK) return st;
    if (!workspace || !aligned(workspace, kAlign))
        return fail(PRENOM_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    if (ws_bytes < p.total) return fail(PRENOM_ERR_WORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, p.total);
    hipStream_t s = (hipStream_t)stream;
    auto put = [&](size_t off, const void* src, size_t bytes) {
        return bytes ? hipMemcpyAsync(at<char>(workspace, off), src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    PRENOM_TRY_HIP(put(p.o_dev, p.dev.data(), sizeof(ObjDev) * p.dev.size()), "upload objects");
    PRENOM_TRY_HIP(put(p.o_sc, p.sc.data(), sizeof(ScatterObj) * p.sc.size()), "upload scatter geometry");
    PRENOM_TRY_HIP(put(p.o_sc_pass, p.sc_pass.data(), sizeof(ScatterObj) * p.sc_pass.size()),
                   "upload scatter passes");
    PRENOM_TRY_HIP(put(p.o_red, p.red.data(), sizeof(MlpRed) * p.red.size()), "upload reductions");
    PRENOM_TRY_HIP(put(p.o_fwd, p.fwd.data(), sizeof(MlpWork) * p.fwd.size()), "upload forward work");
    PRENOM_TRY_HIP(put(p.o_bwd, p.bwd.data(), sizeof(MlpWork) * p.bwd.size()), "upload backward work");
    PRENOM_TRY_HIP(hipStreamSynchronize(s), "prepare: synchronize");
    std::lock_guard<std::mutex> lk(g_prep_mu);
    g_prepared[workspace] = p.fingerprint;
    return PRENOM_OK;
}

prenom_status prenom_batch_sample(const prenom_batch* batch, const prenom_sample_cfg* cfg, const float* rays_o,
                                  const float* rays_d, const float* xi, float* ray_obj, float* t, float* dt,
                                  int32_t* bins, uint8_t* flags, void* workspace, size_t ws_bytes, void* stream)
{
    prenom_status st = check_sample_cfg(cfg, false);
    if (st != PRENOM_OK) return st;
    const int32_t S = cfg->n_fine + (cfg->include_coarse ? cfg->n_coarse : 0);
    Plan p;
    if ((st = build_plan(batch, S, p)) != PRENOM_OK) return st;
    if ((st = check_prepared(p, workspace, ws_bytes)) != PRENOM_OK) return st;
    if (p.n_rays > 0 && (!rays_o || !rays_d || !xi || !ray_obj || !t || !dt || !bins || !flags))
        return fail(PRENOM_ERR_INVALID_ARG, "NULL array argument");
    SampleArgs a{};
    a.n_coarse = cfg->n_coarse;
    a.n_fine = cfg->n_fine;
    a.include_coarse = cfg->include_coarse ? 1 : 0;
    a.use_prior = cfg->uniform_only ? 0 : 1;
    a.eps = (double)cfg->eps;
    a.near_t = (double)cfg->near_t;
    a.far_t = (double)cfg->far_t;
    a.rays_o = rays_o;
    a.rays_d = rays_d;
    a.xi = xi;
    a.n = p.n_rays;
    a.ray_obj = ray_obj;
    a.t = t;
    a.dt = dt;
    a.bins = bins;
    a.flags = flags;
    hipStream_t s = (hipStream_t)stream;
    PRENOM_LAUNCH("k_sample", s, launch_sample_batch(a, at<const ObjDev>(workspace, p.o_dev), p.n_obj, s));
    return PRENOM_OK;
}

prenom_status prenom_batch_render_fwd(const prenom_batch* batch, const prenom_render_cfg* cfg, const float* ray_obj,
                                      const float* t, const float* dt, const uint8_t* flags, const float* bg,
                                      const float* tgt_rgb, const float* tgt_depth, const uint8_t* mask, float* rgb,
                                      float* depth, float* opacity, float* loss, void* workspace, size_t ws_bytes,
                                      void* stream)
{
    prenom_status st = check_render_cfg(cfg);
    if (st != PRENOM_OK) return st;
    Plan p;
    if ((st = build_plan(batch, cfg->n_samples, p)) != PRENOM_OK) return st;
    if ((st = check_prepared(p, workspace, ws_bytes)) != PRENOM_OK) return st;
    if ((st = check_params(batch, p, false)) != PRENOM_OK) return st;
    if ((st = check_ray_arrays(p, ray_obj, t, dt, flags)) != PRENOM_OK) return st;
    if (p.n_rays > 0 && (!rgb || !depth || !opacity)) return fail(PRENOM_ERR_INVALID_ARG, "rgb, depth, opacity required");
    if (loss && !tgt_rgb && p.n_rays > 0) return fail(PRENOM_ERR_INVALID_ARG, "loss requested without tgt_rgb");
    hipStream_t s = (hipStream_t)stream;
    if ((st = fwd_features(batch, p, ray_obj, t, workspace, s)) != PRENOM_OK) return st;
    CompositeArgs c = composite_args(cfg, p, workspace, t, dt, flags, bg);
    c.tgt_rgb = tgt_rgb;
    c.tgt_depth = tgt_depth;
    c.mask = mask;
    c.rgb = rgb;
    c.depth = depth;
    c.opacity = opacity;
    c.ray_loss = loss ? at<double>(workspace, p.ray_loss) : nullptr;
    PRENOM_LAUNCH("k_composite_fwd", s, launch_composite_fwd(c, s));
    if (loss)
        PRENOM_LAUNCH("k_loss_finalize", s,
                      launch_loss_objects(at<const ObjDev>(workspace, p.o_dev), p.n_obj, c.ray_loss, loss, s));
    return PRENOM_OK;
}

prenom_status prenom_batch_render_bwd(const prenom_batch* batch, const prenom_render_cfg* cfg, const float* ray_obj,
                                      const float* t, const float* dt, const uint8_t* flags, const float* bg,
                                      const float* tgt_rgb, const float* tgt_depth, const uint8_t* mask,
                                      const float* d_rgb, const float* d_depth, const float* d_opacity,
                                      void* workspace, size_t ws_bytes, void* stream)
{
    prenom_status st = check_render_cfg(cfg);
    if (st != PRENOM_OK) return st;
    Plan p;
    if ((st = build_plan(batch, cfg->n_samples, p)) != PRENOM_OK) return st;
    if ((st = check_prepared(p, workspace, ws_bytes)) != PRENOM_OK) return st;
    if ((st = check_params(batch, p, true)) != PRENOM_OK) return st;
    if ((st = check_ray_arrays(p, ray_obj, t, dt, flags)) != PRENOM_OK) return st;
    if (!d_rgb && !tgt_rgb && p.n_rays > 0)
        return fail(PRENOM_ERR_INVALID_ARG, "either d_rgb or the loss targets are required");
    hipStream_t s = (hipStream_t)stream;
    if (cfg->recompute) {
        if ((st = fwd_features(batch, p, ray_obj, t, workspace, s)) != PRENOM_OK) return st;
        CompositeArgs f = composite_args(cfg, p, workspace, t, dt, flags, bg);
        PRENOM_LAUNCH("k_composite_fwd", s, launch_composite_fwd(f, s));
    }
    CompositeArgs c = composite_args(cfg, p, workspace, t, dt, flags, bg);
    c.tgt_rgb = tgt_rgb;
    c.tgt_depth = tgt_depth;
    c.mask = mask;
    c.d_rgb = d_rgb;
    c.d_depth = d_depth;
    c.d_opacity = d_opacity;
    c.loss_scale = batch->loss_scale;
    c.dout = at<float>(workspace, p.dout);
    PRENOM_LAUNCH("k_composite_bwd", s, launch_composite_bwd(c, s));
    float* partial = at<float>(workspace, p.partial);
    // the MLP backward also writes the maxima of |dy| per (object, level,
    // scatter block) and flags a non-finite dy, so the scatter starts at its
    // level maxima (phase 1)
    float* block_max = at<float>(workspace, p.block_max);
    int32_t* nonfinite = batch->loss_scale ? batch->scaler_state : nullptr;
    for (const Group& g : p.groups) {
        const MlpWork* work = at<const MlpWork>(workspace, p.o_bwd) + g.bwd_first;
        const int64_t n_mlp = mlp_params_of(g.shape);
        float* y = at<float>(workspace, p.y);
        float* dy = at<float>(workspace, p.dy);
        PRENOM_LAUNCH("k_mlp_bwd", s,
                      g.shape.dtype == PRENOM_F32
                          ? launch_mlp_bwd_batch(g.shape, work, (int)g.n_bwd, batch->params, y, c.dout, c.sc, dy,
                                                 partial + g.partial_off, n_mlp, at<float>(workspace, p.act),
                                                 block_max, nonfinite, s)
                          : launch_mlp_bwd_lp_batch(g.shape, work, (int)g.n_bwd, batch->params, y, c.dout, c.sc, dy,
                                                    partial + g.partial_off, n_mlp, at<float>(workspace, p.act),
                                                    block_max, nonfinite, s));
    }
    PRENOM_LAUNCH("k_reduce_partials", s,
                  launch_reduce_partials_batch(at<const MlpRed>(workspace, p.o_red), p.n_obj, p.n_mlp_total, partial,
                                               batch->grads, s));
    for (const ScatterGroup& g : p.sgroups) {
        const ScatterArgs sa = scatter_args(p, g, workspace, ray_obj, t, batch->grads, nonfinite);
        for (int ph = 1; ph < kScatterPhases; ++ph)
            PRENOM_LAUNCH(kScatterPhaseNames[ph], s, launch_scatter_phase(sa, ph, s));
    }
    return PRENOM_OK;
}

prenom_status prenom_batch_adam_step(const prenom_batch* batch, const prenom_adam_cfg* cfg, void* stream)
{
    if (!batch) return fail(PRENOM_ERR_INVALID_ARG, "batch is NULL");
    prenom_status st = check_objects(batch->objects, batch->n_objects);
    if (st != PRENOM_OK) return st;
    if (!cfg) return fail(PRENOM_ERR_INVALID_ARG, "cfg is NULL");
    if (!batch->step && cfg->step < 1) return fail(PRENOM_ERR_INVALID_ARG, "step must be >= 1");
    if (cfg->growth_interval < 0) return fail(PRENOM_ERR_INVALID_ARG, "growth_interval < 0");
    if (!(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f && cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f && cfg->lr >= 0.0f &&
          cfg->eps >= 0.0f))
        return fail(PRENOM_ERR_INVALID_ARG, "Adam hyper-parameters out of range");
    bool any_f16 = false;
    for (int i = 0; i < batch->n_objects; ++i) any_f16 = any_f16 || batch->objects[i].arch.table_dtype == PRENOM_F16;
    Plan dummy;
    dummy.any_f16_table = any_f16;
    if ((st = check_params(batch, dummy, true)) != PRENOM_OK) return st;
    if (!batch->adam_m || !batch->adam_v || !aligned(batch->adam_m, 256) || !aligned(batch->adam_v, 256))
        return fail(PRENOM_ERR_INVALID_ARG, "adam moments NULL or not 256-byte aligned");
    AdamArgs a{};
    a.p = batch->params;
    a.g = batch->grads;
    a.m = batch->adam_m;
    a.v = batch->adam_v;
    a.n = prenom_batch_param_count(batch->objects, batch->n_objects);
    a.lr = cfg->lr;
    a.beta1 = cfg->beta1;
    a.beta2 = cfg->beta2;
    a.eps = cfg->eps;
    const double k = batch->step ? 1.0 : (double)cfg->step;
    a.inv_c1 = (float)(1.0 / (1.0 - std::pow((double)cfg->beta1, k)));
    a.inv_c2 = (float)(1.0 / (1.0 - std::pow((double)cfg->beta2, k)));
    a.table_f16 = any_f16 ? batch->params_lp : nullptr;
    a.n_table = a.n;
    a.loss_scale = batch->loss_scale;
    a.scaler_state = batch->scaler_state;
    a.growth_interval = cfg->growth_interval;
    a.step_dev = batch->step;
    PRENOM_LAUNCH("k_adam", (hipStream_t)stream, launch_adam(a, (hipStream_t)stream));
    return PRENOM_OK;
}

prenom_status prenom_batch_sgd_step(const prenom_batch* batch, const prenom_sgd_cfg* cfg, void* stream)
{
    if (!batch) return fail(PRENOM_ERR_INVALID_ARG, "batch is NULL");
    prenom_status st = check_objects(batch->objects, batch->n_objects);
    if (st != PRENOM_OK) return st;
    if (!cfg) return fail(PRENOM_ERR_INVALID_ARG, "cfg is NULL");
    if (!(cfg->lr >= 0.0f && std::isfinite(cfg->lr))) return fail(PRENOM_ERR_INVALID_ARG, "lr must be finite and >= 0");
    if (cfg->growth_interval < 0) return fail(PRENOM_ERR_INVALID_ARG, "growth_interval < 0");
    bool any_f16 = false;
    for (int i = 0; i < batch->n_objects; ++i) any_f16 = any_f16 || batch->objects[i].arch.table_dtype == PRENOM_F16;
    Plan dummy;
    dummy.any_f16_table = any_f16;
    if ((st = check_params(batch, dummy, true)) != PRENOM_OK) return st;
    AdamArgs a{};
    a.p = batch->params;
    a.g = batch->grads;
    a.n = prenom_batch_param_count(batch->objects, batch->n_objects);
    a.lr = cfg->lr;
    a.table_f16 = any_f16 ? batch->params_lp : nullptr;
    a.n_table = a.n;
    a.loss_scale = batch->loss_scale;
    a.scaler_state = batch->scaler_state;
    a.growth_interval = cfg->growth_interval;
    a.step_dev = batch->step;
    PRENOM_LAUNCH("k_sgd", (hipStream_t)stream, launch_sgd(a, (hipStream_t)stream));
    return PRENOM_OK;
}

prenom_status prenom_batch_refresh_lowp(const prenom_batch* batch, void* stream)
{
    if (!batch) return fail(PRENOM_ERR_INVALID_ARG, "batch is NULL");
    prenom_status st = check_objects(batch->objects, batch->n_objects);
    if (st != PRENOM_OK) return st;
    if (!batch->params || !batch->params_lp) return fail(PRENOM_ERR_INVALID_ARG, "params and params_lp are required");
    PRENOM_LAUNCH("k_to_f16", (hipStream_t)stream,
                  launch_to_f16(batch->params, batch->params_lp,
                                prenom_batch_param_count(batch->objects, batch->n_objects), (hipStream_t)stream));
    return PRENOM_OK;
}

}  // extern "C"

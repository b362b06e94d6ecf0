/*
 * prenom_oracle.c -- plain FP64 CPU oracle for the per-object NeRF training
 * step of PRENOM (Sec. III-B "Online Object Mapping"): prior-based
 * probabilistic ray sampling (Eq. (4)-(6)), multi-resolution hash encoding and
 * shallow MLP, volume rendering (Eq. (7)), losses (Eq. (8)-(9)), the backward
 * pass and Adam.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load or call this library.  It shares
 * no code, header, table or constant generator with the GPU library, and the
 * GPU library never calls it.
 *
 * Precision and rounding.  Every quantity is computed in IEEE double from
 * FP32 inputs (promotion is exact), scalar, with no fast-math and no
 * floating-point contraction (-ffp-contract=off); fused multiply-adds appear
 * only where written explicitly.  Where a floating-point value decides an
 * integer, the decision is taken in the precision the kernels take it:
 *   - sampled CDF bins: FP64 throughout (ray transform, slab test, coarse
 *     positions, trilinear prior, prefix sums, expm1 ratio, comparison);
 *   - hash-grid cells: the rendered position is formed in FP32 as
 *     clamp(fmaf(t, d, o), 0, 1) and its cell is the floor of the exact FP64
 *     product x * N_l.
 * Everything else is plain FP64 and compared with the GPU under tolerance.
 *
 * Reduced-precision emulation (arch.mlp_dtype BF16 or FP16, arch.table_dtype
 * FP16).  The reduced-precision form rounds every operand of an MLP matrix
 * product to the 16-bit type (from its FP32 value, round to nearest even)
 * and accumulates in FP32; the forward gathers read an FP16 copy of the
 * tables.  A ReLU's on/off decision is a float deciding an integer, and
 * operand rounding moves pre-activations by ~2^-9 (BF16) of their scale, so
 * an oracle without that rounding disagrees on a fraction of the masks and
 * therefore on O(sqrt(eps)) of every gradient.  In this mode the oracle
 * rounds the same operands at the same points (weights, layer inputs, head
 * adjoint, deltas, the activations of the weight-gradient products, FP16
 * table values in the forward) and keeps everything else FP64, so it is the
 * exact result of the reduced-precision method.  Gradients reach the matrix
 * cores multiplied by the loss scale s (a power of two, so scaling is
 * exact), which keeps small FP16 values out of the subnormal range: a
 * gradient operand g is rounded as round(g s) / s.  The rounding helpers follow
 * the IEEE 754 binary16 and the bfloat16 (binary32 with 8 significand bits)
 * definitions.
 *
 * Parallelism: OpenMP over rays for per-ray work; every reduction (loss,
 * gradients) is summed serially in ray order, so results do not depend on the
 * thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_LEVELS 32
#define ORC_N_OUT 4 /* sigma + RGB head */

#define ORC_FLAG_MISS 1u
#define ORC_FLAG_ESCAPED 2u
#define ORC_FLAG_UNIFORM 4u

/* Architecture alpha (Sec. III, III-A): hash-grid levels, table size,
 * features per entry, per-level lattice resolution, MLP width and depth. */
typedef struct {
    int32_t n_levels;
    int32_t log2_table;
    int32_t n_features;
    int32_t res[ORC_MAX_LEVELS];
    int32_t width;
    int32_t hidden;
    int32_t mlp_dtype;   /* 0: FP64 products; 1: BF16 operands; 2: FP16 operands */
    int32_t table_dtype; /* 0: FP32 table values; 2: the forward reads them rounded to FP16 */
} orc_arch;

#define ORC_F32 0
#define ORC_BF16 1
#define ORC_F16 2

/* x rounded to FP32 (the value a kernel holds), then to the nearest value of
 * the 16-bit type, ties to even.  bfloat16: 8 significand bits, the binary32
 * exponent range.  binary16: 11 significand bits, normal exponents -14..15,
 * subnormal spacing 2^-24, overflow to infinity from 65520 up. */
static double orc_round16(double x, int dtype)
{
    if (dtype == ORC_F32) return x;
    const double f = (double)(float)x;
    if (f == 0.0 || isnan(f) || isinf(f)) return f;
    int e;
    frexp(f, &e);  /* |f| in [2^(e-1), 2^e) */
    if (dtype == ORC_BF16) {
        const double q = ldexp(1.0, e - 1 - 7);  /* spacing of 8 significand bits */
        return rint(f / q) * q;                  /* rint: nearest, ties to even */
    }
    if (fabs(f) >= 65520.0) return f > 0 ? INFINITY : -INFINITY;
    const int ee = (e - 1 < -14) ? -14 : e - 1;  /* subnormals share the 2^-14 binade's spacing */
    const double q = ldexp(1.0, ee - 10);
    return rint(f / q) * q;
}

typedef struct {
    int32_t n_coarse;       /* N_c */
    int32_t n_fine;         /* N_r */
    int32_t include_coarse; /* render the coarse midpoints as well */
    int32_t uniform_only;   /* stratified uniform draws, no prior */
    double eps;             /* escape threshold epsilon */
    double near_t, far_t;   /* ray interval before clipping to the box */
    double A[12];           /* world -> object (NOCS) affine, row-major 3x4 */
    const float* prior;     /* prior density grid F, [R][R][R], x fastest */
    int32_t prior_res;      /* R */
} orc_sample_cfg;

typedef struct {
    orc_arch arch;
    int32_t n_samples;  /* rendered samples per ray */
    int32_t loss_mode;  /* 0: mean squared errors, 1: the norms of Eq. (8) */
    double lambda_d;
    double lambda_sigma;
    double grad_scale;  /* emulation: gradients carry this loss scale (a power of two) when rounded */
    double jitter;          /* diagnostic, 0 = off: jitter of MLP pre-activations (orc_jitter) */
    double jitter_features; /* diagnostic, 0 = off: jitter of encoded features (orc_jitter) */
    uint64_t jitter_seed;
} orc_render_cfg;

/* ------------------------------------------------------------------------ */
/* Parameter layout: hash tables [L][T][F], then the MLP layers, each       */
/* row-major [out][in]: W_1 [W][L*F], W_2..W_D [W][W], W_out [4][W].        */
/* ------------------------------------------------------------------------ */

static int64_t orc_table_params(const orc_arch* a)
{
    return ((int64_t)a->n_levels << a->log2_table) * a->n_features;
}

static int64_t orc_mlp_params(const orc_arch* a)
{
    const int64_t in = (int64_t)a->n_levels * a->n_features;
    return (int64_t)a->width * in + (int64_t)(a->hidden - 1) * a->width * a->width +
           (int64_t)ORC_N_OUT * a->width;
}

int64_t orc_param_count(const orc_arch* a) { return orc_table_params(a) + orc_mlp_params(a); }

/* ------------------------------------------------------------------------ */
/* Prior density lookup (Sec. III-B, Eq. (3) and Eq. (4)): trilinear         */
/* interpolation over the fixed-resolution grid F.  Vertex-aligned: grid     */
/* value F[i] belongs to NOCS coordinate i/(R-1); x is clamped to [0,1].     */
/* ------------------------------------------------------------------------ */

static double orc_prior_at(const float* F, int R, const double x_in[3])
{
    int i0[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double x = x_in[a];
        if (!(x >= 0.0)) x = 0.0; /* also maps NaN to 0 */
        if (x > 1.0) x = 1.0;
        const double g = x * (double)(R - 1);
        int i = (int)floor(g);
        if (i > R - 2) i = R - 2;
        i0[a] = i;
        f[a] = g - (double)i;
    }
    double s = 0.0;
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
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

void orc_prior_lookup(const float* F, int32_t R, const double* pts, int64_t n, double* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_prior_at(F, R, pts + 3 * i);
}

/* ------------------------------------------------------------------------ */
/* Rays into the object frame and the bounding-box interval (Sec. III-B,    */
/* "Probabilistic Ray Sampling": rays are moved into the object frame with  */
/* the estimated pose and sampled inside the object's box; the box is the   */
/* NOCS unit cube of Sec. III-A).                                           */
/* ------------------------------------------------------------------------ */

static void orc_to_object(const double A[12], const float* ow, const float* dw, double o[3], double d[3])
{
    for (int r = 0; r < 3; ++r) {
        const double* a = A + 4 * r;
        o[r] = a[0] * (double)ow[0] + a[1] * (double)ow[1] + a[2] * (double)ow[2] + a[3];
        d[r] = a[0] * (double)dw[0] + a[1] * (double)dw[1] + a[2] * (double)dw[2];
    }
}

/* Slab test against [0,1]^3 intersected with [near, far].  An axis with a
 * zero direction component constrains nothing if the origin lies inside that
 * slab and rejects the ray otherwise.  Returns 1 on a hit. */
static int orc_box_interval(const double o[3], const double d[3], double near_t, double far_t,
                            double* tn, double* tf)
{
    double t_enter = -INFINITY, t_exit = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (o[a] < 0.0 || o[a] > 1.0) return 0;
            continue;
        }
        const double ta = (0.0 - o[a]) / d[a];
        const double tb = (1.0 - o[a]) / d[a];
        const double lo = ta < tb ? ta : tb;
        const double hi = ta < tb ? tb : ta;
        if (lo > t_enter) t_enter = lo;
        if (hi < t_exit) t_exit = hi;
    }
    *tn = near_t > t_enter ? near_t : t_enter;
    *tf = far_t < t_exit ? far_t : t_exit;
    return *tn < *tf;
}

/* ------------------------------------------------------------------------ */
/* Probabilistic ray sampling (Sec. III-B, Eq. (4)-(6), escape rule).       */
/*                                                                          */
/* Coarse: N_c points at equal intervals (bin midpoints) in [t_n, t_f].     */
/*   sigma_i = F(x_i);  rho_occ,i = 1 - exp(-sigma_i delta_i)     Eq. (4)   */
/*   rho_term,i = rho_occ,i prod_{j<i} (1 - rho_occ,j)            Eq. (5)   */
/*   CDF(i) = sum_{j<=i} rho_term,j / sum_{j<=N_c} rho_term,j     Eq. (6)   */
/* With S_i = sum_{j<i} sigma_j delta_j the sums telescope:                 */
/*   sum_{j<=i} rho_term,j = 1 - exp(-S_{i+1}),                            */
/* evaluated as -expm1(-S) for accuracy.  Escape: total < epsilon.          */
/* Inverse-transform draws: stratified u_k = (k + xi_k) / N_r, bin          */
/* b_k = first i with CDF_{i+1} >= u_k, linear position inside the bin.     */
/* ------------------------------------------------------------------------ */

void orc_sample(const orc_sample_cfg* c, const float* rays_o, const float* rays_d, const float* xi,
                int64_t n, double* ray_obj, double* t_out, double* dt_out, int32_t* bins,
                uint8_t* flags, double* margin)
{
    const int Nc = c->n_coarse, Nr = c->n_fine;
    const int S = Nr + (c->include_coarse ? Nc : 0);
    const int use_prior = !c->uniform_only && c->prior != NULL;

#pragma omp parallel
    {
        double* m = (double*)malloc(sizeof(double) * (size_t)(Nc > 0 ? Nc : 1));
        double* Sp = (double*)malloc(sizeof(double) * (size_t)(Nc + 1));
        double* C = (double*)malloc(sizeof(double) * (size_t)(Nc + 1));
        double* tf_k = (double*)malloc(sizeof(double) * (size_t)(Nr > 0 ? Nr : 1));
        double* ts = (double*)malloc(sizeof(double) * (size_t)(S > 0 ? S : 1));
#pragma omp for schedule(static)
        for (int64_t r = 0; r < n; ++r) {
            double o[3], d[3], tn = 0.0, tf = 0.0;
            orc_to_object(c->A, rays_o + 3 * r, rays_d + 3 * r, o, d);
            for (int a = 0; a < 3; ++a) {
                ray_obj[6 * r + a] = o[a];
                ray_obj[6 * r + 3 + a] = d[a];
            }
            double* tr = t_out + (int64_t)S * r;
            double* dtr = dt_out + (int64_t)S * r;
            int32_t* br = bins + (int64_t)Nr * r;
            const float* xr = xi + (int64_t)Nr * r;
            double min_margin = INFINITY;

            if (!orc_box_interval(o, d, c->near_t, c->far_t, &tn, &tf)) {
                for (int j = 0; j < S; ++j) tr[j] = dtr[j] = 0.0;
                for (int k = 0; k < Nr; ++k) br[k] = -1;
                flags[r] = ORC_FLAG_MISS;
                if (margin) margin[r] = min_margin;
                continue;
            }
            const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            uint8_t fl = 0;

            /* coarse midpoints and prefix sums of sigma_i * delta_i */
            const double delta = Nc > 0 ? (tf - tn) / (double)Nc : 0.0;
            for (int i = 0; i < Nc; ++i) m[i] = tn + ((double)i + 0.5) * delta;
            int escaped = 0;
            if (use_prior) {
                Sp[0] = 0.0;
                for (int i = 0; i < Nc; ++i) {
                    double x[3];
                    for (int a = 0; a < 3; ++a) {
                        x[a] = fma(m[i], d[a], o[a]);
                        if (!(x[a] >= 0.0)) x[a] = 0.0;
                        if (x[a] > 1.0) x[a] = 1.0;
                    }
                    const double sig = orc_prior_at(c->prior, c->prior_res, x);
                    const double tau = sig * delta * len;
                    Sp[i + 1] = Sp[i] + tau;
                }
                const double total = -expm1(-Sp[Nc]); /* = sum_i rho_term,i */
                escaped = total < c->eps;
                if (!escaped) {
                    const double den = expm1(-Sp[Nc]);
                    C[0] = 0.0;
                    for (int i = 1; i < Nc; ++i) C[i] = expm1(-Sp[i]) / den;
                    C[Nc] = 1.0;
                }
            }
            if (!use_prior) fl |= ORC_FLAG_UNIFORM;
            if (escaped) fl |= ORC_FLAG_ESCAPED;

            for (int k = 0; k < Nr; ++k) {
                const double u = ((double)k + (double)xr[k]) / (double)Nr;
                if (!use_prior || escaped) {
                    tf_k[k] = tn + u * (tf - tn);
                    br[k] = -1;
                } else {
                    int b = 0;
                    while (b + 1 < Nc && C[b + 1] < u) ++b; /* C[Nc] = 1 > u for xi in (0,1) */
                    const double lo = C[b], hi = C[b + 1];
                    tf_k[k] = tn + delta * ((double)b + (u - lo) / (hi - lo));
                    br[k] = b;
                    const double mg = (hi - u) < (u - lo) ? (hi - u) : (u - lo);
                    if (mg < min_margin) min_margin = mg;
                }
            }

            /* rendered set: fine draws, merged with the coarse midpoints
             * (coarse first on ties) when they are rendered too */
            if (c->include_coarse) {
                int i = 0, k = 0, j = 0;
                while (i < Nc && k < Nr) ts[j++] = (m[i] <= tf_k[k]) ? m[i++] : tf_k[k++];
                while (i < Nc) ts[j++] = m[i++];
                while (k < Nr) ts[j++] = tf_k[k++];
            } else {
                for (int k = 0; k < Nr; ++k) ts[k] = tf_k[k];
            }
            for (int j = 0; j < S; ++j) {
                tr[j] = ts[j];
                const double nxt = (j + 1 < S) ? ts[j + 1] : tf;
                dtr[j] = (nxt - ts[j]) * len;
            }
            flags[r] = fl;
            if (margin) margin[r] = min_margin;
        }
        free(m);
        free(Sp);
        free(C);
        free(tf_k);
        free(ts);
    }
}

/* ------------------------------------------------------------------------ */
/* Multi-resolution hash encoding (Sec. III-B, "Object-level NeRFs", which  */
/* uses the encoding of Mueller et al. 2022).  Level l has an integer       */
/* lattice of resolution N_l; the cell is c = min(floor(x N_l), N_l - 1),   */
/* the local coordinate f = x N_l - c.  Each of the 8 cell corners v maps   */
/* to a table row: 1:1 when (N_l+1)^3 <= T, otherwise the XOR-of-primes     */
/* spatial hash (primes 1, 2654435761, 805459861) modulo 2^32, masked to T. */
/* Features are blended with trilinear weights.                             */
/* ------------------------------------------------------------------------ */

static uint32_t orc_corner_index(int32_t N, int32_t log2T, int64_t vx, int64_t vy, int64_t vz)
{
    const int64_t T = (int64_t)1 << log2T;
    const int64_t side = (int64_t)N + 1;
    if (side * side * side <= T) return (uint32_t)(vx + side * (vy + side * vz));
    const uint32_t h = ((uint32_t)vx * 1u) ^ ((uint32_t)vy * 2654435761u) ^ ((uint32_t)vz * 805459861u);
    return h & (uint32_t)(T - 1);
}

/* One level of one point: corner indices and trilinear weights. */
static void orc_level_corners(int32_t N, int32_t log2T, const float x[3], uint32_t idx[8], double w[8])
{
    int64_t c[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        const double g = (double)x[a] * (double)N; /* exact: 24-bit by <=31-bit */
        int64_t ci = (int64_t)floor(g);
        if (ci > N - 1) ci = N - 1;
        if (ci < 0) ci = 0;
        c[a] = ci;
        f[a] = g - (double)ci;
    }
    for (int e = 0; e < 8; ++e) {
        const int ex = e & 1, ey = (e >> 1) & 1, ez = (e >> 2) & 1;
        idx[e] = orc_corner_index(N, log2T, c[0] + ex, c[1] + ey, c[2] + ez);
        w[e] = (ex ? f[0] : 1.0 - f[0]) * (ey ? f[1] : 1.0 - f[1]) * (ez ? f[2] : 1.0 - f[2]);
    }
}

/* A table value as the forward gathers read it. */
static double orc_table_value(const orc_arch* a, float v) { return orc_round16((double)v, a->table_dtype); }

/* Diagnostic only (jitter = 0 leaves x as it is): x + jitter u A, with
 * u = +-[1/2, 1) from a hash of x's bits and the seed, and A the sum of the
 * absolute terms that formed x.  Applied to every encoded feature and every
 * MLP pre-activation before it is rounded or its ReLU decided, it moves each
 * by about what the same sum computed in FP32 instead of FP64 could differ
 * by, so a ReLU signature reveals the decisions such arithmetic could change. */
static double orc_jitter(double jitter, uint64_t seed, double x, double A)
{
    if (!(jitter > 0.0)) return x;
    uint64_t b;
    memcpy(&b, &x, sizeof b);
    uint64_t h = (b ^ seed) * 0x9E3779B97F4A7C15ull;
    h ^= h >> 29;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 32;
    const double u = 0.5 + 0.5 * (double)(h >> 11) * 0x1.0p-53;
    return x + ((h & 1u) ? u : -u) * jitter * A;
}

static void orc_encode_point(const orc_arch* a, const float* table, const float x[3], double* y, double jitter,
                             uint64_t seed)
{
    const int64_t T = (int64_t)1 << a->log2_table;
    const int F = a->n_features;
    for (int l = 0; l < a->n_levels; ++l) {
        uint32_t idx[8];
        double w[8];
        orc_level_corners(a->res[l], a->log2_table, x, idx, w);
        for (int p = 0; p < F; ++p) {
            double s = 0.0, A = 0.0;
            for (int e = 0; e < 8; ++e) {
                const double term = w[e] * orc_table_value(a, table[((int64_t)l * T + idx[e]) * F + p]);
                s += term;
                A += fabs(term);
            }
            y[l * F + p] = orc_jitter(jitter, seed, s, A);
        }
    }
}

/* Encode n points: y [L][n][F] (level-major), optional idx/w [L][n][8]. */
void orc_encode(const orc_arch* a, const float* table, const float* pos, int64_t n, double* y,
                int32_t* idx_out, double* w_out)
{
    const int64_t T = (int64_t)1 << a->log2_table;
    const int F = a->n_features;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int l = 0; l < a->n_levels; ++l) {
            uint32_t idx[8];
            double w[8];
            orc_level_corners(a->res[l], a->log2_table, pos + 3 * i, idx, w);
            for (int p = 0; p < F; ++p) {
                double s = 0.0;
                for (int e = 0; e < 8; ++e) s += w[e] * orc_table_value(a, table[((int64_t)l * T + idx[e]) * F + p]);
                y[((int64_t)l * n + i) * F + p] = s;
            }
            for (int e = 0; e < 8; ++e) {
                if (idx_out) idx_out[((int64_t)l * n + i) * 8 + e] = (int32_t)idx[e];
                if (w_out) w_out[((int64_t)l * n + i) * 8 + e] = w[e];
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Shallow MLP (Sec. III-B, "Object-level NeRFs" and "Volume Rendering"):   */
/* the encoded position alone goes through D ReLU layers of width W with no */
/* biases, then a linear 4-output head; density sigma = exp(o_0), colour    */
/* c = sigmoid(o_1..3).                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    const float* W[8]; /* W[0] = W_1 ... W[hidden-1] = W_D, W[hidden] = W_out */
    int in_dim[8];
    int out_dim[8];
    int n_layers;
    int dtype;         /* operand type of the products (orc_round16) */
    double jitter;          /* diagnostic jitter of pre-activations (orc_jitter), 0 = off */
    double jitter_features; /* diagnostic jitter of encoded features, 0 = off */
    uint64_t jitter_seed;
} orc_mlp_view;

static orc_mlp_view orc_mlp_layers(const orc_arch* a, const float* mlp)
{
    orc_mlp_view v;
    const int in = a->n_levels * a->n_features;
    int64_t off = 0;
    v.n_layers = a->hidden + 1;
    v.dtype = a->mlp_dtype;
    v.jitter = 0.0;
    v.jitter_features = 0.0;
    v.jitter_seed = 0;
    for (int k = 0; k < v.n_layers; ++k) {
        v.in_dim[k] = (k == 0) ? in : a->width;
        v.out_dim[k] = (k == a->hidden) ? ORC_N_OUT : a->width;
        v.W[k] = mlp + off;
        off += (int64_t)v.in_dim[k] * v.out_dim[k];
    }
    return v;
}

/* h[k] holds the activations after layer k (h[0] = input); o = raw outputs */
static void orc_mlp_point(const orc_mlp_view* v, const double* y, double* h /* [(n_layers)][maxw] */,
                          int maxw, double o[ORC_N_OUT])
{
    memcpy(h, y, sizeof(double) * (size_t)v->in_dim[0]);
    for (int k = 0; k < v->n_layers; ++k) {
        const double* hin = h + (size_t)k * maxw;
        double* hout = (k + 1 < v->n_layers) ? h + (size_t)(k + 1) * maxw : o;
        const float* W = v->W[k];
        for (int i = 0; i < v->out_dim[k]; ++i) {
            double s = 0.0, A = 0.0;
            for (int j = 0; j < v->in_dim[k]; ++j) {
                const double term =
                    orc_round16((double)W[(int64_t)i * v->in_dim[k] + j], v->dtype) * orc_round16(hin[j], v->dtype);
                s += term;
                A += fabs(term);
            }
            s = orc_jitter(v->jitter, v->jitter_seed, s, A);
            hout[i] = (k + 1 < v->n_layers) ? (s > 0.0 ? s : 0.0) : s;
        }
    }
}

/* Raw head outputs o[n][4] for inputs y[n][in] (row-major). */
void orc_mlp_fwd(const orc_arch* a, const float* mlp, const double* y, int64_t n, double* out)
{
    const orc_mlp_view v = orc_mlp_layers(a, mlp);
    const int maxw = (a->width > a->n_levels * a->n_features) ? a->width : a->n_levels * a->n_features;
#pragma omp parallel
    {
        double* h = (double*)malloc(sizeof(double) * (size_t)maxw * (size_t)(v.n_layers + 1));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            orc_mlp_point(&v, y + (int64_t)i * v.in_dim[0], h, maxw, out + 4 * i);
        free(h);
    }
}

/* ------------------------------------------------------------------------ */
/* Prior refresh.  The category prior is the NeRF's density output over a  */
/* cubic grid of resolution R (Sec. III-A, "Normalized mesh generation"),   */
/* and during online mapping it is recomputed from the object's current    */
/* NeRF every m iterations (Sec. III-B, "Probabilistic Ray Sampling").      */
/* Vertex (i, j, k) sits at x = (i, j, k) / (R - 1), the alignment of the   */
/* prior lookup; each coordinate is rounded to FP32, the precision of the   */
/* sample positions.  out[(k R + j) R + i] = sigma = exp(o_0).              */
/* ------------------------------------------------------------------------ */
void orc_prior_refresh(const orc_arch* a, const float* params, int32_t R, double* out)
{
    const orc_mlp_view v = orc_mlp_layers(a, params + orc_table_params(a));
    const int in = a->n_levels * a->n_features;
    const int maxw = (a->width > in) ? a->width : in;
    const int64_t n = (int64_t)R * R * R;
#pragma omp parallel
    {
        double* y = (double*)malloc(sizeof(double) * (size_t)in);
        double* h = (double*)malloc(sizeof(double) * (size_t)maxw * (size_t)(v.n_layers + 1));
#pragma omp for schedule(static)
        for (int64_t p = 0; p < n; ++p) {
            const int64_t idx[3] = {p % R, (p / R) % R, p / ((int64_t)R * R)};
            float x[3];
            for (int k = 0; k < 3; ++k) x[k] = (float)((double)idx[k] / (double)(R - 1));
            double o[ORC_N_OUT];
            orc_encode_point(a, params, x, y, 0.0, 0);
            orc_mlp_point(&v, y, h, maxw, o);
            out[p] = exp(o[0]);
        }
        free(y);
        free(h);
    }
}

/* ------------------------------------------------------------------------ */
/* Canonical yaw (Sec. III-B, "Object State Canonicalization", Eq. (3)).    */
/* The object stands on the ground (z up), so only the yaw is searched.     */
/* For K yaws gamma_k = 2 pi k / K the cloud is rotated about z,            */
/* P_gamma = Rz(gamma) P; its extents S (max - min per axis) and their      */
/* midpoint C normalise it into the unit cube, Pn = (P_gamma - C) / S + 1/2 */
/* (an axis of zero extent maps to 1/2); the score of gamma_k is the sum of */
/* the prior's trilinear density over the normalised points, and the       */
/* search returns the first k of largest score.                             */
/* ------------------------------------------------------------------------ */
void orc_canonical_yaw(const float* pts, int64_t n, const float* F, int32_t R, int32_t K, double* scores,
                       double* extents, double* centers, int32_t* best)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < K; ++k) {
        const double g = 2.0 * 3.14159265358979323846 * (double)k / (double)K;
        const double c = cos(g), s = sin(g);
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t j = 0; j < n; ++j) {
            const double x = pts[3 * j], y = pts[3 * j + 1];
            const double q[3] = {c * x - s * y, s * x + c * y, (double)pts[3 * j + 2]};
            for (int a = 0; a < 3; ++a) {
                if (q[a] < lo[a]) lo[a] = q[a];
                if (q[a] > hi[a]) hi[a] = q[a];
            }
        }
        double S[3], C[3];
        for (int a = 0; a < 3; ++a) {
            S[a] = hi[a] - lo[a];
            C[a] = 0.5 * (hi[a] + lo[a]);
            extents[3 * k + a] = S[a];
            centers[3 * k + a] = C[a];
        }
        double sum = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double x = pts[3 * j], y = pts[3 * j + 1];
            const double q[3] = {c * x - s * y, s * x + c * y, (double)pts[3 * j + 2]};
            double u[3];
            for (int a = 0; a < 3; ++a) u[a] = S[a] > 0.0 ? (q[a] - C[a]) / S[a] + 0.5 : 0.5;
            sum += orc_prior_at(F, R, u);
        }
        scores[k] = sum;
    }
    int b = 0;
    for (int k = 1; k < K; ++k)
        if (scores[k] > scores[b]) b = k;
    *best = b;
}

static double orc_sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

/* ------------------------------------------------------------------------ */
/* Volume rendering (Sec. III-B, Eq. (5) and Eq. (7)).  With                */
/* alpha_j = rho_occ(p_j) = 1 - exp(-sigma_j delta_j) and                   */
/* T_j = prod_{i<j} (1 - alpha_i), the weight of sample j is                */
/* rho_term(p_j) = T_j alpha_j.  Colour and depth are the weighted sums;    */
/* the light that passes every sample (T_S) meets the background colour.    */
/* ------------------------------------------------------------------------ */

static void orc_composite_ray(int S, const double* sigma, const double* rgb, const double* t,
                              const double* dt, const double bg[3], double* w, double* T /* [S+1] */,
                              double C[3], double* D, double* A)
{
    T[0] = 1.0;
    C[0] = C[1] = C[2] = 0.0;
    *D = 0.0;
    *A = 0.0;
    for (int j = 0; j < S; ++j) {
        const double alpha = -expm1(-sigma[j] * dt[j]);
        w[j] = T[j] * alpha;
        T[j + 1] = T[j] * exp(-sigma[j] * dt[j]);
        for (int c = 0; c < 3; ++c) C[c] += w[j] * rgb[3 * j + c];
        *D += w[j] * t[j];
        *A += w[j];
    }
    for (int c = 0; c < 3; ++c) C[c] += T[S] * bg[c];
}

/* Adjoint of orc_composite_ray.  gC, gD, gA: upstream gradients of colour,
 * depth and opacity.  Derived from Eq. (7): for k > j,
 * d w_k / d sigma_j = -delta_j w_k, d w_j / d sigma_j = delta_j T_{j+1},
 * d T_S / d sigma_j = -delta_j T_S. */
static void orc_composite_ray_bwd(int S, const double* rgb, const double* t, const double* dt,
                                  const double bg[3], const double* w, const double* T,
                                  const double gC[3], double gD, double gA, double* dsigma,
                                  double* drgb)
{
    const double bg_term = T[S] * (gC[0] * bg[0] + gC[1] * bg[1] + gC[2] * bg[2]);
    double suffix = 0.0; /* sum_{k>j} w_k a_k */
    for (int j = S - 1; j >= 0; --j) {
        const double a = gC[0] * rgb[3 * j] + gC[1] * rgb[3 * j + 1] + gC[2] * rgb[3 * j + 2] +
                         gD * t[j] + gA;
        dsigma[j] = dt[j] * (T[j + 1] * a - suffix - bg_term);
        for (int c = 0; c < 3; ++c) drgb[3 * j + c] = w[j] * gC[c];
        suffix += w[j] * a;
    }
}

/* Batched composite for closed-form checks: arrays [n][S] and [n][S][3]. */
void orc_composite_fwd(int64_t n, int32_t S, const double* sigma, const double* rgb, const double* t,
                       const double* dt, const double* bg, double* C, double* D, double* A,
                       double* w_out, double* T_out)
{
    double* w = (double*)malloc(sizeof(double) * (size_t)S);
    double* T = (double*)malloc(sizeof(double) * (size_t)(S + 1));
    for (int64_t r = 0; r < n; ++r) {
        orc_composite_ray(S, sigma + r * S, rgb + 3 * r * S, t + r * S, dt + r * S, bg + 3 * r, w, T,
                          C + 3 * r, D + r, A + r);
        if (w_out) memcpy(w_out + r * S, w, sizeof(double) * (size_t)S);
        if (T_out) memcpy(T_out + r * (S + 1), T, sizeof(double) * (size_t)(S + 1));
    }
    free(w);
    free(T);
}

void orc_composite_bwd(int64_t n, int32_t S, const double* sigma, const double* rgb, const double* t,
                       const double* dt, const double* bg, const double* gC, const double* gD,
                       const double* gA, double* dsigma, double* drgb)
{
    double* w = (double*)malloc(sizeof(double) * (size_t)S);
    double* T = (double*)malloc(sizeof(double) * (size_t)(S + 1));
    for (int64_t r = 0; r < n; ++r) {
        double C[3], D, A;
        orc_composite_ray(S, sigma + r * S, rgb + 3 * r * S, t + r * S, dt + r * S, bg + 3 * r, w, T, C,
                          &D, &A);
        orc_composite_ray_bwd(S, rgb + 3 * r * S, t + r * S, dt + r * S, bg + 3 * r, w, T, gC + 3 * r,
                              gD[r], gA ? gA[r] : 0.0, dsigma + r * S, drgb + 3 * r * S);
    }
    free(w);
    free(T);
}

/* ------------------------------------------------------------------------ */
/* Losses (Sec. III-B, Eq. (8) and Eq. (9)).  R_o: mask = 1, R_b: mask = 0. */
/* The colour target of a background ray is its background colour (the     */
/* random colour C_rand of Eq. (8)); tgt_rgb carries it for every ray.      */
/*  mode 0 (mean squared):                                                  */
/*   L = 1/(3n) sum_k |C^_k - C_k|^2 + l_d/n sum_{R_o} (D^_k - D_k)^2       */
/*       + l_s/n sum_{R_b} sum_j sigma_kj                                   */
/*  mode 1 (the norms of Eq. (8)):                                          */
/*   L = sum_k |C^_k - C_k|_2 + l_d sum_{R_o} |D^_k - D_k|                  */
/*       + l_s sum_{R_b} sum_j |sigma_kj|                                   */
/* Per-ray loss and the gradient wrt the ray's colour and depth; the        */
/* density term's gradient per sample is returned in dsig_extra.            */
/* ------------------------------------------------------------------------ */

static double orc_ray_loss(const orc_render_cfg* c, int64_t n, const double Ch[3], double Dh,
                           const float* tgt, float tdepth, int is_obj, double sigma_sum, double gC[3],
                           double* gD, double* dsig_extra)
{
    const double e[3] = {Ch[0] - (double)tgt[0], Ch[1] - (double)tgt[1], Ch[2] - (double)tgt[2]};
    const double ed = Dh - (double)tdepth;
    double L;
    if (c->loss_mode == 0) {
        const double inv = 1.0 / (double)n;
        L = (e[0] * e[0] + e[1] * e[1] + e[2] * e[2]) / (3.0 * (double)n);
        for (int k = 0; k < 3; ++k) gC[k] = 2.0 * e[k] / (3.0 * (double)n);
        *gD = 0.0;
        *dsig_extra = 0.0;
        if (is_obj) {
            L += c->lambda_d * ed * ed * inv;
            *gD = 2.0 * c->lambda_d * ed * inv;
        } else {
            L += c->lambda_sigma * sigma_sum * inv;
            *dsig_extra = c->lambda_sigma * inv;
        }
    } else {
        const double nrm = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        L = nrm;
        for (int k = 0; k < 3; ++k) gC[k] = nrm > 0.0 ? e[k] / nrm : 0.0;
        *gD = 0.0;
        *dsig_extra = 0.0;
        if (is_obj) {
            L += c->lambda_d * fabs(ed);
            *gD = c->lambda_d * (ed > 0.0 ? 1.0 : (ed < 0.0 ? -1.0 : 0.0));
        } else {
            L += c->lambda_sigma * sigma_sum; /* sigma = exp(.) > 0 */
            *dsig_extra = c->lambda_sigma;
        }
    }
    return L;
}

/* ------------------------------------------------------------------------ */
/* Forward and backward of the whole rendering path for one ray.            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int S, L, F, in_dim, maxw, n_layers, width;
    double *y;       /* [S][in] encoded features */
    double *h;       /* [S][n_layers+1][maxw] activations */
    double *o;       /* [S][4] raw outputs */
    double *sigma;   /* [S] */
    double *rgb;     /* [S][3] */
    double *tt;      /* [S] */
    double *dtt;     /* [S] */
    double *w;       /* [S] */
    double *T;       /* [S+1] */
    float *x;        /* [S][3] FP32 positions */
} orc_ray_state;

static void orc_state_alloc(orc_ray_state* s, const orc_arch* a, int S)
{
    s->S = S;
    s->L = a->n_levels;
    s->F = a->n_features;
    s->in_dim = s->L * s->F;
    s->maxw = a->width > s->in_dim ? a->width : s->in_dim;
    s->n_layers = a->hidden + 1;
    s->width = a->width;
    s->y = (double*)malloc(sizeof(double) * (size_t)S * (size_t)s->in_dim);
    s->h = (double*)malloc(sizeof(double) * (size_t)S * (size_t)(s->n_layers + 1) * (size_t)s->maxw);
    s->o = (double*)malloc(sizeof(double) * (size_t)S * 4);
    s->sigma = (double*)malloc(sizeof(double) * (size_t)S);
    s->rgb = (double*)malloc(sizeof(double) * (size_t)S * 3);
    s->tt = (double*)malloc(sizeof(double) * (size_t)S);
    s->dtt = (double*)malloc(sizeof(double) * (size_t)S);
    s->w = (double*)malloc(sizeof(double) * (size_t)S);
    s->T = (double*)malloc(sizeof(double) * (size_t)(S + 1));
    s->x = (float*)malloc(sizeof(float) * (size_t)S * 3);
}

static void orc_state_free(orc_ray_state* s)
{
    free(s->y); free(s->h); free(s->o); free(s->sigma); free(s->rgb);
    free(s->tt); free(s->dtt); free(s->w); free(s->T); free(s->x);
}

/* Sample position in the precision the kernels use: FP32 fma, clamped. */
static void orc_position(const float* ro, float t, float x[3])
{
    for (int a = 0; a < 3; ++a) {
        float v = fmaf(t, ro[3 + a], ro[a]);
        if (v < 0.0f) v = 0.0f;
        if (v > 1.0f) v = 1.0f;
        x[a] = v;
    }
}

/* Positions of every rendered sample, [n][S][3] FP32. */
void orc_positions(const float* ray_obj, const float* t, int64_t n, int32_t S, float* pos)
{
    for (int64_t r = 0; r < n; ++r)
        for (int j = 0; j < S; ++j) orc_position(ray_obj + 6 * r, t[r * S + j], pos + (r * S + j) * 3);
}

/* Forward pass of one (non-missed) ray: encode, MLP, composite. */
static void orc_ray_forward(const orc_render_cfg* c, const float* params, const orc_mlp_view* mv,
                            const float* ro, const float* t, const float* dt, const double bg[3],
                            orc_ray_state* s, double C[3], double* D, double* A)
{
    const int S = s->S;
    for (int j = 0; j < S; ++j) {
        orc_position(ro, t[j], s->x + 3 * j);
        orc_encode_point(&c->arch, params, s->x + 3 * j, s->y + (size_t)j * s->in_dim, mv->jitter_features,
                         mv->jitter_seed);
        orc_mlp_point(mv, s->y + (size_t)j * s->in_dim, s->h + (size_t)j * (s->n_layers + 1) * s->maxw,
                      s->maxw, s->o + 4 * j);
        s->sigma[j] = exp(s->o[4 * j]);
        for (int k = 0; k < 3; ++k) s->rgb[3 * j + k] = orc_sigmoid(s->o[4 * j + 1 + k]);
        s->tt[j] = (double)t[j];
        s->dtt[j] = (double)dt[j];
    }
    orc_composite_ray(S, s->sigma, s->rgb, s->tt, s->dtt, bg, s->w, s->T, C, D, A);
}

/* FNV-1a fingerprint of every ReLU on/off decision of a ray; lets a finite-
 * difference check detect perturbations that cross a ReLU kink. */
static uint64_t orc_relu_signature(const orc_ray_state* s)
{
    uint64_t hsh = 1469598103934665603ull;
    for (int j = 0; j < s->S; ++j)
        for (int k = 1; k < s->n_layers; ++k) { /* hidden activations h_1 .. h_D */
            const double* hk = s->h + ((size_t)j * (s->n_layers + 1) + k) * s->maxw;
            for (int i = 0; i < s->width; ++i) {
                hsh ^= (uint64_t)(hk[i] > 0.0);
                hsh *= 1099511628211ull;
            }
        }
    return hsh;
}

void orc_render_fwd(const orc_render_cfg* c, const float* params, const float* ray_obj, const float* t,
                    const float* dt, const uint8_t* flags, int64_t n, const float* bg,
                    const float* tgt_rgb, const float* tgt_depth, const uint8_t* mask, double* rgb,
                    double* depth, double* opacity, double* ray_loss, double* loss, double* sample_out,
                    uint64_t* relu_sig)
{
    const int S = c->n_samples;
    orc_mlp_view mv = orc_mlp_layers(&c->arch, params + orc_table_params(&c->arch));
    mv.jitter = c->jitter;
    mv.jitter_features = c->jitter_features;
    mv.jitter_seed = c->jitter_seed;
    double* per_ray = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel
    {
        orc_ray_state s;
        orc_state_alloc(&s, &c->arch, S);
#pragma omp for schedule(dynamic, 16)
        for (int64_t r = 0; r < n; ++r) {
            double bgc[3] = {0.0, 0.0, 0.0};
            if (bg)
                for (int k = 0; k < 3; ++k) bgc[k] = (double)bg[3 * r + k];
            double C[3], D, A, sigma_sum = 0.0;
            if (flags[r] & ORC_FLAG_MISS) {
                for (int k = 0; k < 3; ++k) C[k] = bgc[k];
                D = 0.0;
                A = 0.0;
                if (sample_out)
                    for (int j = 0; j < 4 * S; ++j) sample_out[(int64_t)r * S * 4 + j] = 0.0;
                if (relu_sig) relu_sig[r] = 0;
            } else {
                orc_ray_forward(c, params, &mv, ray_obj + 6 * r, t + (int64_t)r * S, dt + (int64_t)r * S,
                                bgc, &s, C, &D, &A);
                if (relu_sig) relu_sig[r] = orc_relu_signature(&s);
                for (int j = 0; j < S; ++j) sigma_sum += s.sigma[j];
                if (sample_out)
                    for (int j = 0; j < S; ++j) {
                        double* so = sample_out + ((int64_t)r * S + j) * 4;
                        so[0] = s.sigma[j];
                        so[1] = s.rgb[3 * j];
                        so[2] = s.rgb[3 * j + 1];
                        so[3] = s.rgb[3 * j + 2];
                    }
            }
            for (int k = 0; k < 3; ++k) rgb[3 * r + k] = C[k];
            depth[r] = D;
            opacity[r] = A;
            if (tgt_rgb) {
                double gC[3], gD, ex;
                per_ray[r] = orc_ray_loss(c, n, C, D, tgt_rgb + 3 * r, tgt_depth ? tgt_depth[r] : 0.0f,
                                          mask ? mask[r] != 0 : 1, sigma_sum, gC, &gD, &ex);
            }
        }
        orc_state_free(&s);
    }
    if (tgt_rgb) {
        double total = 0.0;
        for (int64_t r = 0; r < n; ++r) total += per_ray[r];
        if (ray_loss) memcpy(ray_loss, per_ray, sizeof(double) * (size_t)n);
        if (loss) *loss = total;
    }
    free(per_ray);
}

/* Backward of the rendering path; gradients are ADDED to grads [n_params].
 * Upstream gradients d_rgb [n][3] / d_depth [n] / d_opacity [n] replace the
 * loss gradient when d_rgb is not NULL (the density term then contributes
 * nothing). */
void orc_render_bwd(const orc_render_cfg* c, const float* params, const float* ray_obj, const float* t,
                    const float* dt, const uint8_t* flags, int64_t n, const float* bg,
                    const float* tgt_rgb, const float* tgt_depth, const uint8_t* mask,
                    const float* d_rgb, const float* d_depth, const float* d_opacity, double* grads)
{
    const orc_arch* a = &c->arch;
    const int S = c->n_samples;
    const int L = a->n_levels, F = a->n_features, in_dim = L * F;
    const int64_t T = (int64_t)1 << a->log2_table;
    const int64_t n_table = orc_table_params(a);
    const int64_t n_mlp = orc_mlp_params(a);
    const orc_mlp_view mv = orc_mlp_layers(a, params + n_table);
    const int64_t chunk = 256;
    double* dW = (double*)calloc((size_t)(chunk * n_mlp), sizeof(double));  /* per ray of chunk */
    double* dY = (double*)calloc((size_t)(chunk * S * in_dim), sizeof(double));
    float* X = (float*)calloc((size_t)(chunk * S * 3), sizeof(float));
    uint8_t* live = (uint8_t*)calloc((size_t)chunk, 1);

    for (int64_t r0 = 0; r0 < n; r0 += chunk) {
        const int64_t r1 = (r0 + chunk < n) ? r0 + chunk : n;
#pragma omp parallel
        {
            orc_ray_state s;
            orc_state_alloc(&s, a, S);
            double* dsig = (double*)malloc(sizeof(double) * (size_t)S);
            double* drgb = (double*)malloc(sizeof(double) * (size_t)S * 3);
            double* dh = (double*)malloc(sizeof(double) * (size_t)(s.maxw));
            double* dh2 = (double*)malloc(sizeof(double) * (size_t)(s.maxw));
            double* gr = (double*)malloc(sizeof(double) * (size_t)(s.maxw > ORC_N_OUT ? s.maxw : ORC_N_OUT));
#pragma omp for schedule(dynamic, 4)
            for (int64_t r = r0; r < r1; ++r) {
                const int64_t q = r - r0;
                double* dWr = dW + q * n_mlp;
                memset(dWr, 0, sizeof(double) * (size_t)n_mlp);
                live[q] = !(flags[r] & ORC_FLAG_MISS);
                if (!live[q]) continue;
                double bgc[3] = {0.0, 0.0, 0.0};
                if (bg)
                    for (int k = 0; k < 3; ++k) bgc[k] = (double)bg[3 * r + k];
                double C[3], D, A;
                orc_ray_forward(c, params, &mv, ray_obj + 6 * r, t + r * S, dt + r * S, bgc, &s, C, &D, &A);
                double gC[3], gD, gA = 0.0, extra = 0.0;
                if (d_rgb) {
                    for (int k = 0; k < 3; ++k) gC[k] = (double)d_rgb[3 * r + k];
                    gD = d_depth ? (double)d_depth[r] : 0.0;
                    gA = d_opacity ? (double)d_opacity[r] : 0.0;
                } else {
                    double sigma_sum = 0.0;
                    for (int j = 0; j < S; ++j) sigma_sum += s.sigma[j];
                    orc_ray_loss(c, n, C, D, tgt_rgb + 3 * r, tgt_depth ? tgt_depth[r] : 0.0f,
                                 mask ? mask[r] != 0 : 1, sigma_sum, gC, &gD, &extra);
                }
                orc_composite_ray_bwd(S, s.rgb, s.tt, s.dtt, bgc, s.w, s.T, gC, gD, gA, dsig, drgb);
                for (int j = 0; j < S; ++j) {
                    dsig[j] += extra;
                    /* head: sigma = exp(o0), c = sigmoid(o_k) */
                    double dout[ORC_N_OUT];
                    dout[0] = dsig[j] * s.sigma[j];
                    for (int k = 0; k < 3; ++k)
                        dout[1 + k] = drgb[3 * j + k] * s.rgb[3 * j + k] * (1.0 - s.rgb[3 * j + k]);
                    const double* hj = s.h + (size_t)j * (s.n_layers + 1) * s.maxw;
                    /* layer-by-layer adjoint, last layer first */
                    const double* g = dout;
                    int64_t off = n_mlp;
                    for (int k = s.n_layers - 1; k >= 0; --k) {
                        const int in = mv.in_dim[k], out = mv.out_dim[k];
                        off -= (int64_t)in * out;
                        const double* hin = hj + (size_t)k * s.maxw;
                        const float* W = mv.W[k];
                        double* gout = (k > 0) ? dh2 : (dY + (q * S + j) * in_dim);
                        const int dt = mv.dtype;
                        const double gs = (dt == ORC_F32 || !(c->grad_scale > 0.0)) ? 1.0 : c->grad_scale;
                        for (int i = 0; i < out; ++i) gr[i] = orc_round16(g[i] * gs, dt) / gs;
                        for (int i = 0; i < out; ++i)
                            for (int jj = 0; jj < in; ++jj)
                                dWr[off + (int64_t)i * in + jj] += gr[i] * orc_round16(hin[jj], dt);
                        for (int jj = 0; jj < in; ++jj) {
                            double acc = 0.0;
                            for (int i = 0; i < out; ++i) acc += orc_round16((double)W[(int64_t)i * in + jj], dt) * gr[i];
                            /* ReLU' of the layer below (hin > 0 <=> pre-activation > 0) */
                            gout[jj] = (k > 0) ? (hin[jj] > 0.0 ? acc : 0.0) : acc;
                        }
                        if (k > 0) {
                            memcpy(dh, dh2, sizeof(double) * (size_t)in);
                            g = dh;
                        }
                    }
                    memcpy(X + (q * S + j) * 3, s.x + 3 * j, sizeof(float) * 3);
                }
            }
            free(dsig);
            free(drgb);
            free(dh);
            free(dh2);
            free(gr);
            orc_state_free(&s);
        }
        /* serial accumulation in ray order */
        for (int64_t r = r0; r < r1; ++r) {
            const int64_t q = r - r0;
            if (!live[q]) continue;
            for (int64_t p = 0; p < n_mlp; ++p) grads[n_table + p] += dW[q * n_mlp + p];
            for (int j = 0; j < S; ++j) {
                const double* dy = dY + (q * S + j) * in_dim;
                const float* x = X + (q * S + j) * 3;
                for (int l = 0; l < L; ++l) {
                    uint32_t idx[8];
                    double w[8];
                    orc_level_corners(a->res[l], a->log2_table, x, idx, w);
                    for (int e = 0; e < 8; ++e)
                        for (int p = 0; p < F; ++p)
                            grads[((int64_t)l * T + idx[e]) * F + p] += w[e] * dy[l * F + p];
                }
            }
        }
    }
    free(dW);
    free(dY);
    free(X);
    free(live);
}

/* ------------------------------------------------------------------------ */
/* Adam (Sec. III-B, last paragraph: the loss is back-propagated and the    */
/* NeRF parameters are optimised with Adam).  Bias-corrected, dense.        */
/* ------------------------------------------------------------------------ */

void orc_adam(int64_t n, const float* p, const float* g, const float* m, const float* v, double lr,
              double b1, double b2, double eps, int64_t step, double* p_out, double* m_out, double* v_out)
{
    const double c1 = 1.0 - pow(b1, (double)step);
    const double c2 = 1.0 - pow(b2, (double)step);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double gi = (double)g[i];
        const double mi = b1 * (double)m[i] + (1.0 - b1) * gi;
        const double vi = b2 * (double)v[i] + (1.0 - b2) * gi * gi;
        const double mh = mi / c1;
        const double vh = vi / c2;
        p_out[i] = (double)p[i] - lr * mh / (sqrt(vh) + eps);
        m_out[i] = mi;
        v_out[i] = vi;
    }
}

/* Element-wise orc_round16 (for the pins of the rounding rule). */
void orc_round16_array(const double* x, int64_t n, int32_t dtype, double* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_round16(x[i], dtype);
}

/* Thread count of the per-ray parallel loops (timing only; results do not
 * depend on it). */
void orc_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int32_t orc_max_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * CPU oracle for the FilterGS per-frame path.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. The product path (the
 * HIP library and its Python binding) never calls it and shares no code with
 * it.
 *
 * What it computes, one unit at a time, in plain loops:
 *   filter      Sec. 3.2: frustum, R&L filter (R_2D = 3*sigma <= tau_R, leaf
 *               exemption) and Ancestor filter over each node's ancestor path,
 *               evaluated independently for every node (the traversal-free
 *               form, Eq. (4)); selection compacted in ascending node order.
 *   preprocess  Sec. 3.1 Eq. (1) Gaussians projected to 2D (EWA), conic,
 *               view-dependent SH colour; Sec. 3.3 shrink radius
 *               r = sqrt(2 * lambda_max * ln(alpha0 / tau)) bounded by 3 sigma,
 *               tile rectangle and tile count.
 *   sort        Gaussian-tile key/value pairs (Sec. 3.3), key = tile << 32 |
 *               depth bits, sorted by (key, value); per-tile ranges.
 *   render      Eq. (2): front-to-back blending per pixel over its tile's range.
 *
 * Numeric contract (the paper fixes no precision; every stage takes discrete
 * decisions from floating point, so the oracle works in IEEE binary32 with
 * the operation order written here, round-to-nearest, no contraction
 * (-ffp-contract=off), correctly rounded division and square root, and two
 * transcendental functions defined below from published methods).
 *
 * Threads: built with -fopenmp (the timing build), the loops over nodes,
 * selected Gaussians and tiles whose iterations write disjoint outputs are
 * shared among threads. Each unit is still evaluated by the same operations
 * in the same order, so results are bit-identical to the plain build.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct fgo_tree {
    int64_t n;               /* nodes */
    int32_t sh_degree;       /* 0..3 */
    int32_t pad;
    const float* mean;       /* [3][n] */
    const float* scale;      /* [3][n] linear */
    const float* quat;       /* [4][n] w,x,y,z */
    const float* opacity;    /* [n] */
    const float* sh;         /* [n][K][3] */
    const int32_t* parent;   /* [n], -1 root */
    const uint8_t* flags;    /* [n], bit0 leaf */
} fgo_tree;

typedef struct fgo_camera {
    float R[9];
    float t[3];
    float campos[3];
    float fx, fy, cx, cy;
    int32_t width, height;
    float znear, kx, ky;
    uint32_t tile_base;
} fgo_camera;

/* ---------------------------------------------------------------------- */
/* transcendental functions                                               */
/* ---------------------------------------------------------------------- */

/* exp(x) for x <= 88 (0 below -87, where the true value approaches the
 * smallest normal float). Cody & Waite (1980) argument reduction
 * x = n*ln2 + r with ln2 split into a 16-bit head and a tail, then the
 * degree-7 Taylor polynomial of e^r in Horner form with fused multiply-add,
 * then scaling by 2^n. */
float fgo_exp(float x)
{
    const float log2e = 1.44269504f;
    const float ln2_hi = 0.693145751953125f;
    const float ln2_lo = 1.42860677e-06f;
    if (x < -87.0f) return 0.0f;
    float n = rintf(x * log2e);
    float r = fmaf(-n, ln2_hi, x);
    r = fmaf(-n, ln2_lo, r);
    float p = 1.0f / 5040.0f;
    p = fmaf(p, r, 1.0f / 720.0f);
    p = fmaf(p, r, 1.0f / 120.0f);
    p = fmaf(p, r, 1.0f / 24.0f);
    p = fmaf(p, r, 1.0f / 6.0f);
    p = fmaf(p, r, 0.5f);
    p = fmaf(p, r, 1.0f);
    p = fmaf(p, r, 1.0f);
    return ldexpf(p, (int)n);
}

/* ln(x) for x > 1. x = m * 2^e with m in [sqrt(1/2), sqrt(2)); with
 * s = (m - 1) / (m + 1), ln m = 2 atanh(s) = 2s (1 + s^2/3 + ... + s^8/9);
 * ln x = e*ln2 (head + tail) + ln m. The quotient s is carried as s + slo:
 * slo is the exact residual f - s*(m + 1) (two fused multiply-adds, m + 1
 * split into its rounded value and the rounding error) divided by m + 1. */
float fgo_log(float x)
{
    const float ln2_hi = 0.693145751953125f;
    const float ln2_lo = 1.42860677e-06f;
    int e;
    float m = frexpf(x, &e);
    if (m < 0.70710678f) {
        m = m * 2.0f;
        e = e - 1;
    }
    float f = m - 1.0f;
    float d = m + 1.0f;
    float s = f / d;
    float dlo = m - (d - 1.0f);
    float res = fmaf(-s, d, f);
    res = fmaf(-s, dlo, res);
    float slo = res / d;
    float s2 = s * s;
    float q = 1.0f / 9.0f;
    q = fmaf(q, s2, 1.0f / 7.0f);
    q = fmaf(q, s2, 1.0f / 5.0f);
    q = fmaf(q, s2, 1.0f / 3.0f);
    q = q * s2;
    float s_2 = 2.0f * s;
    float lm = s_2 + fmaf(s_2, q, 2.0f * slo);
    float ef = (float)e;
    return fmaf(ef, ln2_hi, fmaf(ef, ln2_lo, lm));
}

/* ---------------------------------------------------------------------- */
/* per-Gaussian geometry                                                  */
/* ---------------------------------------------------------------------- */

/* x_c = R x_w + t (camera space), each row summed left to right. */
static void to_camera(const fgo_camera* c, float mx, float my, float mz, float pc[3])
{
    for (int i = 0; i < 3; i++)
        pc[i] = ((c->R[3 * i + 0] * mx + c->R[3 * i + 1] * my) + c->R[3 * i + 2] * mz) + c->t[i];
}

/* In-frustum test: in front of the near plane and the centre inside the
 * guard band |x| <= kx z, |y| <= ky z. NaN fails every comparison. */
static int in_frustum(const fgo_camera* c, const float pc[3])
{
    return pc[2] > c->znear && fabsf(pc[0]) <= c->kx * pc[2] && fabsf(pc[1]) <= c->ky * pc[2];
}

/* 3D covariance Sigma = M M^T, M = R(q/|q|) diag(s) (Sec. 3.1).
 * Output the 6 unique entries s00 s01 s02 s11 s12 s22. */
static void covariance3d(const float s[3], const float q[4], float S[6])
{
    float norm = sqrtf(((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]);
    float w = q[0] / norm, x = q[1] / norm, y = q[2] / norm, z = q[3] / norm;
    float Rm[3][3];
    Rm[0][0] = 1.0f - 2.0f * (y * y + z * z);
    Rm[0][1] = 2.0f * (x * y - w * z);
    Rm[0][2] = 2.0f * (x * z + w * y);
    Rm[1][0] = 2.0f * (x * y + w * z);
    Rm[1][1] = 1.0f - 2.0f * (x * x + z * z);
    Rm[1][2] = 2.0f * (y * z - w * x);
    Rm[2][0] = 2.0f * (x * z - w * y);
    Rm[2][1] = 2.0f * (y * z + w * x);
    Rm[2][2] = 1.0f - 2.0f * (x * x + y * y);
    float M[3][3];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) M[i][j] = Rm[i][j] * s[j];
    int k = 0;
    for (int i = 0; i < 3; i++)
        for (int j = i; j < 3; j++)
            S[k++] = (M[i][0] * M[j][0] + M[i][1] * M[j][1]) + M[i][2] * M[j][2];
}

/* EWA projection: Sigma_2D = T Sigma T^T with T = J W, J the Jacobian of the
 * pinhole map at the camera-space centre, W the world->camera rotation;
 * the 0.3 px^2 low-pass dilation is added to the diagonal. Returns a, b, c
 * of [[a, b], [b, c]]. */
static void covariance2d(const fgo_camera* c, const float pc[3], const float S[6], float* a, float* b, float* cc)
{
    float x = pc[0], y = pc[1], z = pc[2];
    float j00 = c->fx / z;
    float j02 = -(c->fx * x) / (z * z);
    float j11 = c->fy / z;
    float j12 = -(c->fy * y) / (z * z);
    const float* W = c->R;
    float T[2][3];
    for (int j = 0; j < 3; j++) {
        T[0][j] = j00 * W[0 * 3 + j] + j02 * W[2 * 3 + j];
        T[1][j] = j11 * W[1 * 3 + j] + j12 * W[2 * 3 + j];
    }
    float Sg[3][3] = {{S[0], S[1], S[2]}, {S[1], S[3], S[4]}, {S[2], S[4], S[5]}};
    float U[2][3];
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 3; j++)
            U[i][j] = (T[i][0] * Sg[0][j] + T[i][1] * Sg[1][j]) + T[i][2] * Sg[2][j];
    float s00 = (U[0][0] * T[0][0] + U[0][1] * T[0][1]) + U[0][2] * T[0][2];
    float s01 = (U[0][0] * T[1][0] + U[0][1] * T[1][1]) + U[0][2] * T[1][2];
    float s11 = (U[1][0] * T[1][0] + U[1][1] * T[1][1]) + U[1][2] * T[1][2];
    *a = s00 + 0.3f;
    *b = s01;
    *cc = s11 + 0.3f;
}

/* Largest eigenvalue of [[a, b], [b, c]] (a variance), cancellation-free. */
static float lambda_max(float a, float b, float c)
{
    float h = 0.5f * (a - c);
    return 0.5f * (a + c) + sqrtf(h * h + b * b);
}

static float node_radius3(const fgo_tree* t, const fgo_camera* c, int64_t n, const float pc[3])
{
    float s[3] = {t->scale[n], t->scale[t->n + n], t->scale[2 * t->n + n]};
    float q[4] = {t->quat[n], t->quat[t->n + n], t->quat[2 * t->n + n], t->quat[3 * t->n + n]};
    float S[6], a, b, cc;
    covariance3d(s, q, S);
    covariance2d(c, pc, S, &a, &b, &cc);
    return 3.0f * sqrtf(lambda_max(a, b, cc));
}

/* ---------------------------------------------------------------------- */
/* filter (Sec. 3.2)                                                      */
/* ---------------------------------------------------------------------- */

static int node_frustum(const fgo_tree* t, const fgo_camera* c, int64_t n, float pc[3])
{
    to_camera(c, t->mean[n], t->mean[t->n + n], t->mean[2 * t->n + n], pc);
    return in_frustum(c, pc);
}

/* Per-node predicates, bit 0 = in frustum, bit 1 = small (in frustum and
 * R_2D <= tau_R), bit 2 = passes R&L (in frustum and (leaf or small)),
 * bit 3 = selected (R&L and no ancestor passes R&L). */
void fgo_node_predicates(const fgo_tree* t, const fgo_camera* c, float tau_R, uint8_t* out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < t->n; n++) {
        float pc[3];
        int f = node_frustum(t, c, n, pc);
        int small = f && node_radius3(t, c, n, pc) <= tau_R;
        int leaf = t->flags[n] & 1;
        int rl = f && (leaf || small);
        out[n] = (uint8_t)(f | (small << 1) | (rl << 2));
    }
    uint8_t* selv = (uint8_t*)malloc((size_t)(t->n > 0 ? t->n : 1));
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < t->n; n++) {
        int sel = (out[n] >> 2) & 1;
        for (int32_t a = t->parent[n]; sel && a >= 0; a = t->parent[a])
            if ((out[a] >> 2) & 1) sel = 0;
        selv[n] = (uint8_t)sel;
    }
    for (int64_t n = 0; n < t->n; n++) out[n] |= (uint8_t)(selv[n] << 3);
    free(selv);
}

/* Threads for the loops marked above (the -fopenmp build); returns the count
 * that will be used (always 1 in the plain build). */
int fgo_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* R&L + Ancestor filter for every node independently, then the selected
 * node ids in ascending order. sel_mask [n] (0/1), sel_idx [n] capacity. */
int64_t fgo_filter(const fgo_tree* t, const fgo_camera* c, float tau_R, uint8_t* sel_mask, uint32_t* sel_idx)
{
    uint8_t* pred = (uint8_t*)malloc((size_t)t->n);
    fgo_node_predicates(t, c, tau_R, pred);
    int64_t k = 0;
    for (int64_t n = 0; n < t->n; n++) {
        sel_mask[n] = (pred[n] >> 3) & 1;
        if (sel_mask[n]) sel_idx[k++] = (uint32_t)n;
    }
    free(pred);
    return k;
}

/* The filter result for a list of nodes only (sampled checks on large
 * trees): returns the selection bit of each listed node. */
void fgo_filter_nodes(const fgo_tree* t, const fgo_camera* c, float tau_R, const int64_t* nodes, int64_t m,
                      uint8_t* out)
{
    for (int64_t i = 0; i < m; i++) {
        int64_t n = nodes[i];
        float pc[3];
        int rl_self;
        int f = node_frustum(t, c, n, pc);
        int leaf = t->flags[n] & 1;
        rl_self = f && (leaf || node_radius3(t, c, n, pc) <= tau_R);
        int sel = rl_self;
        for (int32_t a = t->parent[n]; sel && a >= 0; a = t->parent[a]) {
            float pa[3];
            int fa = node_frustum(t, c, a, pa);
            int rla = fa && ((t->flags[a] & 1) || node_radius3(t, c, a, pa) <= tau_R);
            if (rla) sel = 0;
        }
        out[i] = (uint8_t)sel;
    }
}

/* ---------------------------------------------------------------------- */
/* preprocess (Sec. 3.1 projection and colour, Sec. 3.3 shrink)          */
/* ---------------------------------------------------------------------- */

/* Real spherical harmonics up to degree 3, orthonormal on the sphere,
 * closed-form Cartesian polynomials of the unit direction (x, y, z);
 * coefficient order (l, m = -l..l). */
static void sh_basis(int degree, float x, float y, float z, float* Y)
{
    Y[0] = 0.28209479177387814f;
    if (degree < 1) return;
    Y[1] = 0.48860251190291992f * y;
    Y[2] = 0.48860251190291992f * z;
    Y[3] = 0.48860251190291992f * x;
    if (degree < 2) return;
    Y[4] = 1.0925484305920792f * (x * y);
    Y[5] = 1.0925484305920792f * (y * z);
    Y[6] = 0.31539156525252005f * (3.0f * (z * z) - 1.0f);
    Y[7] = 1.0925484305920792f * (x * z);
    Y[8] = 0.54627421529603959f * (x * x - y * y);
    if (degree < 3) return;
    Y[9] = 0.59004358992664352f * (y * (3.0f * (x * x) - y * y));
    Y[10] = 2.8906114426405538f * ((x * y) * z);
    Y[11] = 0.45704579946446572f * (y * (5.0f * (z * z) - 1.0f));
    Y[12] = 0.3731763325901154f * (z * (5.0f * (z * z) - 3.0f));
    Y[13] = 0.45704579946446572f * (x * (5.0f * (z * z) - 1.0f));
    Y[14] = 1.4453057213202769f * (z * (x * x - y * y));
    Y[15] = 0.59004358992664352f * (x * (x * x - 3.0f * (y * y)));
}

void fgo_sh_basis(int degree, float x, float y, float z, float* Y) { sh_basis(degree, x, y, z, Y); }

typedef struct fgo_splat {
    float u, v;            /* 2D mean (pixels; pixel (i,j) centre at (i+0.5, j+0.5)) */
    float A, B, C;         /* conic: inverse of Sigma_2D */
    float opacity;
    float r, g, b;
    float depth;           /* camera-space z */
    float lambda;          /* largest eigenvalue of Sigma_2D */
    float radius;          /* tile-set radius after shrinking */
    int32_t x0, y0, x1, y1; /* tile rectangle [x0,x1) x [y0,y1) */
    uint32_t tiles;        /* (x1-x0)*(y1-y0), 0 if the Gaussian emits nothing */
} fgo_splat;

/* One selected Gaussian: projection, conic, colour, shrink radius, tiles.
 * tau <= 0 selects the 3-sigma rule; otherwise r = min(3 sigma,
 * sqrt(2 lambda_max ln(alpha0 / tau))) and r = 0 when alpha0 <= tau. */
static void preprocess_one(const fgo_tree* t, const fgo_camera* c, float tau, int64_t g, fgo_splat* o)
{
    memset(o, 0, sizeof(*o));
    int64_t N = t->n;
    float mx = t->mean[g], my = t->mean[N + g], mz = t->mean[2 * N + g];
    float pc[3];
    to_camera(c, mx, my, mz, pc);
    float s[3] = {t->scale[g], t->scale[N + g], t->scale[2 * N + g]};
    float q[4] = {t->quat[g], t->quat[N + g], t->quat[2 * N + g], t->quat[3 * N + g]};
    float S[6], a, b, cc;
    covariance3d(s, q, S);
    covariance2d(c, pc, S, &a, &b, &cc);
    float det = a * cc - b * b;
    float op = t->opacity[g];
    if (!(det > 0.0f) || !(op > 0.0f && op <= 1.0f)) return;
    o->A = cc / det;
    o->B = -b / det;
    o->C = a / det;
    o->u = (c->fx * pc[0]) / pc[2] + c->cx;
    o->v = (c->fy * pc[1]) / pc[2] + c->cy;
    o->depth = pc[2];
    o->opacity = op;
    float lam = lambda_max(a, b, cc);
    o->lambda = lam;
    /* radius: 3 sigma, shrunk by the opacity threshold tau */
    float r3 = 3.0f * sqrtf(lam);
    float r;
    if (tau <= 0.0f) {
        r = r3;
    } else {
        float qa = op / tau;
        if (qa <= 1.0f) {
            r = 0.0f;
        } else {
            float rs = sqrtf((2.0f * lam) * fgo_log(qa));
            r = rs < r3 ? rs : r3;
        }
    }
    o->radius = r;
    if (!(r > 0.0f)) return;
    int Wt = (c->width + 15) / 16, Ht = (c->height + 15) / 16;
    float fWt = (float)Wt, fHt = (float)Ht;
    float x0 = floorf((o->u - r) * 0.0625f);
    float x1 = floorf((o->u + r) * 0.0625f) + 1.0f;
    float y0 = floorf((o->v - r) * 0.0625f);
    float y1 = floorf((o->v + r) * 0.0625f) + 1.0f;
    x0 = x0 < 0.0f ? 0.0f : (x0 > fWt ? fWt : x0);
    x1 = x1 < 0.0f ? 0.0f : (x1 > fWt ? fWt : x1);
    y0 = y0 < 0.0f ? 0.0f : (y0 > fHt ? fHt : y0);
    y1 = y1 < 0.0f ? 0.0f : (y1 > fHt ? fHt : y1);
    if (x0 >= x1 || y0 >= y1) return;
    o->x0 = (int32_t)x0; o->x1 = (int32_t)x1;
    o->y0 = (int32_t)y0; o->y1 = (int32_t)y1;
    o->tiles = (uint32_t)((o->x1 - o->x0) * (o->y1 - o->y0));
    /* view-dependent colour, only for a splat that reaches a tile (one that
       reaches none is never blended; its colour stays 0):
       0.5 + sum_k sh_k Y_k(d), clamped below at 0 */
    float dx = mx - c->campos[0], dy = my - c->campos[1], dz = mz - c->campos[2];
    float len = sqrtf((dx * dx + dy * dy) + dz * dz);
    float Y[16];
    sh_basis(t->sh_degree, dx / len, dy / len, dz / len, Y);
    int K = (t->sh_degree + 1) * (t->sh_degree + 1);
    const float* sh = t->sh + (size_t)g * (size_t)K * 3;
    float rgb[3];
    for (int ch = 0; ch < 3; ch++) {
        float acc = Y[0] * sh[ch];
        for (int k = 1; k < K; k++) acc = acc + Y[k] * sh[k * 3 + ch];
        acc = acc + 0.5f;
        rgb[ch] = acc < 0.0f ? 0.0f : acc;
    }
    o->r = rgb[0]; o->g = rgb[1]; o->b = rgb[2];
}

void fgo_preprocess(const fgo_tree* t, const fgo_camera* c, float tau, const uint32_t* sel_idx, int64_t n_sel,
                    fgo_splat* out)
{
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n_sel; i++) preprocess_one(t, c, tau, (int64_t)sel_idx[i], &out[i]);
}

/* ---------------------------------------------------------------------- */
/* keys, sort, ranges                                                     */
/* ---------------------------------------------------------------------- */

typedef struct { uint64_t key; uint32_t val; } fgo_pair;

static int pair_cmp(const void* pa, const void* pb)
{
    const fgo_pair* a = (const fgo_pair*)pa;
    const fgo_pair* b = (const fgo_pair*)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->val != b->val) return a->val < b->val ? -1 : 1;
    return 0;
}

static uint32_t float_bits(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

/* Total number of pairs the splats emit. */
int64_t fgo_count_pairs(const fgo_splat* s, int64_t n)
{
    int64_t total = 0;
    for (int64_t i = 0; i < n; i++) total += s[i].tiles;
    return total;
}

/* Emit one pair per covered tile (Gaussian order, then tile rows, then tile
 * columns), key = (tile_base + ty*Wt + tx) << 32 | bits(depth), value = the
 * Gaussian's position in the splat list; sort by (key, value); per-tile
 * ranges [start, end), [0, 0) for empty tiles. keys/vals hold n_pairs. */
void fgo_sort(const fgo_splat* s, int64_t n, const fgo_camera* c, uint64_t* keys, uint32_t* vals, uint32_t* ranges)
{
    int Wt = (c->width + 15) / 16, Ht = (c->height + 15) / 16;
    int64_t np = fgo_count_pairs(s, n);
    fgo_pair* p = (fgo_pair*)malloc(sizeof(fgo_pair) * (size_t)(np > 0 ? np : 1));
    int64_t k = 0;
    for (int64_t i = 0; i < n; i++) {
        if (!s[i].tiles) continue;
        for (int ty = s[i].y0; ty < s[i].y1; ty++)
            for (int tx = s[i].x0; tx < s[i].x1; tx++) {
                uint64_t tile = (uint64_t)(c->tile_base + (uint32_t)(ty * Wt + tx));
                p[k].key = (tile << 32) | (uint64_t)float_bits(s[i].depth);
                p[k].val = (uint32_t)i;
                k++;
            }
    }
    qsort(p, (size_t)np, sizeof(fgo_pair), pair_cmp);
    for (int64_t i = 0; i < np; i++) { keys[i] = p[i].key; vals[i] = p[i].val; }
    memset(ranges, 0, sizeof(uint32_t) * 2 * (size_t)(Wt * Ht));
    for (int64_t i = 0; i < np; i++) {
        uint32_t tile = (uint32_t)(p[i].key >> 32) - c->tile_base;
        if (i == 0 || (uint32_t)(p[i - 1].key >> 32) - c->tile_base != tile) ranges[2 * tile] = (uint32_t)i;
        ranges[2 * tile + 1] = (uint32_t)(i + 1);
    }
    free(p);
}

/* ---------------------------------------------------------------------- */
/* blending, Eq. (2)                                                      */
/* ---------------------------------------------------------------------- */

/* Blend one pixel (px, py) over the sorted list vals[start..end):
 * power = -0.5 (A dx^2 + C dy^2) - B dx dy with d = mean2d - pixel centre;
 * skip power > 0; alpha = min(0.99, o * exp(power)), skip alpha < 1/255;
 * stop before a Gaussian that would take T below 1e-4;
 * C += rgb * alpha * T. Returns the number of list entries consumed up to
 * and including the last blended one. */
static uint32_t blend_pixel(const fgo_splat* s, const uint32_t* vals, uint32_t start, uint32_t end, int px, int py,
                            float out[3], float* T_out)
{
    float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
    float T = 1.0f;
    float C[3] = {0.0f, 0.0f, 0.0f};
    uint32_t last = 0;
    for (uint32_t k = start; k < end; k++) {
        const fgo_splat* g = &s[vals[k]];
        float dx = g->u - fpx;
        float dy = g->v - fpy;
        float power = -0.5f * ((g->A * dx) * dx + (g->C * dy) * dy) - (g->B * dx) * dy;
        if (power > 0.0f) continue;
        float alpha = g->opacity * fgo_exp(power);
        alpha = alpha < 0.99f ? alpha : 0.99f;
        if (alpha < 1.0f / 255.0f) continue;
        float Tn = T * (1.0f - alpha);
        if (Tn < 1e-4f) break;
        C[0] = C[0] + (g->r * alpha) * T;
        C[1] = C[1] + (g->g * alpha) * T;
        C[2] = C[2] + (g->b * alpha) * T;
        T = Tn;
        last = k - start + 1;
    }
    out[0] = C[0]; out[1] = C[1]; out[2] = C[2];
    *T_out = T;
    return last;
}

/* Tiled render: every pixel of tile t blends over range[t]. image [3][H][W],
 * final_T [H][W], n_contrib [H][W]; output colour C + T * bg. */
void fgo_render(const fgo_splat* s, const uint32_t* vals, const uint32_t* ranges, const fgo_camera* c,
                const float bg[3], float* image, float* final_T, uint32_t* n_contrib)
{
    int W = c->width, H = c->height;
    int Wt = (W + 15) / 16, Ht = (H + 15) / 16;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < Wt * Ht; t++) {
            int ty = t / Wt, tx = t % Wt;
            for (int py = ty * 16; py < ty * 16 + 16 && py < H; py++)
                for (int px = tx * 16; px < tx * 16 + 16 && px < W; px++) {
                    float C[3], T;
                    uint32_t last = blend_pixel(s, vals, ranges[2 * t], ranges[2 * t + 1], px, py, C, &T);
                    size_t o = (size_t)py * W + px;
                    for (int ch = 0; ch < 3; ch++) image[(size_t)ch * W * H + o] = C[ch] + T * bg[ch];
                    final_T[o] = T;
                    n_contrib[o] = last;
                }
        }
}

/* Render only the listed pixels (sampled checks at full size). */
void fgo_render_pixels(const fgo_splat* s, const uint32_t* vals, const uint32_t* ranges, const fgo_camera* c,
                       const float bg[3], const int32_t* px, const int32_t* py, int64_t m, float* rgb /*[m][3]*/,
                       float* T_out, uint32_t* n_contrib)
{
    int Wt = (c->width + 15) / 16;
    for (int64_t i = 0; i < m; i++) {
        int t = (py[i] / 16) * Wt + px[i] / 16;
        float C[3], T;
        n_contrib[i] = blend_pixel(s, vals, ranges[2 * t], ranges[2 * t + 1], px[i], py[i], C, &T);
        for (int ch = 0; ch < 3; ch++) rgb[3 * i + ch] = C[ch] + T * bg[ch];
        T_out[i] = T;
    }
}

int fgo_splat_size(void) { return (int)sizeof(fgo_splat); }

/* Elementwise helpers for the test suite. */
void fgo_exp_array(const float* x, float* y, int64_t n)
{
    for (int64_t i = 0; i < n; i++) y[i] = fgo_exp(x[i]);
}

void fgo_log_array(const float* x, float* y, int64_t n)
{
    for (int64_t i = 0; i < n; i++) y[i] = fgo_log(x[i]);
}

/* ---------------------------------------------------------------------- */
/* Key-value pair contribution, Eq. (5)                                   */
/* ---------------------------------------------------------------------- */

/* KPC of every pair of the sorted list: for each pixel of tile t, the
 * product alpha * T (T the transmittance before the splat) of each splat the
 * pixel actually blends is added to that pair's entry, in float64. Pairs a
 * pixel skips (power > 0, alpha < 1/255) or never reaches (terminated)
 * receive nothing from it. kpc has one entry per sorted pair. */
void fgo_kpc(const fgo_splat* s, const uint32_t* vals, const uint32_t* ranges, const fgo_camera* c, double* kpc)
{
    int W = c->width, H = c->height;
    int Wt = (W + 15) / 16, Ht = (H + 15) / 16;
    uint32_t np = 0;
    for (int t = 0; t < Wt * Ht; t++)
        if (ranges[2 * t + 1] > np) np = ranges[2 * t + 1];
    for (uint32_t k = 0; k < np; k++) kpc[k] = 0.0;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < Wt * Ht; t++) {
            int ty = t / Wt, tx = t % Wt;
            for (int py = ty * 16; py < ty * 16 + 16 && py < H; py++)
                for (int px = tx * 16; px < tx * 16 + 16 && px < W; px++) {
                    float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
                    float T = 1.0f;
                    for (uint32_t k = ranges[2 * t]; k < ranges[2 * t + 1]; k++) {
                        const fgo_splat* g = &s[vals[k]];
                        float dx = g->u - fpx;
                        float dy = g->v - fpy;
                        float power = -0.5f * ((g->A * dx) * dx + (g->C * dy) * dy) - (g->B * dx) * dy;
                        if (power > 0.0f) continue;
                        float alpha = g->opacity * fgo_exp(power);
                        alpha = alpha < 0.99f ? alpha : 0.99f;
                        if (alpha < 1.0f / 255.0f) continue;
                        float Tn = T * (1.0f - alpha);
                        if (Tn < 1e-4f) break;
                        kpc[k] += (double)alpha * (double)T;
                        T = Tn;
                    }
                }
        }
}

/* ---------------------------------------------------------------------- */
/* Differentiable form: activation, float64 replay forward and backward   */
/* ---------------------------------------------------------------------- */

/* Raw (unconstrained) Gaussian parameters of M Gaussians. */
typedef struct fgo_params {
    int64_t m;
    int32_t sh_degree;
    int32_t pad;
    const float* mean;      /* [3][m] */
    const float* log_scale; /* [3][m] */
    const float* quat;      /* [4][m] (w, x, y, z), any non-zero norm */
    const float* logit;     /* [m] opacity logits */
    const float* sh;        /* [m][K][3] */
} fgo_params;

/* float32 activations: scale = exp(log_scale), opacity = 1 / (1 + exp(-logit)),
 * with the same exponential as the blend (valid for |x| <= 87). */
void fgo_activate(const float* log_scale, const float* logit, int64_t m, float* scale, float* opacity)
{
    for (int64_t i = 0; i < 3 * m; i++) scale[i] = fgo_exp(log_scale[i]);
    for (int64_t i = 0; i < m; i++) opacity[i] = 1.0f / (1.0f + fgo_exp(-logit[i]));
}

typedef struct {
    double u, v, A, B, C, o, rgb[3], z;
    double pc[3], S2[3], Q[4];  /* camera-space centre, Sigma_2D (a, b, c) */
    double rgb_raw[3];          /* colour before the clamp at 0 */
    double dir[3], dlen;        /* unit view direction, distance */
    double s[3], qh[4], qn, R[9], M[9], Sig[6], J[4], T[6], Y[16];
} proj64;

static void sh_basis64(int degree, double x, double y, double z, double* Y)
{
    const double c0 = 0.28209479177387814, c1 = 0.48860251190291992, c2a = 1.0925484305920792,
                 c2b = 0.31539156525252005, c2c = 0.54627421529603959, c3a = 0.59004358992664352,
                 c3b = 2.8906114426405538, c3c = 0.45704579946446572, c3d = 0.3731763325901154,
                 c3e = 1.4453057213202769;
    Y[0] = c0;
    if (degree < 1) return;
    Y[1] = c1 * y; Y[2] = c1 * z; Y[3] = c1 * x;
    if (degree < 2) return;
    Y[4] = c2a * x * y; Y[5] = c2a * y * z; Y[6] = c2b * (3 * z * z - 1); Y[7] = c2a * x * z;
    Y[8] = c2c * (x * x - y * y);
    if (degree < 3) return;
    Y[9] = c3a * y * (3 * x * x - y * y); Y[10] = c3b * x * y * z; Y[11] = c3c * y * (5 * z * z - 1);
    Y[12] = c3d * z * (5 * z * z - 3); Y[13] = c3c * x * (5 * z * z - 1); Y[14] = c3e * z * (x * x - y * y);
    Y[15] = c3a * x * (x * x - 3 * y * y);
}

/* Partial derivatives dY_k/d(x, y, z) of the same polynomials. */
static void sh_basis_grad64(int degree, double x, double y, double z, double* dY /* [16][3] */)
{
    const double c1 = 0.48860251190291992, c2a = 1.0925484305920792, c2b = 0.31539156525252005,
                 c2c = 0.54627421529603959, c3a = 0.59004358992664352, c3b = 2.8906114426405538,
                 c3c = 0.45704579946446572, c3d = 0.3731763325901154, c3e = 1.4453057213202769;
    for (int i = 0; i < 48; i++) dY[i] = 0.0;
    if (degree < 1) return;
    dY[1 * 3 + 1] = c1; dY[2 * 3 + 2] = c1; dY[3 * 3 + 0] = c1;
    if (degree < 2) return;
    dY[4 * 3 + 0] = c2a * y; dY[4 * 3 + 1] = c2a * x;
    dY[5 * 3 + 1] = c2a * z; dY[5 * 3 + 2] = c2a * y;
    dY[6 * 3 + 2] = 6 * c2b * z;
    dY[7 * 3 + 0] = c2a * z; dY[7 * 3 + 2] = c2a * x;
    dY[8 * 3 + 0] = 2 * c2c * x; dY[8 * 3 + 1] = -2 * c2c * y;
    if (degree < 3) return;
    dY[9 * 3 + 0] = 6 * c3a * x * y; dY[9 * 3 + 1] = c3a * (3 * x * x - 3 * y * y);
    dY[10 * 3 + 0] = c3b * y * z; dY[10 * 3 + 1] = c3b * x * z; dY[10 * 3 + 2] = c3b * x * y;
    dY[11 * 3 + 1] = c3c * (5 * z * z - 1); dY[11 * 3 + 2] = 10 * c3c * y * z;
    dY[12 * 3 + 2] = c3d * (15 * z * z - 3);
    dY[13 * 3 + 0] = c3c * (5 * z * z - 1); dY[13 * 3 + 2] = 10 * c3c * x * z;
    dY[14 * 3 + 0] = 2 * c3e * x * z; dY[14 * 3 + 1] = -2 * c3e * y * z; dY[14 * 3 + 2] = c3e * (x * x - y * y);
    dY[15 * 3 + 0] = c3a * (3 * x * x - 3 * y * y); dY[15 * 3 + 1] = -6 * c3a * x * y;
}

/* float64 projection of raw Gaussian g (same formulas as preprocess_one). */
static void project64(const fgo_params* p, const fgo_camera* c, int64_t g, proj64* o)
{
    int64_t m = p->m;
    double mu[3] = {p->mean[g], p->mean[m + g], p->mean[2 * m + g]};
    const double* Wd;
    double W[9];
    for (int i = 0; i < 9; i++) W[i] = c->R[i];
    Wd = W;
    for (int i = 0; i < 3; i++) o->pc[i] = Wd[3 * i] * mu[0] + Wd[3 * i + 1] * mu[1] + Wd[3 * i + 2] * mu[2] + (double)c->t[i];
    for (int i = 0; i < 3; i++) o->s[i] = exp((double)p->log_scale[i * m + g]);
    double q[4] = {p->quat[g], p->quat[m + g], p->quat[2 * m + g], p->quat[3 * m + g]};
    o->qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int i = 0; i < 4; i++) o->qh[i] = q[i] / o->qn;
    double w = o->qh[0], x = o->qh[1], y = o->qh[2], z = o->qh[3];
    double* R = o->R;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) o->M[3 * i + j] = R[3 * i + j] * o->s[j];
    int k = 0;
    for (int i = 0; i < 3; i++)
        for (int j = i; j < 3; j++)
            o->Sig[k++] = o->M[3 * i] * o->M[3 * j] + o->M[3 * i + 1] * o->M[3 * j + 1] + o->M[3 * i + 2] * o->M[3 * j + 2];
    double X = o->pc[0], Yc = o->pc[1], Z = o->pc[2];
    o->J[0] = c->fx / Z; o->J[1] = -c->fx * X / (Z * Z); o->J[2] = c->fy / Z; o->J[3] = -c->fy * Yc / (Z * Z);
    for (int j = 0; j < 3; j++) {
        o->T[j] = o->J[0] * W[j] + o->J[1] * W[6 + j];
        o->T[3 + j] = o->J[2] * W[3 + j] + o->J[3] * W[6 + j];
    }
    double Sg[9] = {o->Sig[0], o->Sig[1], o->Sig[2], o->Sig[1], o->Sig[3], o->Sig[4], o->Sig[2], o->Sig[4], o->Sig[5]};
    double U[6];
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 3; j++)
            U[3 * i + j] = o->T[3 * i] * Sg[j] + o->T[3 * i + 1] * Sg[3 + j] + o->T[3 * i + 2] * Sg[6 + j];
    double s00 = U[0] * o->T[0] + U[1] * o->T[1] + U[2] * o->T[2];
    double s01 = U[0] * o->T[3] + U[1] * o->T[4] + U[2] * o->T[5];
    double s11 = U[3] * o->T[3] + U[4] * o->T[4] + U[5] * o->T[5];
    o->S2[0] = s00 + 0.3; o->S2[1] = s01; o->S2[2] = s11 + 0.3;
    double det = o->S2[0] * o->S2[2] - o->S2[1] * o->S2[1];
    o->A = o->S2[2] / det; o->B = -o->S2[1] / det; o->C = o->S2[0] / det;
    o->u = c->fx * X / Z + c->cx;
    o->v = c->fy * Yc / Z + c->cy;
    o->z = Z;
    o->o = 1.0 / (1.0 + exp(-(double)p->logit[g]));
    double d[3] = {mu[0] - c->campos[0], mu[1] - c->campos[1], mu[2] - c->campos[2]};
    o->dlen = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int i = 0; i < 3; i++) o->dir[i] = d[i] / o->dlen;
    sh_basis64(p->sh_degree, o->dir[0], o->dir[1], o->dir[2], o->Y);
    int K = (p->sh_degree + 1) * (p->sh_degree + 1);
    const float* sh = p->sh + (size_t)g * K * 3;
    for (int ch = 0; ch < 3; ch++) {
        double acc = 0.5;
        for (int kk = 0; kk < K; kk++) acc += o->Y[kk] * sh[kk * 3 + ch];
        o->rgb_raw[ch] = acc;
        o->rgb[ch] = acc < 0 ? 0 : acc;
    }
}

/* The float32 decisions of the blend for (pixel, splat): 1 = blended
 * (position < n_contrib and both skip tests pass), with *clamped = 1 when
 * alpha hit the 0.99 cap. Same arithmetic as blend_pixel. */
static int blended32(const fgo_splat* g, int px, int py, uint32_t pos, uint32_t n_contrib, int* clamped)
{
    if (pos >= n_contrib) return 0;
    float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
    float dx = g->u - fpx, dy = g->v - fpy;
    float power = -0.5f * ((g->A * dx) * dx + (g->C * dy) * dy) - (g->B * dx) * dy;
    if (power > 0.0f) return 0;
    float a = g->opacity * fgo_exp(power);
    *clamped = !(a < 0.99f);
    a = a < 0.99f ? a : 0.99f;
    return a >= 1.0f / 255.0f;
}

/* Float64 replay of the blend and its gradient. For every pixel the set of
 * blended splats, their order and the alpha clamp are those of the float32
 * forward (splats32, vals, ranges, n_contrib); all values are recomputed in
 * float64 from the raw parameters, so the result is the image of the smooth
 * piece the float32 forward is on and, with dL_dimage, its exact gradient.
 * image64 [3][H][W] (may be NULL); gradients (may be NULL) are accumulated
 * into float64 arrays shaped like the raw parameters. */
void fgo_replay64(const fgo_params* p, const fgo_camera* c, const float bg[3], const uint32_t* sel_idx, int64_t n_sel,
                  const fgo_splat* splats32, const uint32_t* vals, const uint32_t* ranges, const uint32_t* n_contrib,
                  const double* dL_dimage, double* image64, double* g_mean, double* g_log_scale, double* g_quat,
                  double* g_logit, double* g_sh)
{
    int W = c->width, H = c->height;
    int Wt = (W + 15) / 16, Ht = (H + 15) / 16;
    int64_t m = p->m;
    int K = (p->sh_degree + 1) * (p->sh_degree + 1);
    proj64* P = (proj64*)malloc(sizeof(proj64) * (size_t)(n_sel > 0 ? n_sel : 1));
    double* gs = (double*)calloc((size_t)(n_sel > 0 ? n_sel : 1) * 9, sizeof(double)); /* du dv dA dB dC do dr dg db */
    for (int64_t i = 0; i < n_sel; i++) project64(p, c, (int64_t)sel_idx[i], &P[i]);
    uint32_t maxlen = 1;
    for (int t = 0; t < Wt * Ht; t++)
        if (ranges[2 * t + 1] - ranges[2 * t] > maxlen) maxlen = ranges[2 * t + 1] - ranges[2 * t];
    uint32_t* list = (uint32_t*)malloc(sizeof(uint32_t) * maxlen);
    int* clampv = (int*)malloc(sizeof(int) * maxlen);
    for (int ty = 0; ty < Ht; ty++)
        for (int tx = 0; tx < Wt; tx++) {
            int t = ty * Wt + tx;
            uint32_t r0 = ranges[2 * t], r1 = ranges[2 * t + 1];
            for (int py = ty * 16; py < ty * 16 + 16 && py < H; py++)
                for (int px = tx * 16; px < tx * 16 + 16 && px < W; px++) {
                    size_t o = (size_t)py * W + px;
                    int nb = 0;
                    for (uint32_t k = r0; k < r1; k++) {
                        int cl = 0;
                        if (blended32(&splats32[vals[k]], px, py, k - r0, n_contrib[o], &cl)) {
                            list[nb] = vals[k];
                            clampv[nb] = cl;
                            nb++;
                        }
                    }
                    double fpx = px + 0.5, fpy = py + 0.5;
                    double Tv = 1.0, C[3] = {0, 0, 0};
                    for (int b = 0; b < nb; b++) {
                        const proj64* q = &P[list[b]];
                        double dx = q->u - fpx, dy = q->v - fpy;
                        double power = -0.5 * (q->A * dx * dx + q->C * dy * dy) - q->B * dx * dy;
                        double a = clampv[b] ? 0.99 : q->o * exp(power);
                        for (int ch = 0; ch < 3; ch++) C[ch] += q->rgb[ch] * a * Tv;
                        Tv *= (1.0 - a);
                    }
                    if (image64)
                        for (int ch = 0; ch < 3; ch++) image64[(size_t)ch * W * H + o] = C[ch] + Tv * bg[ch];
                    if (!dL_dimage) continue;
                    double G[3] = {dL_dimage[o], dL_dimage[(size_t)W * H + o], dL_dimage[2 * (size_t)W * H + o]};
                    double S[3] = {Tv * bg[0], Tv * bg[1], Tv * bg[2]};
                    double Tn = Tv;
                    for (int b = nb - 1; b >= 0; b--) {
                        const proj64* q = &P[list[b]];
                        double* gq = &gs[9 * (size_t)list[b]];
                        double dx = q->u - fpx, dy = q->v - fpy;
                        double power = -0.5 * (q->A * dx * dx + q->C * dy * dy) - q->B * dx * dy;
                        double e = exp(power);
                        double a = clampv[b] ? 0.99 : q->o * e;
                        double Tk = Tn / (1.0 - a);
                        double dLda = 0.0;
                        for (int ch = 0; ch < 3; ch++) {
                            gq[6 + ch] += G[ch] * a * Tk;
                            dLda += G[ch] * (q->rgb[ch] * Tk - S[ch] / (1.0 - a));
                            S[ch] += q->rgb[ch] * a * Tk;
                        }
                        Tn = Tk;
                        if (clampv[b]) continue;
                        double dLdp = dLda * a;
                        gq[5] += dLda * e;
                        gq[0] += dLdp * (-(q->A * dx + q->B * dy));
                        gq[1] += dLdp * (-(q->C * dy + q->B * dx));
                        gq[2] += dLdp * (-0.5 * dx * dx);
                        gq[3] += dLdp * (-dx * dy);
                        gq[4] += dLdp * (-0.5 * dy * dy);
                    }
                }
        }
    free(list);
    free(clampv);
    if (!dL_dimage) {
        free(P);
        free(gs);
        return;
    }
    /* projection backward: splat gradients -> raw parameters */
    for (int64_t i = 0; i < n_sel; i++) {
        const proj64* q = &P[i];
        const double* gq = &gs[9 * (size_t)i];
        int64_t g = sel_idx[i];
        double W9[9];
        for (int k = 0; k < 9; k++) W9[k] = c->R[k];
        double dmu[3] = {0, 0, 0}, dpc[3] = {0, 0, 0};
        /* colour -> SH and view direction */
        double dd[3] = {0, 0, 0};
        double dY[48];
        sh_basis_grad64(p->sh_degree, q->dir[0], q->dir[1], q->dir[2], dY);
        const float* sh = p->sh + (size_t)g * K * 3;
        for (int ch = 0; ch < 3; ch++) {
            double gr = q->rgb_raw[ch] < 0 ? 0.0 : gq[6 + ch];
            for (int k = 0; k < K; k++) {
                if (g_sh) g_sh[((size_t)g * K + k) * 3 + ch] += gr * q->Y[k];
                for (int a = 0; a < 3; a++) dd[a] += gr * sh[k * 3 + ch] * dY[k * 3 + a];
            }
        }
        double ddot = dd[0] * q->dir[0] + dd[1] * q->dir[1] + dd[2] * q->dir[2];
        for (int a = 0; a < 3; a++) dmu[a] += (dd[a] - q->dir[a] * ddot) / q->dlen;
        /* opacity */
        if (g_logit) g_logit[g] += gq[5] * q->o * (1.0 - q->o);
        /* 2D mean */
        double X = q->pc[0], Yc = q->pc[1], Z = q->pc[2];
        dpc[0] += gq[0] * c->fx / Z;
        dpc[1] += gq[1] * c->fy / Z;
        dpc[2] += -(gq[0] * c->fx * X + gq[1] * c->fy * Yc) / (Z * Z);
        /* conic (A, B, C) -> Sigma_2D: dL/dSigma = -Q G Q, G = [[gA, gB/2], [gB/2, gC]] */
        double Q[4] = {q->A, q->B, q->B, q->C};
        double Gm[4] = {gq[2], gq[3] / 2, gq[3] / 2, gq[4]};
        double QG[4] = {Q[0] * Gm[0] + Q[1] * Gm[2], Q[0] * Gm[1] + Q[1] * Gm[3], Q[2] * Gm[0] + Q[3] * Gm[2],
                        Q[2] * Gm[1] + Q[3] * Gm[3]};
        double QGQ[4] = {QG[0] * Q[0] + QG[1] * Q[2], QG[0] * Q[1] + QG[1] * Q[3], QG[2] * Q[0] + QG[3] * Q[2],
                         QG[2] * Q[1] + QG[3] * Q[3]};
        double Hs[4] = {-QGQ[0], -QGQ[1], -QGQ[2], -QGQ[3]}; /* symmetric dL/dSigma_2D */
        /* Sigma_2D = T Sigma T^T: dL/dSigma = T^T H T, dL/dT = 2 H T Sigma */
        const double* T = q->T;
        double Sg[9] = {q->Sig[0], q->Sig[1], q->Sig[2], q->Sig[1], q->Sig[3], q->Sig[4], q->Sig[2], q->Sig[4], q->Sig[5]};
        double dSig[9];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                double v = 0;
                for (int r = 0; r < 2; r++)
                    for (int s2 = 0; s2 < 2; s2++) v += T[3 * r + a] * Hs[2 * r + s2] * T[3 * s2 + b];
                dSig[3 * a + b] = v;
            }
        double HT[6];
        for (int r = 0; r < 2; r++)
            for (int b = 0; b < 3; b++) HT[3 * r + b] = Hs[2 * r] * T[b] + Hs[2 * r + 1] * T[3 + b];
        double dT[6];
        for (int r = 0; r < 2; r++)
            for (int b = 0; b < 3; b++)
                dT[3 * r + b] = 2 * (HT[3 * r] * Sg[b] + HT[3 * r + 1] * Sg[3 + b] + HT[3 * r + 2] * Sg[6 + b]);
        /* T = J W: dL/dJ = dT W^T; J00 = fx/z, J02 = -fx x/z^2, J11 = fy/z, J12 = -fy y/z^2 */
        double dJ00 = 0, dJ02 = 0, dJ11 = 0, dJ12 = 0;
        for (int b = 0; b < 3; b++) {
            dJ00 += dT[b] * W9[b];
            dJ02 += dT[b] * W9[6 + b];
            dJ11 += dT[3 + b] * W9[3 + b];
            dJ12 += dT[3 + b] * W9[6 + b];
        }
        dpc[0] += dJ02 * (-c->fx / (Z * Z));
        dpc[1] += dJ12 * (-c->fy / (Z * Z));
        dpc[2] += dJ00 * (-c->fx / (Z * Z)) + dJ11 * (-c->fy / (Z * Z)) + dJ02 * (2 * c->fx * X / (Z * Z * Z)) +
                  dJ12 * (2 * c->fy * Yc / (Z * Z * Z));
        for (int a = 0; a < 3; a++) dmu[a] += W9[a] * dpc[0] + W9[3 + a] * dpc[1] + W9[6 + a] * dpc[2];
        /* Sigma = M M^T: dL/dM = 2 dSig M (dSig symmetric) */
        double dM[9];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++)
                dM[3 * a + b] = 2 * (dSig[3 * a] * q->M[b] + dSig[3 * a + 1] * q->M[3 + b] + dSig[3 * a + 2] * q->M[6 + b]);
        double ds[3] = {0, 0, 0}, dR[9];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                ds[b] += dM[3 * a + b] * q->R[3 * a + b];
                dR[3 * a + b] = dM[3 * a + b] * q->s[b];
            }
        double w = q->qh[0], x = q->qh[1], y = q->qh[2], z = q->qh[3];
        double dqh[4];
        dqh[0] = 2 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
        dqh[1] = 2 * (y * dR[1] + z * dR[2] + y * dR[3] - 2 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] - 2 * x * dR[8]);
        dqh[2] = 2 * (-2 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] - 2 * y * dR[8]);
        dqh[3] = 2 * (-2 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2 * z * dR[4] + y * dR[5] + x * dR[6] + y * dR[7]);
        double qd = dqh[0] * w + dqh[1] * x + dqh[2] * y + dqh[3] * z;
        if (g_quat)
            for (int a = 0; a < 4; a++) g_quat[a * m + g] += (dqh[a] - q->qh[a] * qd) / q->qn;
        if (g_log_scale)
            for (int a = 0; a < 3; a++) g_log_scale[a * m + g] += ds[a] * q->s[a];
        if (g_mean)
            for (int a = 0; a < 3; a++) g_mean[a * m + g] += dmu[a];
    }
    free(P);
    free(gs);
}

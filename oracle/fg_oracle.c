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
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

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

/* exp(x) for x <= 0 (0 below -87, where the true value approaches the
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
    for (int64_t n = 0; n < t->n; n++) {
        float pc[3];
        int f = node_frustum(t, c, n, pc);
        int small = f && node_radius3(t, c, n, pc) <= tau_R;
        int leaf = t->flags[n] & 1;
        int rl = f && (leaf || small);
        out[n] = (uint8_t)(f | (small << 1) | (rl << 2));
    }
    for (int64_t n = 0; n < t->n; n++) {
        int sel = (out[n] >> 2) & 1;
        for (int32_t a = t->parent[n]; sel && a >= 0; a = t->parent[a])
            if ((out[a] >> 2) & 1) sel = 0;
        out[n] |= (uint8_t)(sel << 3);
    }
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
    /* view-dependent colour: 0.5 + sum_k sh_k Y_k(d), clamped below at 0 */
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
}

void fgo_preprocess(const fgo_tree* t, const fgo_camera* c, float tau, const uint32_t* sel_idx, int64_t n_sel,
                    fgo_splat* out)
{
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
    for (int ty = 0; ty < Ht; ty++)
        for (int tx = 0; tx < Wt; tx++) {
            int t = ty * Wt + tx;
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
    for (int ty = 0; ty < Ht; ty++)
        for (int tx = 0; tx < Wt; tx++) {
            int t = ty * Wt + tx;
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

/*
 * FP64 CPU oracle of the differentiable point-splat renderer.
 *
 * TEST INFRASTRUCTURE ONLY.  This file defines what the renderer computes so
 * that the GPU implementation can be checked against it.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it.  It shares
 * no code, header, table or constant with the HIP library.
 *
 * Every step follows the paper (Zhang et al., "Differentiable Point-Based
 * Radiance Fields for Efficient View Synthesis", SIGGRAPH Asia 2022):
 *   Sec. 3.1 Eq. (1)   projection p = M (R P + t) followed by the perspective divide
 *   Sec. 3.1 Eq. (3)   view direction v = (R P + t) / |R P + t|
 *   Sec. 3.1 Eq. (2,4) colour c = sum_{l<=lmax} sum_m h_lm Y_lm(v)
 *   Sec. 3.2 Eq. (5)   Gaussian RBF opacity of a splat at pixel u
 *   Sec. 3.2 Eq. (6,7) front-to-back alpha blending over points sorted by z
 *   Sec. 3.2 (end)     only points near u with non-negligible opacity count
 *
 * Readings where the paper leaves a choice open (each one is listed in the
 * design notes of the repository):
 *   - the 1/sqrt(2 pi r^2) prefactor of Eq. (5) is dropped; a per-point opacity
 *     o_i multiplies the Gaussian and alpha is clamped to alpha_max;
 *   - the splat radius r is in world units and is perspective-scaled into
 *     pixels, sigma_x = fx r / Z, sigma_y = fy r / Z;
 *   - "non-negligible opacity" is the predicate o_i G_i(u) >= alpha_min;
 *   - compositing stops once the transmittance falls below t_min;
 *   - the z-distance is camera-space Z; ties are broken by point index.  The
 *     sort key and the near-plane cull are decided in float32 on
 *     Z32 = fmaf(R20, x, fmaf(R21, y, fmaf(R22, z, t2))), the same rule the GPU
 *     path uses, so both sides visit points in the same order;
 *   - real orthonormal SH without the Condon-Shortley phase, index
 *     k = l^2 + l + m;
 *   - pixel (x, y) is sampled at its centre (x + 0.5, y + 0.5); background 0.
 *
 * Everything else is computed in double from the float inputs widened exactly.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAX_K 16

/* ---------------------------------------------------------------------------
 * Real spherical harmonics, Sec. 3.1 Eq. (4).  Y[k] for k = l^2 + l + m and the
 * gradient dY[k][3] with respect to the unconstrained direction vector
 * (the polynomials below are evaluated for any 3-vector; only their values and
 * tangential derivatives on the unit sphere enter the result).
 * Normalisation constants are written from their closed forms.
 * ------------------------------------------------------------------------- */
static int sh_count(int degree) { return (degree + 1) * (degree + 1); }

static void sh_basis(int degree, const double d[3], double Y[OR_MAX_K], double dY[OR_MAX_K][3])
{
    const double pi = 3.14159265358979323846;
    const double x = d[0], y = d[1], z = d[2];
    int k;
    for (k = 0; k < OR_MAX_K; ++k) { Y[k] = 0.0; dY[k][0] = dY[k][1] = dY[k][2] = 0.0; }

    /* l = 0 */
    Y[0] = 0.5 * sqrt(1.0 / pi);
    if (degree < 1) return;

    /* l = 1: m = -1, 0, 1 -> y, z, x */
    {
        const double c1 = sqrt(3.0 / (4.0 * pi));
        Y[1] = c1 * y; dY[1][1] = c1;
        Y[2] = c1 * z; dY[2][2] = c1;
        Y[3] = c1 * x; dY[3][0] = c1;
    }
    if (degree < 2) return;

    /* l = 2: m = -2 .. 2 -> xy, yz, (2z^2 - x^2 - y^2), xz, (x^2 - y^2) */
    {
        const double a = 0.5 * sqrt(15.0 / pi);
        const double b = 0.25 * sqrt(5.0 / pi);
        const double c = 0.25 * sqrt(15.0 / pi);
        Y[4] = a * x * y;  dY[4][0] = a * y; dY[4][1] = a * x;
        Y[5] = a * y * z;  dY[5][1] = a * z; dY[5][2] = a * y;
        Y[6] = b * (2.0 * z * z - x * x - y * y);
        dY[6][0] = -2.0 * b * x; dY[6][1] = -2.0 * b * y; dY[6][2] = 4.0 * b * z;
        Y[7] = a * x * z;  dY[7][0] = a * z; dY[7][2] = a * x;
        Y[8] = c * (x * x - y * y);
        dY[8][0] = 2.0 * c * x; dY[8][1] = -2.0 * c * y;
    }
    if (degree < 3) return;

    /* l = 3: m = -3 .. 3 */
    {
        const double a = 0.25 * sqrt(35.0 / (2.0 * pi));   /* m = +-3 */
        const double b = 0.5 * sqrt(105.0 / pi);           /* m = -2  */
        const double c = 0.25 * sqrt(21.0 / (2.0 * pi));   /* m = +-1 */
        const double e = 0.25 * sqrt(7.0 / pi);            /* m = 0   */
        const double f = 0.25 * sqrt(105.0 / pi);          /* m = +2  */
        const double r1 = 4.0 * z * z - x * x - y * y;
        Y[9] = a * y * (3.0 * x * x - y * y);
        dY[9][0] = a * 6.0 * x * y; dY[9][1] = a * (3.0 * x * x - 3.0 * y * y);
        Y[10] = b * x * y * z;
        dY[10][0] = b * y * z; dY[10][1] = b * x * z; dY[10][2] = b * x * y;
        Y[11] = c * y * r1;
        dY[11][0] = c * y * (-2.0 * x); dY[11][1] = c * (r1 - 2.0 * y * y); dY[11][2] = c * y * 8.0 * z;
        Y[12] = e * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y);
        dY[12][0] = e * z * (-6.0 * x); dY[12][1] = e * z * (-6.0 * y);
        dY[12][2] = e * (6.0 * z * z - 3.0 * x * x - 3.0 * y * y);
        Y[13] = c * x * r1;
        dY[13][0] = c * (r1 - 2.0 * x * x); dY[13][1] = c * x * (-2.0 * y); dY[13][2] = c * x * 8.0 * z;
        Y[14] = f * z * (x * x - y * y);
        dY[14][0] = f * z * 2.0 * x; dY[14][1] = -f * z * 2.0 * y; dY[14][2] = f * (x * x - y * y);
        Y[15] = a * x * (x * x - 3.0 * y * y);
        dY[15][0] = a * (3.0 * x * x - 3.0 * y * y); dY[15][1] = a * (-6.0 * x * y);
    }
}

/* Exported for the basis pins (orthonormality by quadrature, closed forms). */
int oracle_sh_basis(int degree, const double *dirs, int64_t n, double *Y_out, double *dY_out)
{
    int64_t i;
    int K, k;
    if (degree < 0 || degree > 3) return 1;
    K = sh_count(degree);
    for (i = 0; i < n; ++i) {
        double Y[OR_MAX_K], dY[OR_MAX_K][3];
        sh_basis(degree, dirs + 3 * i, Y, dY);
        for (k = 0; k < K; ++k) {
            Y_out[i * K + k] = Y[k];
            if (dY_out) {
                dY_out[(i * K + k) * 3 + 0] = dY[k][0];
                dY_out[(i * K + k) * 3 + 1] = dY[k][1];
                dY_out[(i * K + k) * 3 + 2] = dY[k][2];
            }
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Per-point, per-view quantities (Sec. 3.1, Eq. 1-4).
 * cam[16] = R (row-major 3x3), t (3), fx, fy, cx, cy.
 * ------------------------------------------------------------------------- */
typedef struct {
    double X[3];       /* camera-space position R P + t            */
    double norm;       /* |X|                                      */
    double px, py;     /* projected position, Eq. (1)              */
    double sx, sy;     /* screen-space Gaussian sigma (pixels)     */
    double dir[3];     /* SH direction (Eq. 3, camera or world)    */
    double c[3];       /* colour, Eq. (4)                          */
    double k;          /* kernel prefactor: 1, or (2 pi sx sy)^-1/2 with the literal Eq. (5) normalisation */
    float zkey;        /* float32 depth key used for ordering      */
    int valid;         /* in front of the near plane               */
} or_point;

static float depth_key(const double *cam, const double *P)
{
    /* float32, evaluated as fmaf(R20, x, fmaf(R21, y, fmaf(R22, z, t2))) */
    float acc = fmaf((float)cam[8], (float)P[2], (float)cam[11]);
    acc = fmaf((float)cam[7], (float)P[1], acc);
    acc = fmaf((float)cam[6], (float)P[0], acc);
    return acc;
}

static void project_point(const double *cam, const double *P, const double *h, int degree,
                          double radius, double z_near, int sh_frame, int kernel_norm, or_point *o)
{
    const double *R = cam, *t = cam + 9;
    const double fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15];
    int r, k, ch, K = sh_count(degree);
    double Y[OR_MAX_K], dY[OR_MAX_K][3];

    for (r = 0; r < 3; ++r)
        o->X[r] = R[3 * r + 0] * P[0] + R[3 * r + 1] * P[1] + R[3 * r + 2] * P[2] + t[r];
    o->zkey = depth_key(cam, P);
    o->valid = (o->zkey > (float)z_near);
    o->norm = sqrt(o->X[0] * o->X[0] + o->X[1] * o->X[1] + o->X[2] * o->X[2]);
    if (!o->valid) return;

    /* Eq. (1): p = (M X)^down with M = [[fx, 0, cx], [0, fy, cy], [0, 0, 1]] */
    o->px = fx * o->X[0] / o->X[2] + cx;
    o->py = fy * o->X[1] / o->X[2] + cy;
    /* world radius scaled into pixels by the perspective divide */
    o->sx = fx * radius / o->X[2];
    o->sy = fy * radius / o->X[2];
    /* Eq. (5) as printed carries 1/sqrt(2 pi r^2) with r the kernel radius; with
     * a per-axis sigma the 2-D analogue is 1/sqrt(2 pi sx sy) */
    o->k = kernel_norm ? 1.0 / sqrt(2.0 * OR_PI * o->sx * o->sy) : 1.0;

    /* Eq. (3): camera-frame unit direction; sh_frame = 1 rotates it back to world */
    {
        double v[3] = { o->X[0] / o->norm, o->X[1] / o->norm, o->X[2] / o->norm };
        if (sh_frame == 1) {
            for (r = 0; r < 3; ++r)
                o->dir[r] = R[0 * 3 + r] * v[0] + R[1 * 3 + r] * v[1] + R[2 * 3 + r] * v[2];
        } else {
            o->dir[0] = v[0]; o->dir[1] = v[1]; o->dir[2] = v[2];
        }
    }
    /* Eq. (4): c = sum_k h_k Y_k(v), per colour channel, no activation */
    sh_basis(degree, o->dir, Y, dY);
    for (ch = 0; ch < 3; ++ch) {
        double s = 0.0;
        for (k = 0; k < K; ++k) s += h[k * 3 + ch] * Y[k];
        o->c[ch] = s;
    }
}

/* out[n][12] = px, py, sx, sy, Z, c0, c1, c2, dir0, dir1, dir2, valid;
 * zkey[n] = float32 depth key. */
int oracle_project(int64_t n, const double *xyz, const double *sh, int degree,
                   const double *radius, const double *cam, double z_near, int sh_frame,
                   double *out, float *zkey)
{
    int64_t i;
    int K;
    if (degree < 0 || degree > 3) return 1;
    K = sh_count(degree);
    for (i = 0; i < n; ++i) {
        or_point p;
        memset(&p, 0, sizeof(p));
        project_point(cam, xyz + 3 * i, sh + (int64_t)K * 3 * i, degree, radius[i], z_near, sh_frame, 0, &p);
        out[i * 12 + 0] = p.px;  out[i * 12 + 1] = p.py;
        out[i * 12 + 2] = p.sx;  out[i * 12 + 3] = p.sy;
        out[i * 12 + 4] = p.X[2];
        out[i * 12 + 5] = p.c[0]; out[i * 12 + 6] = p.c[1]; out[i * 12 + 7] = p.c[2];
        out[i * 12 + 8] = p.dir[0]; out[i * 12 + 9] = p.dir[1]; out[i * 12 + 10] = p.dir[2];
        out[i * 12 + 11] = p.valid ? 1.0 : 0.0;
        zkey[i] = p.zkey;
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Depth order (Sec. 3.2: sort by z-distance, front to back).
 * ------------------------------------------------------------------------- */
typedef struct { float z; int64_t i; } or_key;

static int cmp_key(const void *a, const void *b)
{
    const or_key *x = (const or_key *)a, *y = (const or_key *)b;
    if (x->z < y->z) return -1;
    if (x->z > y->z) return 1;
    return (x->i < y->i) ? -1 : (x->i > y->i);
}

/* Returns the number of valid points; order[] holds their indices front to back. */
static int64_t depth_order(int64_t n, const or_point *pts, int64_t *order)
{
    int64_t i, m = 0;
    or_key *keys = (or_key *)malloc(sizeof(or_key) * (size_t)(n > 0 ? n : 1));
    for (i = 0; i < n; ++i)
        if (pts[i].valid) { keys[m].z = pts[i].zkey; keys[m].i = i; ++m; }
    qsort(keys, (size_t)m, sizeof(or_key), cmp_key);
    for (i = 0; i < m; ++i) order[i] = keys[i].i;
    free(keys);
    return m;
}

/* Exported so the tests can check the GPU's depth permutation exactly. */
int oracle_depth_order(int64_t n, const double *xyz, const double *cam, double z_near,
                       int64_t *order, int64_t *m_out)
{
    int64_t i;
    or_point *pts = (or_point *)calloc((size_t)(n > 0 ? n : 1), sizeof(or_point));
    for (i = 0; i < n; ++i) {
        pts[i].zkey = depth_key(cam, xyz + 3 * i);
        pts[i].valid = pts[i].zkey > (float)z_near;
    }
    *m_out = depth_order(n, pts, order);
    free(pts);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Splat opacity at a pixel, Sec. 3.2 Eq. (5) under the readings above:
 *   G = exp(-1/2 [ (px-ux)^2/sx^2 + (py-uy)^2/sy^2 ]),  a = o G,
 *   candidate iff a >= alpha_min,  alpha = min(alpha_max, a).
 * ------------------------------------------------------------------------- */
typedef struct {
    double alpha_min, t_min, alpha_max, z_near;
    int64_t max_splats;      /* > 0: a pixel blends at most this many splats */
    int kernel_norm;         /* 1: Eq. (5)'s normalisation prefactor is kept  */
} or_params;

/* Relative distance to alpha_min within which a capped pixel's predicate
 * decision counts as a near tie (see composite_pixel).  A float32 evaluation of
 * the exponent (from float32 splat centres and shapes) differs from this
 * float64 one by up to a few 1e-5 relative in alpha. */
#define OR_NEAR_TIE 1e-4

static void read_params(const double *params, or_params *pr)
{
    pr->alpha_min = params[0]; pr->t_min = params[1]; pr->alpha_max = params[2]; pr->z_near = params[3];
    pr->max_splats = (int64_t)params[4];
    pr->kernel_norm = params[5] != 0.0;
}

static int splat_alpha(const or_point *p, double o, double ux, double uy, const or_params *pr,
                       double *alpha, double *G, int *clamped, double *dx, double *dy, double *a_raw)
{
    double ex = p->px - ux, ey = p->py - uy;
    double q = ex * ex / (p->sx * p->sx) + ey * ey / (p->sy * p->sy);
    double g = exp(-0.5 * q);
    double a = o * p->k * g;
    *a_raw = a;
    if (!(a >= pr->alpha_min)) return 0;
    *G = g; *dx = ex; *dy = ey;
    if (a > pr->alpha_max) { *alpha = pr->alpha_max; *clamped = 1; }
    else { *alpha = a; *clamped = 0; }
    return 1;
}

/* Support of the predicate: the ellipse (ex/sx)^2 + (ey/sy)^2 <= 2 ln(o/alpha_min).
 * Under a cap it reaches down to alpha_min (1 - OR_NEAR_TIE), so that a pixel
 * also meets the splats it flags as near ties without blending them. */
static int support_box(const or_point *p, double o, const or_params *pr,
                       double *x0, double *x1, double *y0, double *y1)
{
    double s, lo = pr->max_splats > 0 ? pr->alpha_min * (1.0 - OR_NEAR_TIE) : pr->alpha_min;
    if (!(pr->alpha_min > 0.0)) return -1;            /* unbounded */
    if (!(o * p->k >= lo)) return 0;                   /* never a candidate */
    s = sqrt(2.0 * log(o * p->k / lo)) * (1.0 + 1e-9) + 1e-9;
    *x0 = p->px - s * p->sx; *x1 = p->px + s * p->sx;
    *y0 = p->py - s * p->sy; *y1 = p->py + s * p->sy;
    return 1;
}

/* ---------------------------------------------------------------------------
 * Candidate lists.  Mode 0 (brute force): every pixel walks the full depth
 * order.  Mode 1 (ordered grid): the depth order is split into 8x8-pixel cells
 * by the bounding box of each splat's exact support; a cell's list keeps the
 * depth order, so a pixel visits the same candidates in the same order and the
 * result is bitwise identical to mode 0 (checked by the tests).
 * ------------------------------------------------------------------------- */
#define OR_CELL 8

typedef struct {
    int64_t m;               /* number of valid points in depth order */
    int64_t *order;          /* [m] */
    int cells_x, cells_y;
    int64_t *cell_start;     /* [cells + 1], NULL in brute-force mode */
    int64_t *cell_items;     /* indices into the point array */
} or_lists;

static void build_lists(int64_t n, const or_point *pts, const double *opacity, int width, int height,
                        const or_params *pr, int mode, or_lists *L)
{
    int64_t s, total = 0;
    int cx0, cx1, cy0, cy1, a, b, nc;
    memset(L, 0, sizeof(*L));
    L->order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    L->m = depth_order(n, pts, L->order);
    if (mode == 0 || !(pr->alpha_min > 0.0)) return;

    L->cells_x = (width + OR_CELL - 1) / OR_CELL;
    L->cells_y = (height + OR_CELL - 1) / OR_CELL;
    nc = L->cells_x * L->cells_y;
    L->cell_start = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
    /* pass 1: count, pass 2: fill in depth order */
    for (b = 0; b < 2; ++b) {
        int64_t *fill = NULL;
        if (b == 1) {
            for (a = 0; a < nc; ++a) L->cell_start[a + 1] += L->cell_start[a];
            total = L->cell_start[nc];
            L->cell_items = (int64_t *)malloc(sizeof(int64_t) * (size_t)(total > 0 ? total : 1));
            fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)nc);
            for (a = 0; a < nc; ++a) fill[a] = L->cell_start[a];
        }
        for (s = 0; s < L->m; ++s) {
            int64_t i = L->order[s];
            double x0, x1, y0, y1;
            int r = support_box(&pts[i], opacity[i], pr, &x0, &x1, &y0, &y1);
            if (r == 0) continue;
            /* pixel centres x + 0.5 inside [x0, x1] */
            {
                double fx0 = ceil(x0 - 0.5), fx1 = floor(x1 - 0.5);
                double fy0 = ceil(y0 - 0.5), fy1 = floor(y1 - 0.5);
                if (fx1 < 0 || fy1 < 0 || fx0 > width - 1 || fy0 > height - 1) continue;
                if (fx0 < 0) fx0 = 0;
                if (fy0 < 0) fy0 = 0;
                if (fx1 > width - 1) fx1 = width - 1;
                if (fy1 > height - 1) fy1 = height - 1;
                cx0 = (int)fx0 / OR_CELL; cx1 = (int)fx1 / OR_CELL;
                cy0 = (int)fy0 / OR_CELL; cy1 = (int)fy1 / OR_CELL;
            }
            {
                int gy, gx;
                for (gy = cy0; gy <= cy1; ++gy) {
                    for (gx = cx0; gx <= cx1; ++gx) {
                        int c = gy * L->cells_x + gx;
                        if (fill) L->cell_items[fill[c]++] = i;
                        else L->cell_start[c + 1] += 1;
                    }
                }
            }
        }
        free(fill);
    }
}

static void free_lists(or_lists *L)
{
    free(L->order); free(L->cell_start); free(L->cell_items);
    memset(L, 0, sizeof(*L));
}

static void pixel_list(const or_lists *L, int width, int x, int y, const int64_t **items,
                       int64_t *count, int *indirect)
{
    (void)width;
    if (!L->cell_start) { *items = L->order; *count = L->m; *indirect = 0; return; }
    {
        int c = (y / OR_CELL) * L->cells_x + (x / OR_CELL);
        *items = L->cell_items + L->cell_start[c];
        *count = L->cell_start[c + 1] - L->cell_start[c];
        *indirect = 1;
    }
}

/* ---------------------------------------------------------------------------
 * One pixel, Sec. 3.2 Eq. (6)-(7): I = sum_i alpha_i prod_{k<i}(1 - alpha_k) c_i
 * over the candidates in front-to-back order, stopping once T < t_min.
 * ------------------------------------------------------------------------- */
typedef struct {
    int64_t i;
    double alpha, T, G, dx, dy;
    int clamped;
} or_hit;

/* Under a cap (max_splats > 0) the splats a pixel blends depend on every
 * predicate decision before the cap is reached: a candidate decided within a
 * relative OR_NEAR_TIE of alpha_min may be decided the other way by an
 * evaluation in another precision, and then the pixel's n-th splat, and its
 * colour, change by a whole splat.  Such a pixel has two valid results;
 * *near_tie is set for it (never without a cap). */
static int64_t composite_pixel(const or_lists *L, const or_point *pts, const double *opacity,
                               int width, int x, int y, const or_params *pr,
                               double I[3], double *T_out, int *stopped, int *near_tie, or_hit *hits,
                               int64_t hit_cap)
{
    const int64_t *items;
    int64_t cnt, s, nh = 0;
    int indirect;
    double T = 1.0;
    double ux = x + 0.5, uy = y + 0.5;
    I[0] = I[1] = I[2] = 0.0;
    *stopped = 0;
    *near_tie = 0;
    pixel_list(L, width, x, y, &items, &cnt, &indirect);
    for (s = 0; s < cnt; ++s) {
        int64_t i = items[s];
        double alpha, G, dx, dy, a;
        int clamped, hit = splat_alpha(&pts[i], opacity[i], ux, uy, pr, &alpha, &G, &clamped, &dx, &dy, &a);
        if (pr->max_splats > 0 && fabs(a - pr->alpha_min) <= OR_NEAR_TIE * pr->alpha_min) *near_tie = 1;
        if (!hit) continue;
        if (hits && nh < hit_cap) {
            hits[nh].i = i; hits[nh].alpha = alpha; hits[nh].T = T; hits[nh].G = G;
            hits[nh].dx = dx; hits[nh].dy = dy; hits[nh].clamped = clamped;
        }
        I[0] += T * alpha * pts[i].c[0];
        I[1] += T * alpha * pts[i].c[1];
        I[2] += T * alpha * pts[i].c[2];
        T *= (1.0 - alpha);
        ++nh;
        if (T < pr->t_min) { *stopped = 1; break; }
        if (pr->max_splats > 0 && nh >= pr->max_splats) { *stopped = 1; break; }
    }
    (void)indirect;
    *T_out = T;
    return nh;
}

static void project_all(int64_t n, const double *xyz, const double *sh, int degree, const double *radius,
                        const double *cam, const or_params *pr, int sh_frame, or_point *pts)
{
    int64_t i;
    int K = sh_count(degree);
    for (i = 0; i < n; ++i)
        project_point(cam, xyz + 3 * i, sh + (int64_t)K * 3 * i, degree, radius[i], pr->z_near, sh_frame,
                      pr->kernel_norm, &pts[i]);
}

/*
 * Forward render of one view.
 *   params[6] = alpha_min, t_min, alpha_max, z_near, max_splats (0: no cap), kernel_norm (0/1)
 *   pix: npix linear pixel indices (y * width + x), or NULL for the whole image
 *        in row-major order (npix must then equal width * height)
 *   image[npix][3], trans[npix]; ncontrib[npix] (nullable) = number of blended
 *   splats; stopped[npix] (nullable): bit 0 where the early stop fired, bit 1
 *   where a cap's outcome rests on a near-threshold predicate (composite_pixel).
 */
int oracle_render(int64_t n, const double *xyz, const double *sh, int degree, const double *opacity,
                  const double *radius, const double *cam, int width, int height,
                  const double *params, int sh_frame, int mode, int64_t npix, const int64_t *pix,
                  double *image, double *trans, int64_t *ncontrib, int32_t *stopped, int nthreads)
{
    or_params pr;
    or_point *pts;
    or_lists L;
    int64_t p;
    if (degree < 0 || degree > 3 || width < 1 || height < 1 || n < 0) return 1;
    if (!pix && npix != (int64_t)width * height) return 1;
    read_params(params, &pr);
    pts = (or_point *)calloc((size_t)(n > 0 ? n : 1), sizeof(or_point));
    project_all(n, xyz, sh, degree, radius, cam, &pr, sh_frame, pts);
    build_lists(n, pts, opacity, width, height, &pr, mode, &L);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (p = 0; p < npix; ++p) {
        int64_t lin = pix ? pix[p] : p;
        int x = (int)(lin % width), y = (int)(lin / width);
        double I[3], T;
        int st, tie;
        int64_t nh = composite_pixel(&L, pts, opacity, width, x, y, &pr, I, &T, &st, &tie, NULL, 0);
        image[3 * p + 0] = I[0]; image[3 * p + 1] = I[1]; image[3 * p + 2] = I[2];
        trans[p] = T;
        if (ncontrib) ncontrib[p] = nh;
        if (stopped) stopped[p] = st | (tie << 1);
    }
    free_lists(&L);
    free(pts);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Backward: the exact reverse-mode derivative of the forward above, with the
 * candidate sets and the stop index held fixed (piecewise-constant structure).
 *
 * Per pixel, with T_i the transmittance in front of splat i and Q_i the product
 * of (1 - alpha_k) over the blended splats k behind i,
 *   dI/dc_i     = T_i alpha_i
 *   dI/dalpha_i = T_i (c_i - R_i),  R_i = sum_{k>i} alpha_k c_k prod_{i<m<k}(1 - alpha_m)
 *   dT/dalpha_i = -T_i Q_i
 * and through Eq. (5): dalpha/do = G, dalpha/dq = -o G / 2 for the quadratic form
 * q = ex^2/sx^2 + ey^2/sy^2 (zero where alpha is clamped).  The per-point
 * chain rule then goes through Eq. (1), the perspective-scaled sigma, Eq. (3)
 * and Eq. (4) back to P, h and o.
 * Gradients are ADDED into dxyz[n][3], dsh[n][K][3], dopacity[n].
 * ------------------------------------------------------------------------- */
typedef struct { double dpx, dpy, dsx, dsy, dop, dc[3]; } or_pgrad;

int oracle_backward(int64_t n, const double *xyz, const double *sh, int degree, const double *opacity,
                    const double *radius, const double *cam, int width, int height,
                    const double *params, int sh_frame, int mode, int64_t npix, const int64_t *pix,
                    const double *dL_dimage, const double *dL_dtrans,
                    double *dxyz, double *dsh, double *dopacity, int nthreads)
{
    or_params pr;
    or_point *pts;
    or_lists L;
    or_pgrad *acc;
    int nth = 1, K, t;
    int64_t i;
    if (degree < 0 || degree > 3 || width < 1 || height < 1 || n < 0) return 1;
    if (!pix && npix != (int64_t)width * height) return 1;
    K = sh_count(degree);
    read_params(params, &pr);
    pts = (or_point *)calloc((size_t)(n > 0 ? n : 1), sizeof(or_point));
    project_all(n, xyz, sh, degree, radius, cam, &pr, sh_frame, pts);
    build_lists(n, pts, opacity, width, height, &pr, mode, &L);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    nth = omp_get_max_threads();
#endif
    acc = (or_pgrad *)calloc((size_t)nth * (size_t)(n > 0 ? n : 1), sizeof(or_pgrad));

#ifdef _OPENMP
#pragma omp parallel
#endif
    {
        int tid = 0;
        int64_t p, cap = L.m > 0 ? L.m : 1;
        or_hit *hits = (or_hit *)malloc(sizeof(or_hit) * (size_t)cap);
        or_pgrad *mine;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        mine = acc + (size_t)tid * (size_t)(n > 0 ? n : 1);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
        for (p = 0; p < npix; ++p) {
            int64_t lin = pix ? pix[p] : p;
            int x = (int)(lin % width), y = (int)(lin / width);
            double I[3], T, R[3] = {0.0, 0.0, 0.0}, Q = 1.0;
            const double *gI = dL_dimage + 3 * p;
            double gT = dL_dtrans ? dL_dtrans[p] : 0.0;
            int st;
            int tie;
            int64_t h, nh = composite_pixel(&L, pts, opacity, width, x, y, &pr, I, &T, &st, &tie, hits, cap);
            for (h = nh - 1; h >= 0; --h) {
                const or_hit *e = &hits[h];
                const or_point *q = &pts[e->i];
                or_pgrad *g = &mine[e->i];
                double dA = e->T * (gI[0] * (q->c[0] - R[0]) + gI[1] * (q->c[1] - R[1]) + gI[2] * (q->c[2] - R[2]))
                            - gT * e->T * Q;
                int ch;
                for (ch = 0; ch < 3; ++ch) g->dc[ch] += e->T * e->alpha * gI[ch];
                for (ch = 0; ch < 3; ++ch) R[ch] = e->alpha * q->c[ch] + (1.0 - e->alpha) * R[ch];
                Q *= (1.0 - e->alpha);
                if (!e->clamped) {
                    /* alpha = o k G: dalpha/do = k G, dalpha/dq = -o k G / 2, and with the
                     * normalisation k = (2 pi sx sy)^-1/2 also dalpha/dsx = -alpha / (2 sx) */
                    double o = opacity[e->i];
                    double dq = dA * (-0.5 * o * q->k * e->G);
                    g->dop += dA * q->k * e->G;
                    g->dpx += dq * 2.0 * e->dx / (q->sx * q->sx);
                    g->dpy += dq * 2.0 * e->dy / (q->sy * q->sy);
                    g->dsx += dq * (-2.0 * e->dx * e->dx / (q->sx * q->sx * q->sx));
                    g->dsy += dq * (-2.0 * e->dy * e->dy / (q->sy * q->sy * q->sy));
                    if (pr.kernel_norm) {
                        g->dsx += dA * (-0.5 * e->alpha / q->sx);
                        g->dsy += dA * (-0.5 * e->alpha / q->sy);
                    }
                }
            }
        }
        free(hits);
    }

    /* per-point chain rule, threads' partial sums added in thread order */
    for (i = 0; i < n; ++i) {
        or_pgrad g;
        const or_point *q = &pts[i];
        const double *R = cam;
        const double fx = cam[12], fy = cam[13];
        double dX[3], Z, Y[OR_MAX_K], dY[OR_MAX_K][3], dd[3] = {0.0, 0.0, 0.0}, dv[3];
        int k, ch, r;
        memset(&g, 0, sizeof(g));
        for (t = 0; t < nth; ++t) {
            const or_pgrad *s = &acc[(size_t)t * (size_t)n + (size_t)i];
            g.dpx += s->dpx; g.dpy += s->dpy; g.dsx += s->dsx; g.dsy += s->dsy; g.dop += s->dop;
            g.dc[0] += s->dc[0]; g.dc[1] += s->dc[1]; g.dc[2] += s->dc[2];
        }
        if (!q->valid) continue;
        Z = q->X[2];
        /* Eq. (1) and sigma = f r / Z */
        dX[0] = g.dpx * fx / Z;
        dX[1] = g.dpy * fy / Z;
        dX[2] = -g.dpx * fx * q->X[0] / (Z * Z) - g.dpy * fy * q->X[1] / (Z * Z)
                - g.dsx * q->sx / Z - g.dsy * q->sy / Z;
        /* Eq. (4): dc/dh_k = Y_k(dir); dc/ddir = sum_k h_k grad Y_k */
        sh_basis(degree, q->dir, Y, dY);
        for (k = 0; k < K; ++k) {
            double w = 0.0;
            for (ch = 0; ch < 3; ++ch) {
                dsh[(i * K + k) * 3 + ch] += Y[k] * g.dc[ch];
                w += g.dc[ch] * sh[(i * K + k) * 3 + ch];
            }
            dd[0] += w * dY[k][0]; dd[1] += w * dY[k][1]; dd[2] += w * dY[k][2];
        }
        /* direction frame: dir = v (camera) or R^T v (world) */
        if (sh_frame == 1) {
            for (r = 0; r < 3; ++r) dv[r] = R[3 * r + 0] * dd[0] + R[3 * r + 1] * dd[1] + R[3 * r + 2] * dd[2];
        } else {
            dv[0] = dd[0]; dv[1] = dd[1]; dv[2] = dd[2];
        }
        /* Eq. (3): v = X / |X|  ->  dX += (dv - v (v . dv)) / |X| */
        {
            double v[3] = { q->X[0] / q->norm, q->X[1] / q->norm, q->X[2] / q->norm };
            double vd = v[0] * dv[0] + v[1] * dv[1] + v[2] * dv[2];
            for (r = 0; r < 3; ++r) dX[r] += (dv[r] - v[r] * vd) / q->norm;
        }
        /* X = R P + t  ->  dP = R^T dX */
        for (r = 0; r < 3; ++r)
            dxyz[i * 3 + r] += R[0 * 3 + r] * dX[0] + R[1 * 3 + r] * dX[1] + R[2 * 3 + r] * dX[2];
        dopacity[i] += g.dop;
    }
    free(acc);
    free_lists(&L);
    free(pts);
    return 0;
}

/* Number of OpenMP threads a parallel region would use. */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

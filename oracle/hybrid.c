/*
 * FP64 CPU oracle of the hybrid coarse-to-fine update (Sec. 3.3 "Hybrid
 * Coarse-to-Fine Updates", Alg. 1).  Test infrastructure only; it shares no
 * code with the HIP library.
 *
 * A point carries its position, its SH coefficients (K3 = 3 (l_max + 1)^2
 * floats), its opacity and its radius; "all parameters" of a point are
 * averaged together.  Where a float comparison decides an integer (a voxel
 * index, a neighbour set, a removal) it is evaluated in float32 with the
 * operations spelled out below, no contraction, so the GPU decides the same
 * way; averages are taken in FP64.
 *
 * Readings (the algorithm leaves them open):
 *  - voxels: the points' axis-aligned bounding box [lo, hi] split into N equal
 *    cells per axis; per axis s = N / (hi - lo) (float32), index
 *    floor((p - lo) * s) clamped to [0, N - 1] (an axis with hi == lo maps to
 *    0); key (iz N + iy) N + ix; output in ascending key order.
 *  - neighbours of a point: the other points ordered by the float32 squared
 *    distance ((dx dx + dy dy) + dz dz), dx = x_j - x_i, ties by index; the
 *    first min(K, m - 1).
 *  - spread: d_k = sqrt(d2_k); mean = (sum d_k) / k; delta = sqrt(sum (d_k -
 *    mean)^2 / k), float32, sums in neighbour order (population deviation);
 *    a point is removed when delta > eps (a point without neighbours stays).
 *  - removal and generation are each decided against the set before that step
 *    (no mutation while iterating); generated points follow the kept ones, in
 *    the order of the point they come from; a point without neighbours
 *    generates nothing.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int cmp_u64_i64(const void *a, const void *b)
{
    const uint64_t *x = (const uint64_t *)a, *y = (const uint64_t *)b;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    return x[1] < y[1] ? -1 : (x[1] > y[1] ? 1 : 0);
}

static void bbox32(int64_t n, const float *xyz, float lo[3], float hi[3])
{
    int64_t i;
    int a;
    for (a = 0; a < 3; ++a) { lo[a] = xyz[a]; hi[a] = xyz[a]; }
    for (i = 1; i < n; ++i)
        for (a = 0; a < 3; ++a) {
            float v = xyz[3 * i + a];
            if (v < lo[a]) lo[a] = v;
            if (v > hi[a]) hi[a] = v;
        }
}

static uint32_t axis_cell(float p, float lo, float s, int N)
{
    float t;
    long c;
    if (!(s > 0.0f)) return 0;
    t = (p - lo) * s;
    c = (long)floorf(t);
    if (c < 0) c = 0;
    if (c > N - 1) c = N - 1;
    return (uint32_t)c;
}

/* Voxel key of every point (float32 decisions as documented above). */
int hybrid_voxel_keys(int64_t n, const float *xyz, int N, uint64_t *keys)
{
    float lo[3], hi[3], s[3];
    int64_t i;
    int a;
    if (n < 1 || N < 1) return 1;
    bbox32(n, xyz, lo, hi);
    for (a = 0; a < 3; ++a) s[a] = hi[a] > lo[a] ? (float)N / (hi[a] - lo[a]) : 0.0f;
    for (i = 0; i < n; ++i) {
        uint32_t ix = axis_cell(xyz[3 * i + 0], lo[0], s[0], N);
        uint32_t iy = axis_cell(xyz[3 * i + 1], lo[1], s[1], N);
        uint32_t iz = axis_cell(xyz[3 * i + 2], lo[2], s[2], N);
        keys[i] = ((uint64_t)iz * (uint64_t)N + iy) * (uint64_t)N + ix;
    }
    return 0;
}

/*
 * Step 1 of Alg. 1: every non-empty voxel becomes the average of its points.
 * In: n points (float32 arrays).  Out (capacity n): the averages in ascending
 * voxel order, FP64; returns their number, or -1 on bad input.
 */
int64_t hybrid_voxel_reduce(int64_t n, int k3, const float *xyz, const float *sh, const float *op,
                            const float *rad, int N, double *oxyz, double *osh, double *oop, double *orad)
{
    uint64_t *kv, *keys;
    int64_t i, m = 0;
    if (n < 1 || N < 1 || k3 < 0) return -1;
    keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    kv = (uint64_t *)malloc(sizeof(uint64_t) * 2 * (size_t)n);
    hybrid_voxel_keys(n, xyz, N, keys);
    for (i = 0; i < n; ++i) { kv[2 * i] = keys[i]; kv[2 * i + 1] = (uint64_t)i; }
    qsort(kv, (size_t)n, 2 * sizeof(uint64_t), cmp_u64_i64);
    i = 0;
    while (i < n) {
        int64_t j = i, c, q;
        int a;
        while (j < n && kv[2 * j] == kv[2 * i]) ++j;
        c = j - i;
        for (a = 0; a < 3; ++a) oxyz[3 * m + a] = 0.0;
        for (a = 0; a < k3; ++a) osh[(int64_t)k3 * m + a] = 0.0;
        oop[m] = 0.0; orad[m] = 0.0;
        for (q = i; q < j; ++q) {
            int64_t p = (int64_t)kv[2 * q + 1];
            for (a = 0; a < 3; ++a) oxyz[3 * m + a] += xyz[3 * p + a];
            for (a = 0; a < k3; ++a) osh[(int64_t)k3 * m + a] += sh[(int64_t)k3 * p + a];
            oop[m] += op[p]; orad[m] += rad[p];
        }
        for (a = 0; a < 3; ++a) oxyz[3 * m + a] /= (double)c;
        for (a = 0; a < k3; ++a) osh[(int64_t)k3 * m + a] /= (double)c;
        oop[m] /= (double)c; orad[m] /= (double)c;
        ++m;
        i = j;
    }
    free(kv);
    free(keys);
    return m;
}

/* float32 squared distance ((dx dx + dy dy) + dz dz), dx = x_j - x_i */
static float dist2(const float *a, const float *b)
{
    float dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
    float s = dx * dx;
    s = s + dy * dy;
    s = s + dz * dz;
    return s;
}

typedef struct { float d2; int64_t j; } hy_nb;

static int cmp_nb(const void *a, const void *b)
{
    const hy_nb *x = (const hy_nb *)a, *y = (const hy_nb *)b;
    if (x->d2 != y->d2) return x->d2 < y->d2 ? -1 : 1;
    return x->j < y->j ? -1 : (x->j > y->j ? 1 : 0);
}

/*
 * Brute-force K nearest neighbours of every point among the others.
 * idx[m][K] (-1 past min(K, m - 1)), d2[m][K] (float32 squared distances).
 */
int hybrid_knn(int64_t m, const float *xyz, int K, int64_t *idx, float *d2)
{
    hy_nb *all;
    int64_t i, j, c;
    int k;
    if (m < 1 || K < 1) return 1;
    all = (hy_nb *)malloc(sizeof(hy_nb) * (size_t)(m > 1 ? m - 1 : 1));
    for (i = 0; i < m; ++i) {
        c = 0;
        for (j = 0; j < m; ++j) {
            if (j == i) continue;
            all[c].d2 = dist2(xyz + 3 * i, xyz + 3 * j);
            all[c].j = j;
            ++c;
        }
        qsort(all, (size_t)c, sizeof(hy_nb), cmp_nb);
        for (k = 0; k < K; ++k) {
            idx[i * K + k] = k < c ? all[k].j : -1;
            d2[i * K + k] = k < c ? all[k].d2 : 0.0f;
        }
    }
    free(all);
    return 0;
}

/* delta of Alg. 1 from a point's neighbour distances (float32, see above) */
static float spread(const float *d2, int k)
{
    float sum = 0.0f, mean, var = 0.0f;
    int q;
    for (q = 0; q < k; ++q) sum = sum + sqrtf(d2[q]);
    mean = sum / (float)k;
    for (q = 0; q < k; ++q) {
        float e = sqrtf(d2[q]) - mean;
        var = var + e * e;
    }
    return sqrtf(var / (float)k);
}

/*
 * Steps 2 and 3 of Alg. 1 on m points (float32 in): keep[m] (0/1) after the
 * outlier test, then one generated point per kept point with neighbours, the
 * FP64 average of its min(K, kept - 1) nearest kept neighbours.
 * Out: the kept points (FP64 copies) followed by the generated ones, capacity
 * 2 m; returns the output count, or -1 on bad input.
 */
int64_t hybrid_filter_generate(int64_t m, int k3, const float *xyz, const float *sh, const float *op,
                               const float *rad, int K, float eps, int32_t *keep, double *oxyz, double *osh,
                               double *oop, double *orad)
{
    int64_t *idx, *kept_idx, i, nk = 0, out;
    float *d2, *kxyz;
    int a, q, kq;
    if (m < 1 || K < 1 || k3 < 0) return -1;
    idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)m * (size_t)K);
    d2 = (float *)malloc(sizeof(float) * (size_t)m * (size_t)K);
    hybrid_knn(m, xyz, K, idx, d2);
    kq = (int)(m - 1 < K ? m - 1 : K);
    for (i = 0; i < m; ++i) keep[i] = kq == 0 ? 1 : !(spread(d2 + i * K, kq) > eps);
    kept_idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    for (i = 0; i < m; ++i)
        if (keep[i]) kept_idx[nk++] = i;
    for (i = 0; i < nk; ++i) {
        int64_t p = kept_idx[i];
        for (a = 0; a < 3; ++a) oxyz[3 * i + a] = xyz[3 * p + a];
        for (a = 0; a < k3; ++a) osh[(int64_t)k3 * i + a] = sh[(int64_t)k3 * p + a];
        oop[i] = op[p]; orad[i] = rad[p];
    }
    out = nk;
    if (nk >= 2) {
        kxyz = (float *)malloc(sizeof(float) * 3 * (size_t)nk);
        for (i = 0; i < nk; ++i)
            for (a = 0; a < 3; ++a) kxyz[3 * i + a] = xyz[3 * kept_idx[i] + a];
        hybrid_knn(nk, kxyz, K, idx, d2);
        kq = (int)(nk - 1 < K ? nk - 1 : K);
        for (i = 0; i < nk; ++i) {
            for (a = 0; a < 3; ++a) oxyz[3 * out + a] = 0.0;
            for (a = 0; a < k3; ++a) osh[(int64_t)k3 * out + a] = 0.0;
            oop[out] = 0.0; orad[out] = 0.0;
            for (q = 0; q < kq; ++q) {
                int64_t p = kept_idx[idx[i * K + q]];
                for (a = 0; a < 3; ++a) oxyz[3 * out + a] += xyz[3 * p + a];
                for (a = 0; a < k3; ++a) osh[(int64_t)k3 * out + a] += sh[(int64_t)k3 * p + a];
                oop[out] += op[p]; orad[out] += rad[p];
            }
            for (a = 0; a < 3; ++a) oxyz[3 * out + a] /= (double)kq;
            for (a = 0; a < k3; ++a) osh[(int64_t)k3 * out + a] /= (double)kq;
            oop[out] /= (double)kq; orad[out] /= (double)kq;
            ++out;
        }
        free(kxyz);
    }
    free(kept_idx);
    free(d2);
    free(idx);
    return out;
}

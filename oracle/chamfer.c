/*
 * CPU oracle of the video warm start (Sec. 3.4 "Video Synthesis"): the
 * Chamfer distance of Eq. (9) between the learned cloud S1 of one frame and
 * the initial cloud S2 of the next, its gradient with respect to the
 * positions of S2, one Adam step on those positions, and the transfer of the
 * mean SH of each S2 point's k nearest S1 points.  Test infrastructure only;
 * it shares no code with the HIP library.
 *
 * Readings (the paper leaves them open):
 *  - squared distance d2(x, y) = ((x0 - y0)^2 + (x1 - y1)^2) + (x2 - y2)^2 in
 *    float32, each operation rounded once (it is symmetric in x and y);
 *  - the nearest neighbour of a point is the one with the smallest d2, ties to
 *    the lower index;
 *  - CD = (1/|S1|) sum_x d2(x, nn(x)) + (1/|S2|) sum_y d2(y, nn(y)), summed in
 *    FP64 in index order;
 *  - its gradient (a subgradient where neighbours tie) with respect to y_j in
 *    S2: (2/|S2|) (y_j - nn(y_j)) + (2/|S1|) sum over x with nn(x) = y_j of
 *    (y_j - x), in FP64;
 *  - top-k transfer: the k = min(K, |S1|) S1 points with the smallest
 *    (d2, index) to y_j; their SH coefficients averaged in FP64 in that order;
 *  - Adam (Kingma and Ba, ICLR 2015) with bias correction at step t >= 1:
 *    m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 *    p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), in FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static float d2f(const float *x, const float *y)
{
    float a = x[0] - y[0], b = x[1] - y[1], c = x[2] - y[2];
    float s = a * a;
    s = s + b * b;
    s = s + c * c;
    return s;
}

/* nearest point of B for every point of A: nn[i], d2[i] */
int chamfer_nn(int64_t na, const float *a, int64_t nb, const float *b, int64_t *nn, float *d2)
{
    int64_t i, j;
    if (na < 0 || nb < 1) return 1;
    for (i = 0; i < na; ++i) {
        float best = INFINITY;
        int64_t bj = -1;
        for (j = 0; j < nb; ++j) {
            const float d = d2f(a + 3 * i, b + 3 * j);
            if (d < best) { best = d; bj = j; }
        }
        nn[i] = bj;
        d2[i] = best;
    }
    return 0;
}

/* CD of Eq. (9) and its gradient with respect to S2 (grad2[n2][3], FP64). */
int chamfer_forward_backward(int64_t n1, const float *s1, int64_t n2, const float *s2, double *cd, double *grad2)
{
    int64_t i, *nn12, *nn21;
    float *d12, *d21;
    double t1 = 0.0, t2 = 0.0;
    if (n1 < 1 || n2 < 1) return 1;
    nn12 = (int64_t *)malloc(sizeof(int64_t) * (size_t)n1);
    nn21 = (int64_t *)malloc(sizeof(int64_t) * (size_t)n2);
    d12 = (float *)malloc(sizeof(float) * (size_t)n1);
    d21 = (float *)malloc(sizeof(float) * (size_t)n2);
    chamfer_nn(n1, s1, n2, s2, nn12, d12);
    chamfer_nn(n2, s2, n1, s1, nn21, d21);
    for (i = 0; i < n1; ++i) t1 += d12[i];
    for (i = 0; i < n2; ++i) t2 += d21[i];
    *cd = t1 / (double)n1 + t2 / (double)n2;
    for (i = 0; i < n2; ++i) {
        int a;
        const int64_t k = nn21[i];
        for (a = 0; a < 3; ++a)
            grad2[3 * i + a] = 2.0 / (double)n2 * ((double)s2[3 * i + a] - (double)s1[3 * k + a]);
    }
    for (i = 0; i < n1; ++i) {
        int a;
        const int64_t j = nn12[i];
        for (a = 0; a < 3; ++a)
            grad2[3 * j + a] += 2.0 / (double)n1 * ((double)s2[3 * j + a] - (double)s1[3 * i + a]);
    }
    free(nn12); free(nn21); free(d12); free(d21);
    return 0;
}

typedef struct { float d2; int64_t j; } cf_nb;

static int cmp_nb(const void *p, const void *q)
{
    const cf_nb *x = (const cf_nb *)p, *y = (const cf_nb *)q;
    if (x->d2 != y->d2) return x->d2 < y->d2 ? -1 : 1;
    return x->j < y->j ? -1 : (x->j > y->j ? 1 : 0);
}

/* Top-k SH transfer: out_sh[n2][k3] (FP64) and the neighbour indices idx[n2][K] (-1 past k). */
int chamfer_topk_sh(int64_t n1, const float *s1, const float *sh1, int64_t n2, const float *s2, int k3, int K,
                    double *out_sh, int64_t *idx)
{
    cf_nb *all;
    int64_t i, j;
    int q, a, kk;
    if (n1 < 1 || n2 < 0 || K < 1 || k3 < 1) return 1;
    kk = (int)(n1 < K ? n1 : K);
    all = (cf_nb *)malloc(sizeof(cf_nb) * (size_t)n1);
    for (i = 0; i < n2; ++i) {
        for (j = 0; j < n1; ++j) { all[j].d2 = d2f(s2 + 3 * i, s1 + 3 * j); all[j].j = j; }
        qsort(all, (size_t)n1, sizeof(cf_nb), cmp_nb);
        for (a = 0; a < k3; ++a) out_sh[(int64_t)k3 * i + a] = 0.0;
        for (q = 0; q < K; ++q) idx[i * K + q] = q < kk ? all[q].j : -1;
        for (q = 0; q < kk; ++q)
            for (a = 0; a < k3; ++a) out_sh[(int64_t)k3 * i + a] += (double)sh1[(int64_t)k3 * all[q].j + a];
        for (a = 0; a < k3; ++a) out_sh[(int64_t)k3 * i + a] /= (double)kk;
    }
    free(all);
    return 0;
}

/* One Adam step on n values (FP64 state), step t >= 1. */
int adam_step(int64_t n, double *p, const double *g, double *m, double *v, int t, double lr, double b1, double b2,
              double eps)
{
    int64_t i;
    double c1, c2;
    if (n < 0 || t < 1) return 1;
    c1 = 1.0 - pow(b1, (double)t);
    c2 = 1.0 - pow(b2, (double)t);
    for (i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
    return 0;
}

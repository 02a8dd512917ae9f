/*
 * CPU oracle of the visual-hull initialisation and the multi-view consistency
 * filter (Sec. 3.1 "Initialization"; appendix "Additional Initialization
 * Details", the consistency check CC).  Test infrastructure only; it shares
 * no code with the HIP library.
 *
 * Readings (the paper leaves them open):
 *  - Point P is inside mask i when its projection (Eq. 1) falls on a pixel
 *    (floor(px), floor(py)) of image i whose mask byte is non-zero.  A point
 *    with Z <= 0, or whose projection leaves the image, is not inside.  The
 *    decision is taken in float32 with these operations, each rounded once:
 *      X_c = fma(R_c0, x, fma(R_c1, y, fma(R_c2, z, t_c)))   (c = 0, 1, 2)
 *      px = fma(fx, X_0 / X_2, cx),  py = fma(fy, X_1 / X_2, cy)
 *    inside the image iff 0 <= px < W and 0 <= py < H.
 *  - CC(P) = 1 iff P is inside every one of the N masks.
 *  - Rejection sampling: candidate j (j = 0 .. n-1) comes from Philox4x32-10
 *    (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2,
 *    3", SC 2011) with counter (j mod 2^32, j div 2^32, 0, 0) and key
 *    (seed mod 2^32, seed div 2^32).  Its first three output words r give
 *    u = (r >> 8) * 2^-24 in [0, 1) and the coordinate fma(u, hi - lo, lo)
 *    (float32, hi - lo rounded once).  Kept candidates are returned in
 *    candidate order.
 *  - Filter: the points with CC = 1, in input order, every parameter copied.
 *
 * A camera is 16 floats: R (row-major 3x3), t, fx, fy, cx, cy.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

/* Philox4x32 round constants and key schedule constants of the SC 2011 paper. */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

static void mulhilo(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo)
{
    const uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

/* Ten rounds of Philox4x32 on counter ctr with key key -> out. */
void hull_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int r;
    for (r = 0; r < 10; ++r) {
        uint32_t hi0, lo0, hi1, lo1;
        if (r > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        mulhilo(PHILOX_M0, c0, &hi0, &lo0);
        mulhilo(PHILOX_M1, c2, &hi1, &lo1);
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 1 if P = (x, y, z) is inside the mask of camera cam (W x H bytes, row-major). */
static int inside_mask(float x, float y, float z, const float *cam, int32_t W, int32_t H, const uint8_t *mask)
{
    float X[3], u, v, px, py;
    int c;
    for (c = 0; c < 3; ++c) X[c] = fmaf(cam[3 * c + 0], x, fmaf(cam[3 * c + 1], y, fmaf(cam[3 * c + 2], z, cam[9 + c])));
    if (!(X[2] > 0.0f)) return 0;
    u = X[0] / X[2];
    v = X[1] / X[2];
    px = fmaf(cam[12], u, cam[14]);
    py = fmaf(cam[13], v, cam[15]);
    if (!(px >= 0.0f && px < (float)W && py >= 0.0f && py < (float)H)) return 0;
    return mask[(int64_t)(int32_t)py * W + (int32_t)px] != 0;
}

static int consistent(float x, float y, float z, int32_t n_cams, const float *cams, const int32_t *dims,
                      const uint8_t *const *masks)
{
    int32_t i;
    for (i = 0; i < n_cams; ++i)
        if (!inside_mask(x, y, z, cams + 16 * i, dims[2 * i], dims[2 * i + 1], masks[i])) return 0;
    return 1;
}

/* keep[j] = CC(P_j) for n points (float32 xyz).  dims: W, H per camera. */
int hull_consistent(int64_t n, const float *xyz, int32_t n_cams, const float *cams, const int32_t *dims,
                    const uint8_t *const *masks, uint8_t *keep)
{
    int64_t j;
    if (n < 0 || n_cams < 1) return 1;
    for (j = 0; j < n; ++j) keep[j] = (uint8_t)consistent(xyz[3 * j], xyz[3 * j + 1], xyz[3 * j + 2], n_cams, cams,
                                                        dims, masks);
    return 0;
}

/* Candidate j of the rejection sampler (see the readings above). */
void hull_candidate(uint64_t seed, uint64_t j, const float lo[3], const float hi[3], float p[3])
{
    uint32_t ctr[4], key[2], r[4];
    int a;
    ctr[0] = (uint32_t)j; ctr[1] = (uint32_t)(j >> 32); ctr[2] = 0; ctr[3] = 0;
    key[0] = (uint32_t)seed; key[1] = (uint32_t)(seed >> 32);
    hull_philox(ctr, key, r);
    for (a = 0; a < 3; ++a) {
        const float u = (float)(r[a] >> 8) * 0x1p-24f;
        p[a] = fmaf(u, hi[a] - lo[a], lo[a]);
    }
}

/*
 * Rejection sampling of n candidates in the box [lo, hi]: the consistent ones,
 * in candidate order, go to out_xyz (first `capacity` of them).  Returns the
 * number of consistent candidates (which may exceed capacity), -1 on bad input.
 */
int64_t hull_sample(int32_t n_cams, const float *cams, const int32_t *dims, const uint8_t *const *masks,
                    const float lo[3], const float hi[3], uint64_t seed, int64_t n, float *out_xyz,
                    int64_t capacity)
{
    int64_t j, kept = 0;
    if (n < 0 || n_cams < 1 || capacity < 0) return -1;
    for (j = 0; j < n; ++j) {
        float p[3];
        hull_candidate(seed, (uint64_t)j, lo, hi, p);
        if (!consistent(p[0], p[1], p[2], n_cams, cams, dims, masks)) continue;
        if (kept < capacity) memcpy(out_xyz + 3 * kept, p, sizeof(p));
        ++kept;
    }
    return kept;
}

/* The first n candidates of the sampler, unfiltered (for tests). */
void hull_candidates(uint64_t seed, int64_t n, const float lo[3], const float hi[3], float *out_xyz)
{
    int64_t j;
    for (j = 0; j < n; ++j) hull_candidate(seed, (uint64_t)j, lo, hi, out_xyz + 3 * j);
}

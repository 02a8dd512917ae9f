// Real spherical harmonics up to degree 3 in float32 (Sec. 3.1, Eq. 4).
// Index k = l^2 + l + m, no Condon-Shortley phase.  The polynomials are the
// homogeneous forms, valid for any 3-vector; only their values and tangential
// derivatives on the unit sphere enter the renderer.
#pragma once

#include <hip/hip_runtime.h>

namespace dpr {

// 1/(2 sqrt(pi)), sqrt(3/(4 pi)), sqrt(15/(4 pi)), sqrt(5/(16 pi)), sqrt(15/(16 pi)),
// sqrt(35/(32 pi)), sqrt(105/(4 pi)), sqrt(21/(32 pi)), sqrt(7/(16 pi)), sqrt(105/(16 pi))
constexpr float kSH0 = 0.28209479177387814f;
constexpr float kSH1 = 0.48860251190291992f;
constexpr float kSH2a = 1.0925484305920792f;
constexpr float kSH2b = 0.31539156525252005f;
constexpr float kSH2c = 0.54627421529603959f;
constexpr float kSH3a = 0.59004358992664352f;
constexpr float kSH3b = 2.8906114426405538f;
constexpr float kSH3c = 0.45704579946446572f;
constexpr float kSH3d = 0.3731763325901154f;
constexpr float kSH3e = 1.4453057213202769f;

__device__ __forceinline__ void sh_values(int degree, float x, float y, float z, float Y[16]) {
    Y[0] = kSH0;
    if (degree < 1) return;
    Y[1] = kSH1 * y;
    Y[2] = kSH1 * z;
    Y[3] = kSH1 * x;
    if (degree < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kSH2a * x * y;
    Y[5] = kSH2a * y * z;
    Y[6] = kSH2b * (2.f * zz - xx - yy);
    Y[7] = kSH2a * x * z;
    Y[8] = kSH2c * (xx - yy);
    if (degree < 3) return;
    const float r1 = 4.f * zz - xx - yy;
    Y[9] = kSH3a * y * (3.f * xx - yy);
    Y[10] = kSH3b * x * y * z;
    Y[11] = kSH3c * y * r1;
    Y[12] = kSH3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
    Y[13] = kSH3c * x * r1;
    Y[14] = kSH3e * z * (xx - yy);
    Y[15] = kSH3a * x * (xx - 3.f * yy);
}

// Accumulates g += sum_k w[k] * grad Y_k(x, y, z).
__device__ __forceinline__ void sh_grad_dot(int degree, float x, float y, float z, const float w[16],
                                            float &gx, float &gy, float &gz) {
    gx = 0.f; gy = 0.f; gz = 0.f;
    if (degree < 1) return;
    gy += kSH1 * w[1];
    gz += kSH1 * w[2];
    gx += kSH1 * w[3];
    if (degree < 2) return;
    gx += kSH2a * (w[4] * y + w[7] * z) + kSH2b * w[6] * (-2.f * x) + kSH2c * w[8] * (2.f * x);
    gy += kSH2a * (w[4] * x + w[5] * z) + kSH2b * w[6] * (-2.f * y) + kSH2c * w[8] * (-2.f * y);
    gz += kSH2a * (w[5] * y + w[7] * x) + kSH2b * w[6] * (4.f * z);
    if (degree < 3) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    const float r1 = 4.f * zz - xx - yy;
    // Y9 = a y (3x^2 - y^2)
    gx += kSH3a * w[9] * (6.f * x * y);
    gy += kSH3a * w[9] * (3.f * xx - 3.f * yy);
    // Y10 = b x y z
    gx += kSH3b * w[10] * (y * z);
    gy += kSH3b * w[10] * (x * z);
    gz += kSH3b * w[10] * (x * y);
    // Y11 = c y r1
    gx += kSH3c * w[11] * (-2.f * x * y);
    gy += kSH3c * w[11] * (r1 - 2.f * yy);
    gz += kSH3c * w[11] * (8.f * y * z);
    // Y12 = d z (2z^2 - 3x^2 - 3y^2)
    gx += kSH3d * w[12] * (-6.f * x * z);
    gy += kSH3d * w[12] * (-6.f * y * z);
    gz += kSH3d * w[12] * (6.f * zz - 3.f * xx - 3.f * yy);
    // Y13 = c x r1
    gx += kSH3c * w[13] * (r1 - 2.f * xx);
    gy += kSH3c * w[13] * (-2.f * x * y);
    gz += kSH3c * w[13] * (8.f * x * z);
    // Y14 = e z (x^2 - y^2)
    gx += kSH3e * w[14] * (2.f * x * z);
    gy += kSH3e * w[14] * (-2.f * y * z);
    gz += kSH3e * w[14] * (xx - yy);
    // Y15 = a x (x^2 - 3y^2)
    gx += kSH3a * w[15] * (3.f * xx - 3.f * yy);
    gy += kSH3a * w[15] * (-6.f * x * y);
}

}  // namespace dpr

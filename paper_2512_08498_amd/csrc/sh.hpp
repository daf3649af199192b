// Real orthonormal spherical harmonics up to degree 3 and the gradient of a
// weighted sum of them with respect to the (unnormalised-treated) direction.
// Order k = l^2 + l + m, m = -l..l; constant of Y_lm is
// sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) times the Cartesian factor below.
#pragma once

#include "common.hpp"

namespace gsr {

constexpr float kSh0 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
constexpr float kSh1 = 0.4886025119029199f;    // sqrt(3/(4 pi))
constexpr float kSh2a = 1.0925484305920792f;   // sqrt(15/pi)/2
constexpr float kSh2b = 0.31539156525252005f;  // sqrt(5/pi)/4
constexpr float kSh2c = 0.5462742152960396f;   // sqrt(15/pi)/4
constexpr float kSh3a = 0.5900435899266435f;   // sqrt(35/(2 pi))/4
constexpr float kSh3b = 2.890611442640554f;    // sqrt(105/pi)/2
constexpr float kSh3c = 0.4570457994644658f;   // sqrt(21/(2 pi))/4
constexpr float kSh3d = 0.3731763325901154f;   // sqrt(7/pi)/4
constexpr float kSh3e = 1.445305721320277f;    // sqrt(105/pi)/4

__device__ __forceinline__ void sh_basis(float x, float y, float z, int deg, float Y[16]) {
  Y[0] = kSh0;
  if (deg < 1) return;
  Y[1] = -kSh1 * y;
  Y[2] = kSh1 * z;
  Y[3] = -kSh1 * x;
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = kSh2a * x * y;
  Y[5] = -kSh2a * y * z;
  Y[6] = kSh2b * (2.0f * zz - xx - yy);
  Y[7] = -kSh2a * x * z;
  Y[8] = kSh2c * (xx - yy);
  if (deg < 3) return;
  Y[9] = -kSh3a * y * (3.0f * xx - yy);
  Y[10] = kSh3b * x * y * z;
  Y[11] = -kSh3c * y * (4.0f * zz - xx - yy);
  Y[12] = kSh3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
  Y[13] = -kSh3c * x * (4.0f * zz - xx - yy);
  Y[14] = kSh3e * z * (xx - yy);
  Y[15] = -kSh3a * x * (xx - 3.0f * yy);
}

// g = sum_k w[k] * (dY_k/dx, dY_k/dy, dY_k/dz), the polynomials' partials.
__device__ __forceinline__ void sh_grad_dot(float x, float y, float z, int deg, const float w[16],
                                            float g[3]) {
  g[0] = g[1] = g[2] = 0.0f;
  if (deg < 1) return;
  g[0] += -kSh1 * w[3];
  g[1] += -kSh1 * w[1];
  g[2] += kSh1 * w[2];
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  // Y4 = a xy, Y5 = -a yz, Y6 = b (2zz - xx - yy), Y7 = -a xz, Y8 = c (xx - yy)
  g[0] += kSh2a * y * w[4] - 2.0f * kSh2b * x * w[6] - kSh2a * z * w[7] + 2.0f * kSh2c * x * w[8];
  g[1] += kSh2a * x * w[4] - kSh2a * z * w[5] - 2.0f * kSh2b * y * w[6] - 2.0f * kSh2c * y * w[8];
  g[2] += -kSh2a * y * w[5] + 4.0f * kSh2b * z * w[6] - kSh2a * x * w[7];
  if (deg < 3) return;
  // Y9  = -a y (3xx - yy)            Y10 = b xyz
  // Y11 = -c y (4zz - xx - yy)       Y12 = d z (2zz - 3xx - 3yy)
  // Y13 = -c x (4zz - xx - yy)       Y14 = e z (xx - yy)
  // Y15 = -a x (xx - 3yy)
  g[0] += -6.0f * kSh3a * x * y * w[9] + kSh3b * y * z * w[10] + 2.0f * kSh3c * x * y * w[11] -
          6.0f * kSh3d * x * z * w[12] - kSh3c * (4.0f * zz - 3.0f * xx - yy) * w[13] +
          2.0f * kSh3e * x * z * w[14] - kSh3a * (3.0f * xx - 3.0f * yy) * w[15];
  g[1] += -kSh3a * (3.0f * xx - 3.0f * yy) * w[9] + kSh3b * x * z * w[10] -
          kSh3c * (4.0f * zz - xx - 3.0f * yy) * w[11] - 6.0f * kSh3d * y * z * w[12] +
          2.0f * kSh3c * x * y * w[13] - 2.0f * kSh3e * y * z * w[14] + 6.0f * kSh3a * x * y * w[15];
  g[2] += kSh3b * x * y * w[10] - 8.0f * kSh3c * y * z * w[11] +
          kSh3d * (6.0f * zz - 3.0f * xx - 3.0f * yy) * w[12] - 8.0f * kSh3c * x * z * w[13] +
          kSh3e * (xx - yy) * w[14];
}

}  // namespace gsr

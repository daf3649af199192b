// FP32 binning rules evaluated on the device.
//
// Visibility, depth bits and the pixel box decide which (tile, Gaussian)
// pairs exist and in what order, so they must come out bit-identical to the
// reference evaluation.  Every operation below rounds once, in the written
// order: contraction into FMA is switched off, division and square root are
// the correctly rounded IEEE operations (the HIP default), and exp is the
// project's own Cody-Waite + polynomial exponential built from + - * only.
#pragma once

#include "common.hpp"

namespace gsr {

// exp(x) = 2^k exp(r), k = rint(x log2 e), r = (x - k ln2_hi) - k ln2_lo,
// exp(r) by its degree-7 Taylor polynomial (|r| <= ln2/2), 2^k placed in the
// exponent field.  ln2_hi has 9 significant bits so k * ln2_hi is exact.
__device__ __forceinline__ float bexp32(float x) {
#pragma clang fp contract(off)
  if (x != x) return x;
  if (x > 88.0f) return __builtin_inff();
  if (x < -86.0f) return 0.0f;
  const float t = x * kLog2e;
  const float k = (t + 0x1.8p+23f) - 0x1.8p+23f;  // round to nearest integer
  const float r = (x - k * 0x1.63p-1f) - k * -0x1.bd0106p-13f;
  float p = 0x1.a01a02p-13f;    // 1/7!
  p = p * r + 0x1.6c16c2p-10f;  // 1/6!
  p = p * r + 0x1.111112p-7f;   // 1/5!
  p = p * r + 0x1.555556p-5f;   // 1/4!
  p = p * r + 0x1.555556p-3f;   // 1/3!
  p = p * r + 0.5f;
  p = p * r + 1.0f;
  p = p * r + 1.0f;
  const int ki = (int)k;
  const float scale = __uint_as_float((uint32_t)(ki + 127) << 23);
  return p * scale;
}

// Everything the forward and the backward need from one (view, Gaussian).
struct Proj {
  bool visible;
  int i0, i1, j0, j1;   // inclusive pixel box, clamped to the image
  uint32_t zbits;
  float qn[4];          // unit quaternion (w, x, y, z)
  float rq[3][3];       // its rotation matrix
  float s[3];           // scales exp(log_scale)
  float xc, yc, zc;     // camera-space centre
  float xz, yz;         // xc / zc, yc / zc
  bool clx, cly;        // Jacobian guard active
  float xt, yt;         // clamped xz, yz
  float j00, j02, j11, j12;
  float t0[3], t1[3];   // rows of J R_view
  float a0[3], a1[3];   // rows of A = J R_view R_q diag(s)
  float p0, p1;         // |a0|^2, |a1|^2 (undilated covariance diagonal)
};

// The binning rules, step for step.  mean/ls/q are one Gaussian's float32
// parameters, c the camera.
__device__ __forceinline__ void project_spec(const float mean[3], const float ls[3],
                                             const float q[4], const Cam &c, Proj &o) {
#pragma clang fp contract(off)
  o.visible = false;
  // 1. normalise the quaternion
  const float n2 = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
  const bool q_ok = n2 > 0.0f;
  const float nrm = sqrtf(q_ok ? n2 : 1.0f);
  const float qw = q[0] / nrm, qx = q[1] / nrm, qy = q[2] / nrm, qz = q[3] / nrm;
  o.qn[0] = qw; o.qn[1] = qx; o.qn[2] = qy; o.qn[3] = qz;
  // 2. rotation of the unit quaternion
  o.rq[0][0] = 1.0f - 2.0f * (qy * qy + qz * qz);
  o.rq[0][1] = 2.0f * (qx * qy - qw * qz);
  o.rq[0][2] = 2.0f * (qx * qz + qw * qy);
  o.rq[1][0] = 2.0f * (qx * qy + qw * qz);
  o.rq[1][1] = 1.0f - 2.0f * (qx * qx + qz * qz);
  o.rq[1][2] = 2.0f * (qy * qz - qw * qx);
  o.rq[2][0] = 2.0f * (qx * qz - qw * qy);
  o.rq[2][1] = 2.0f * (qy * qz + qw * qx);
  o.rq[2][2] = 1.0f - 2.0f * (qx * qx + qy * qy);
  // 3-4. scales and M = R_q diag(s)
  float m[3][3];
  for (int j = 0; j < 3; ++j) o.s[j] = bexp32(ls[j]);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) m[i][j] = o.rq[i][j] * o.s[j];
  // 5. camera-space centre
  const float *R = c.R;
  o.xc = ((R[0] * mean[0] + R[1] * mean[1]) + R[2] * mean[2]) + c.t[0];
  o.yc = ((R[3] * mean[0] + R[4] * mean[1]) + R[5] * mean[2]) + c.t[1];
  o.zc = ((R[6] * mean[0] + R[7] * mean[1]) + R[8] * mean[2]) + c.t[2];
  const bool z_ok = o.zc > kNearZ;
  // 6. projected centre
  o.xz = o.xc / o.zc;
  o.yz = o.yc / o.zc;
  const float u = c.fx * o.xz + c.cx;
  const float v = c.fy * o.yz + c.cy;
  // 7. Jacobian guard
  const float wf = (float)c.w, hf = (float)c.h;
  const float lim_x = kClampFov * (fmaxf(c.cx, wf - c.cx) / c.fx);
  const float lim_y = kClampFov * (fmaxf(c.cy, hf - c.cy) / c.fy);
  o.xt = fminf(fmaxf(o.xz, -lim_x), lim_x);
  o.yt = fminf(fmaxf(o.yz, -lim_y), lim_y);
  o.clx = (o.xz < -lim_x) || (o.xz > lim_x);
  o.cly = (o.yz < -lim_y) || (o.yz > lim_y);
  // 8. Jacobian
  o.j00 = c.fx / o.zc;
  o.j02 = -((c.fx * o.xt) / o.zc);
  o.j11 = c.fy / o.zc;
  o.j12 = -((c.fy * o.yt) / o.zc);
  // 9. T = J R_view
  for (int k = 0; k < 3; ++k) {
    o.t0[k] = o.j00 * R[k] + o.j02 * R[6 + k];
    o.t1[k] = o.j11 * R[3 + k] + o.j12 * R[6 + k];
  }
  // 10. A = T M
  for (int k = 0; k < 3; ++k) {
    o.a0[k] = (o.t0[0] * m[0][k] + o.t0[1] * m[1][k]) + o.t0[2] * m[2][k];
    o.a1[k] = (o.t1[0] * m[0][k] + o.t1[1] * m[1][k]) + o.t1[2] * m[2][k];
  }
  // 11. covariance diagonal, then 12. box half extents
  o.p0 = (o.a0[0] * o.a0[0] + o.a0[1] * o.a0[1]) + o.a0[2] * o.a0[2];
  o.p1 = (o.a1[0] * o.a1[0] + o.a1[1] * o.a1[1]) + o.a1[2] * o.a1[2];
  const float sxx = o.p0 + kDilation;
  const float syy = o.p1 + kDilation;
  const float hx = sqrtf(kSupportK * sxx);
  const float hy = sqrtf(kSupportK * syy);
  // 13. pixel box
  const bool finite = isfinite(u) && isfinite(v) && isfinite(hx) && isfinite(hy);
  if (!(q_ok && z_ok && finite)) return;
  const int i0 = (int)fminf(fmaxf(ceilf((u - hx) - 0.5f), -1.0f), wf);
  const int i1 = (int)fminf(fmaxf(floorf((u + hx) - 0.5f), -1.0f), wf);
  const int j0 = (int)fminf(fmaxf(ceilf((v - hy) - 0.5f), -1.0f), hf);
  const int j1 = (int)fminf(fmaxf(floorf((v + hy) - 0.5f), -1.0f), hf);
  // 14. visibility, then clamp to the image
  if (!(i0 <= i1 && j0 <= j1 && i1 >= 0 && i0 <= c.w - 1 && j1 >= 0 && j0 <= c.h - 1)) return;
  o.visible = true;
  o.i0 = max(i0, 0);
  o.i1 = min(i1, c.w - 1);
  o.j0 = max(j0, 0);
  o.j1 = min(j1, c.h - 1);
  // 16. depth bits
  o.zbits = __float_as_uint(o.zc);
}

__device__ __forceinline__ void load_gaussian(const float *__restrict__ mean, const float *__restrict__ ls,
                                              const float *__restrict__ quat, int64_t n, int64_t g,
                                              float m3[3], float l3[3], float q4[4]) {
  for (int k = 0; k < 3; ++k) {
    m3[k] = mean[k * n + g];
    l3[k] = ls[k * n + g];
  }
  for (int k = 0; k < 4; ++k) q4[k] = quat[k * n + g];
}

__device__ __forceinline__ Cam load_cam(const Cam *__restrict__ cams, int v) {
  Cam c;
  const float *src = reinterpret_cast<const float *>(cams + v);
  float *dst = reinterpret_cast<float *>(&c);
#pragma unroll
  for (int k = 0; k < 18; ++k) dst[k] = src[k];
  return c;
}

}  // namespace gsr

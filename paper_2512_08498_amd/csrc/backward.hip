// Per-Gaussian backward: from each record's reduced 2D gradients to the
// Gaussian's parameters, summed over all views in registers; optionally
// followed directly by the Adam update (so gradients never reach memory).
//
// Chain, per view (notation of spec.hpp / preprocess.hip):
//   (qa, qb, qc) -> 2D covariance S:  qa = k S_yy/det, qb = -S_xy/S_yy,
//                                     qc = k/S_yy, k = -log2(e)/2
//   S = A A^T + 0.3 I,  A = T M,  T = J R_view,  M = R(q) diag(exp(l))
//   J(x_c) with the guard clamp (zero derivative where it clamps)
//   mean offset -> 2D mean -> x_c = R_view mu + t
//   colour = max(0, sum sh Y(d) + 0.5) -> SH coefficients and d -> mu
//   opacity = sigmoid(theta)
// and, once over all views, the quaternion normalisation.  With CAM each
// record also leaves its view's pose gradient through the geometry (T = J R
// and x_c = R mu + t; the SH direction is detached from the pose) in cam_rec,
// 12 floats per record, for the per-view sums of pose.hip.
#include <algorithm>

#include "kernels.hpp"
#include "sh.hpp"
#include "spec.hpp"
#include "util.hpp"

namespace gsr {

__device__ __forceinline__ void adam_update(float &p, float &m, float &v, float g, float lr, float b1, float b2,
                                            float eps, float bc1, float bc2) {
  m = b1 * m + (1.0f - b1) * g;
  v = b2 * v + (1.0f - b2) * g * g;
  const float mh = m / bc1, vh = v / bc2;
  p = p - lr * mh / (sqrtf(vh) + eps);
}

__device__ __forceinline__ void bias_corrections(const AdamArgs &a, float &bc1, float &bc2) {
  const float t = (float)(*a.step);
  bc1 = 1.0f - exp2f(t * log2f(a.beta1));
  bc2 = 1.0f - exp2f(t * log2f(a.beta2));
}

// Colour cotangent of record r: dL/drgb where the channel was not clamped.
__device__ __forceinline__ void colour_cot(const Ws &ws, uint32_t r, float c[3]) {
  const float4 gb = ws.g2d[(size_t)r * 3 + 1], gc = ws.g2d[(size_t)r * 3 + 2];
  const uint32_t pass = __float_as_uint(ws.rec_payload[(size_t)r * 4 + 3].w);
  c[0] = (pass & 1u) ? gb.z : 0.0f;
  c[1] = (pass & 2u) ? gb.w : 0.0f;
  c[2] = (pass & 4u) ? gc.x : 0.0f;
}

// Unit direction from the camera centre -R^T t to the mean, and 1/|mean - C|.
__device__ __forceinline__ void view_dir(const Cam &c, const float m3[3], float d[3], float &inv) {
  const float cxw = -(c.R[0] * c.t[0] + c.R[3] * c.t[1] + c.R[6] * c.t[2]);
  const float cyw = -(c.R[1] * c.t[0] + c.R[4] * c.t[1] + c.R[7] * c.t[2]);
  const float czw = -(c.R[2] * c.t[0] + c.R[5] * c.t[1] + c.R[8] * c.t[2]);
  const float ex = m3[0] - cxw, ey = m3[1] - cyw, ez = m3[2] - czw;
  inv = 1.0f / sqrtf(ex * ex + ey * ey + ez * ez);
  d[0] = ex * inv;
  d[1] = ey * inv;
  d[2] = ez * inv;
}

template <int NN>
struct GroupN {
  static constexpr int N = NN;
};

// Three waves per SIMD: the CAM variant's extra live values would otherwise
// push the degree-3 kernel past 168 registers and down to one or two waves,
// which costs more than the few spills that keep it at three.
template <int DEG, bool ADAM, bool CAM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_pre_bwd(
    GaussPtrs gp, const Cam *__restrict__ cams, Ws ws, Sizes sz, MutPtrs grads, int accumulate, AdamArgs adam,
    float4 *__restrict__ cam_rec) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  if (ws.scalars[kOverflow]) return;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= sz.n) return;
  const int64_t n = sz.n;
  float m3[3], l3[3], q4[4];
  load_gaussian(gp.mean, gp.log_scale, gp.quat, n, g, m3, l3, q4);
  float d_mean[3] = {0.f, 0.f, 0.f}, d_s[3] = {0.f, 0.f, 0.f}, d_op = 0.f;
  float d_rq[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
  Proj P;
  bool seen = false;
  const uint32_t r0 = ws.rec_start[g], r1 = ws.rec_start[g + 1];

  // pass 1: geometry and opacity (the colour's dependence on the direction
  // is added in pass 2, where the SH coefficients are in registers)
  for (uint32_t r = r0; r < r1; ++r) {
    const int v = (int)ws.rec_view[r];
    const Cam c = load_cam(cams, v);
    project_spec(m3, l3, q4, c, P);
    seen = true;
    const float4 ga = ws.g2d[(size_t)r * 3 + 0], gb = ws.g2d[(size_t)r * 3 + 1];
    const float d_offx = ga.x, d_offy = ga.y, d_qa = ga.z, d_qb = ga.w, d_qc = gb.x;
    d_op += gb.y;


    // conic (Cholesky form) -> 2D covariance
    const float syy = P.p1 + kDilation;
    const float sxy = (P.a0[0] * P.a1[0] + P.a0[1] * P.a1[1]) + P.a0[2] * P.a1[2];
    const float cx_ = P.a0[1] * P.a1[2] - P.a0[2] * P.a1[1];
    const float cy_ = P.a0[2] * P.a1[0] - P.a0[0] * P.a1[2];
    const float cz_ = P.a0[0] * P.a1[1] - P.a0[1] * P.a1[0];
    const float det = (cx_ * cx_ + cy_ * cy_ + cz_ * cz_) + kDilation * (P.p0 + P.p1) + kDilation * kDilation;
    const float kk = -kHalfLog2e;
    const float inv_det = 1.0f / det, inv_syy = 1.0f / syy;
    const float qa = kk * syy * inv_det;
    const float dSxx = d_qa * (-qa * syy * inv_det);
    const float dSyy = d_qa * (-kk * sxy * sxy * inv_det * inv_det) + d_qb * (sxy * inv_syy * inv_syy) +
                       d_qc * (-kk * inv_syy * inv_syy);
    const float dSxy = d_qa * (2.0f * kk * syy * sxy * inv_det * inv_det) - d_qb * inv_syy;
    // S = A A^T + 0.3 I
    float dA0[3], dA1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      dA0[k] = 2.0f * dSxx * P.a0[k] + dSxy * P.a1[k];
      dA1[k] = dSxy * P.a0[k] + 2.0f * dSyy * P.a1[k];
    }
    // A = T M,  M = R_q diag(s)
    float dT0[3] = {0.f, 0.f, 0.f}, dT1[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float mik = P.rq[i][k] * P.s[k];
        const float dM = P.t0[i] * dA0[k] + P.t1[i] * dA1[k];
        d_s[k] += dM * P.rq[i][k];
        d_rq[i][k] += dM * P.s[k];
        dT0[i] += dA0[k] * mik;
        dT1[i] += dA1[k] * mik;
      }
    }
    // T = J R_view
    const float *R = c.R;
    const float dj00 = dT0[0] * R[0] + dT0[1] * R[1] + dT0[2] * R[2];
    const float dj02 = dT0[0] * R[6] + dT0[1] * R[7] + dT0[2] * R[8];
    const float dj11 = dT1[0] * R[3] + dT1[1] * R[4] + dT1[2] * R[5];
    const float dj12 = dT1[0] * R[6] + dT1[1] * R[7] + dT1[2] * R[8];
    const float z = P.zc, iz = 1.0f / z, iz2 = iz * iz;
    float dxc = 0.f, dyc = 0.f, dzc = 0.f;
    dzc += -dj00 * c.fx * iz2 - dj11 * c.fy * iz2;
    if (!P.clx) {
      dxc += -dj02 * c.fx * iz2;
      dzc += dj02 * 2.0f * c.fx * P.xc * iz2 * iz;
    } else {
      dzc += dj02 * c.fx * P.xt * iz2;
    }
    if (!P.cly) {
      dyc += -dj12 * c.fy * iz2;
      dzc += dj12 * 2.0f * c.fy * P.yc * iz2 * iz;
    } else {
      dzc += dj12 * c.fy * P.yt * iz2;
    }
    // 2D mean (the offset differs from it by a constant)
    dxc += d_offx * c.fx * iz;
    dyc += d_offy * c.fy * iz;
    dzc += -(d_offx * c.fx * P.xc + d_offy * c.fy * P.yc) * iz2;
    // x_c = R_view mu + t
    d_mean[0] += R[0] * dxc + R[3] * dyc + R[6] * dzc;
    d_mean[1] += R[1] * dxc + R[4] * dyc + R[7] * dzc;
    d_mean[2] += R[2] * dxc + R[5] * dyc + R[8] * dzc;
    if (CAM) {
      // dL/dR_view: rows of T = J R (row 0 = j00 R_0 + j02 R_2, row 1 =
      // j11 R_1 + j12 R_2) plus x_c = R mu + t; dL/dt = dL/dx_c
      float4 *o = cam_rec + (size_t)r * 3;
      o[0] = make_float4(P.j00 * dT0[0] + dxc * m3[0], P.j00 * dT0[1] + dxc * m3[1], P.j00 * dT0[2] + dxc * m3[2],
                         P.j11 * dT1[0] + dyc * m3[0]);
      o[1] = make_float4(P.j11 * dT1[1] + dyc * m3[1], P.j11 * dT1[2] + dyc * m3[2],
                         (P.j02 * dT0[0] + P.j12 * dT1[0]) + dzc * m3[0],
                         (P.j02 * dT0[1] + P.j12 * dT1[1]) + dzc * m3[1]);
      o[2] = make_float4((P.j02 * dT0[2] + P.j12 * dT1[2]) + dzc * m3[2], dxc, dyc, dzc);
    }
  }

  // view-independent parts: scales, quaternion, opacity
  float d_l[3] = {0.f, 0.f, 0.f}, d_q[4] = {0.f, 0.f, 0.f, 0.f};
  if (seen) {
    d_l[0] = d_s[0] * P.s[0];
    d_l[1] = d_s[1] * P.s[1];
    d_l[2] = d_s[2] * P.s[2];
    const float w = P.qn[0], x = P.qn[1], y = P.qn[2], zq = P.qn[3];
    const float(&D)[3][3] = d_rq;
    const float gw = 2.f * (-zq * D[0][1] + y * D[0][2] + zq * D[1][0] - x * D[1][2] - y * D[2][0] + x * D[2][1]);
    const float gx = 2.f * (y * D[0][1] + zq * D[0][2] + y * D[1][0] - 2.f * x * D[1][1] - w * D[1][2] +
                            zq * D[2][0] + w * D[2][1] - 2.f * x * D[2][2]);
    const float gy = 2.f * (-2.f * y * D[0][0] + x * D[0][1] + w * D[0][2] + x * D[1][0] + zq * D[1][2] -
                            w * D[2][0] + zq * D[2][1] - 2.f * y * D[2][2]);
    const float gz = 2.f * (-2.f * zq * D[0][0] - w * D[0][1] + x * D[0][2] + w * D[1][0] - 2.f * zq * D[1][1] +
                            y * D[1][2] + x * D[2][0] + y * D[2][1]);
    const float qdot = gw * w + gx * x + gy * y + gz * zq;
    const float n2 = ((q4[0] * q4[0] + q4[1] * q4[1]) + q4[2] * q4[2]) + q4[3] * q4[3];
    const float inv_n = 1.0f / sqrtf(n2);
    d_q[0] = (gw - qdot * w) * inv_n;
    d_q[1] = (gx - qdot * x) * inv_n;
    d_q[2] = (gy - qdot * y) * inv_n;
    d_q[3] = (gz - qdot * zq) * inv_n;
  }
  const float theta = gp.opacity_logit[g];
  const float op = 1.0f / (1.0f + expf(-theta));
  const float d_theta = op * (1.0f - op) * d_op;

  float bc1 = 1.0f, bc2 = 1.0f;
  if (ADAM) bias_corrections(adam, bc1, bc2);
  // Gradients of a group of N parameters (pointer offsets off[i] from the
  // group's arrays) whose current values pv the thread already holds.
  // Without Adam they are written out (or added).  With Adam a group's loads
  // (the moments, and the values unless the parameters are the forward's own
  // arrays) are issued apart from its update and stores, so the loads of
  // several groups are in flight before any of their stores: the three
  // view-independent groups together, and each SH group (then the mean)
  // while the group before it is stored.  Parameters, moments and gradient
  // outputs are distinct arrays, so no store feeds a later load.
  auto write_grads = [&](auto tag, float *gout, const int64_t(&off)[decltype(tag)::N],
                         const float(&gv)[decltype(tag)::N]) {
#pragma unroll
    for (int i = 0; i < decltype(tag)::N; ++i) gout[off[i]] = accumulate ? gout[off[i]] + gv[i] : gv[i];
  };
  auto adam_load = [&](auto tag, const float *p, const float *m, const float *v,
                       const int64_t(&off)[decltype(tag)::N], const float(&pv)[decltype(tag)::N],
                       float(&pp)[decltype(tag)::N], float(&mm)[decltype(tag)::N], float(&vv)[decltype(tag)::N]) {
#pragma unroll
    for (int i = 0; i < decltype(tag)::N; ++i) {
      pp[i] = adam.p_is_g ? pv[i] : p[off[i]];
      mm[i] = m[off[i]];
      vv[i] = v[off[i]];
    }
  };
  auto adam_store = [&](auto tag, float *p, float *m, float *v, float *gout, const int64_t(&off)[decltype(tag)::N],
                        float(&pp)[decltype(tag)::N], float(&mm)[decltype(tag)::N], float(&vv)[decltype(tag)::N],
                        const float(&gv)[decltype(tag)::N], const float(&lr)[decltype(tag)::N]) {
    constexpr int N = decltype(tag)::N;
#pragma unroll
    for (int i = 0; i < N; ++i) adam_update(pp[i], mm[i], vv[i], gv[i], lr[i], adam.beta1, adam.beta2, adam.eps, bc1, bc2);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      p[off[i]] = pp[i];
      m[off[i]] = mm[i];
      v[off[i]] = vv[i];
      if (gout) gout[off[i]] = gv[i];
    }
  };

  // the view-independent groups, from the values loaded at the start
  {
    const int64_t o3[3] = {g, n + g, 2 * n + g}, o4[4] = {g, n + g, 2 * n + g, 3 * n + g}, o1[1] = {g};
    const float lr1[3] = {adam.lr[1], adam.lr[1], adam.lr[1]};
    const float lr2[4] = {adam.lr[2], adam.lr[2], adam.lr[2], adam.lr[2]}, lr3[1] = {adam.lr[3]};
    const float gth[1] = {d_theta}, th[1] = {theta};
    if (!ADAM) {
      write_grads(GroupN<3>{}, grads.log_scale, o3, d_l);
      write_grads(GroupN<4>{}, grads.quat, o4, d_q);
      write_grads(GroupN<1>{}, grads.opacity_logit, o1, gth);
    } else {
      float ps[3], ms[3], vs[3], pq[4], mq[4], vq[4], po[1], mo[1], vo[1];
      adam_load(GroupN<3>{}, adam.p.log_scale, adam.m.log_scale, adam.v.log_scale, o3, l3, ps, ms, vs);
      adam_load(GroupN<4>{}, adam.p.quat, adam.m.quat, adam.v.quat, o4, q4, pq, mq, vq);
      adam_load(GroupN<1>{}, adam.p.opacity_logit, adam.m.opacity_logit, adam.v.opacity_logit, o1, th, po, mo, vo);
      adam_store(GroupN<3>{}, adam.p.log_scale, adam.m.log_scale, adam.v.log_scale, grads.log_scale, o3, ps, ms, vs,
                 d_l, lr1);
      adam_store(GroupN<4>{}, adam.p.quat, adam.m.quat, adam.v.quat, grads.quat, o4, pq, mq, vq, d_q, lr2);
      adam_store(GroupN<1>{}, adam.p.opacity_logit, adam.m.opacity_logit, adam.v.opacity_logit,
                 grads.opacity_logit, o1, po, mo, vo, gth, lr3);
    }
  }

  // pass 2: the SH coefficients, loaded once (the values the Adam update
  // starts from too), and one walk over the records for the colour's
  // dependence on the viewing direction and the coefficients' gradient sums;
  // those sums sit in this thread's column of LDS (registers would spill),
  // then the updates go in groups of two coefficients (six parameters; three
  // at degree 2)
  float shv[K][3];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) shv[k][ch] = gp.sh[((int64_t)k * 3 + ch) * n + g];
  __shared__ float a_lds[3 * K][256];
  const int tc = (int)threadIdx.x;
#pragma unroll
  for (int i = 0; i < 3 * K; ++i) a_lds[i][tc] = 0.0f;
  float d_dir[3] = {0.f, 0.f, 0.f};
  for (uint32_t r = r0; r < r1; ++r) {
    const Cam c = load_cam(cams, (int)ws.rec_view[r]);
    float cc[3], d[3], inv;
    colour_cot(ws, r, cc);
    view_dir(c, m3, d, inv);
    {
      float Y[16];
      sh_basis(d[0], d[1], d[2], DEG, Y);
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) a_lds[3 * k + ch][tc] += Y[k] * cc[ch];
    }
    if (DEG > 0) {
      float w[16];
      w[0] = 0.0f;
#pragma unroll
      for (int k = 1; k < K; ++k) w[k] = cc[0] * shv[k][0] + cc[1] * shv[k][1] + cc[2] * shv[k][2];
#pragma unroll
      for (int k = K; k < 16; ++k) w[k] = 0.0f;
      float gd[3];
      sh_grad_dot(d[0], d[1], d[2], DEG, w, gd);
      const float dot = gd[0] * d[0] + gd[1] * d[1] + gd[2] * d[2];
      d_dir[0] += (gd[0] - dot * d[0]) * inv;
      d_dir[1] += (gd[1] - dot * d[1]) * inv;
      d_dir[2] += (gd[2] - dot * d[2]) * inv;
    }
  }
  // coefficients per group: a divisor of K (degree 2 has nine), so no group
  // runs past the last coefficient
  constexpr int KC = K % 2 == 0 ? 2 : (K % 3 == 0 ? 3 : 1);
  constexpr int NG = 3 * KC;
  // offsets, current values and learning rates of the SH group at kc
  auto sh_group = [&](int kc, int64_t(&off)[NG], float(&pv)[NG], float(&lr)[NG]) {
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const int k = kc + kk;
        off[3 * kk + ch] = ((int64_t)k * 3 + ch) * n + g;
        pv[3 * kk + ch] = shv[k][ch];
        lr[3 * kk + ch] = k == 0 ? adam.lr[4] : adam.lr[5];
      }
  };
  auto sh_grads = [&](int kc, float(&gv)[NG]) {
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) gv[3 * kk + ch] = a_lds[3 * (kc + kk) + ch][tc];
  };
  const float dm[3] = {d_mean[0] + d_dir[0], d_mean[1] + d_dir[1], d_mean[2] + d_dir[2]};
  const int64_t o3[3] = {g, n + g, 2 * n + g};
  const float lr0[3] = {adam.lr[0], adam.lr[0], adam.lr[0]};
  if (!ADAM) {
#pragma unroll
    for (int kc = 0; kc < K; kc += KC) {
      int64_t off[NG];
      float pv[NG], gv[NG], lr[NG];
      sh_group(kc, off, pv, lr);
      sh_grads(kc, gv);
      write_grads(GroupN<NG>{}, grads.sh, off, gv);
    }
    // the mean, now that the direction term is in
    write_grads(GroupN<3>{}, grads.mean, o3, dm);
  } else {
    // only the loaded values are carried from one group to the next; the
    // offsets and rates are recomputed
    float np[NG], nm[NG], nv[NG];
    {
      int64_t off[NG];
      float pv[NG], lr[NG];
      sh_group(0, off, pv, lr);
      adam_load(GroupN<NG>{}, adam.p.sh, adam.m.sh, adam.v.sh, off, pv, np, nm, nv);
    }
    float pmn[3], mmn[3], vmn[3];
#pragma unroll
    for (int kc = 0; kc < K; kc += KC) {
      float pp[NG], mm[NG], vv[NG];
#pragma unroll
      for (int i = 0; i < NG; ++i) {
        pp[i] = np[i];
        mm[i] = nm[i];
        vv[i] = nv[i];
      }
      if (kc + KC < K) {
        int64_t off[NG];
        float pv[NG], lr[NG];
        sh_group(kc + KC, off, pv, lr);
        adam_load(GroupN<NG>{}, adam.p.sh, adam.m.sh, adam.v.sh, off, pv, np, nm, nv);
      } else {
        adam_load(GroupN<3>{}, adam.p.mean, adam.m.mean, adam.v.mean, o3, m3, pmn, mmn, vmn);
      }
      int64_t off[NG];
      float pv[NG], lr[NG], gv[NG];
      sh_group(kc, off, pv, lr);
      sh_grads(kc, gv);
      adam_store(GroupN<NG>{}, adam.p.sh, adam.m.sh, adam.v.sh, grads.sh, off, pp, mm, vv, gv, lr);
    }
    // the mean, now that the direction term is in
    adam_store(GroupN<3>{}, adam.p.mean, adam.m.mean, adam.v.mean, grads.mean, o3, pmn, mmn, vmn, dm, lr0);
  }
}

__global__ void k_step_inc(int32_t *step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *step += 1;
}

// Dense Adam over the six parameter groups in one launch.
struct AdamSeg {
  float *p, *g, *m, *v;
  int64_t count;
  float lr;
};
struct AdamSegs {
  AdamSeg s[6];
};

__global__ __launch_bounds__(256) void k_adam(AdamSegs segs, float b1, float b2, float eps, const int32_t *step,
                                               int64_t total) {
  const float t = (float)(*step);
  const float bc1 = 1.0f - exp2f(t * log2f(b1));
  const float bc2 = 1.0f - exp2f(t * log2f(b2));
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    int64_t j = i;
    int s = 0;
    while (s < 5 && j >= segs.s[s].count) {
      j -= segs.s[s].count;
      ++s;
    }
    const AdamSeg &S = segs.s[s];
    float p = S.p[j], m = S.m[j], v = S.v[j];
    adam_update(p, m, v, S.g[j], S.lr, b1, b2, eps, bc1, bc2);
    S.p[j] = p;
    S.m[j] = m;
    S.v[j] = v;
  }
}

void launch_pre_bwd(const GaussPtrs &gp, const Cam *cams, const Ws &ws, const Sizes &sz, int sh_degree,
                    const MutPtrs *grads, int accumulate, const AdamArgs *adam, float4 *cam_rec, hipStream_t st) {
  if (sz.n == 0) return;
  const unsigned blocks = (unsigned)((sz.n + 255) / 256);
  MutPtrs gr = grads ? *grads : MutPtrs{nullptr, nullptr, nullptr, nullptr, nullptr};
  AdamArgs a{};
  if (adam) a = *adam;
#define GSR_PRE_BWD_C(D, A)                                                                        \
  if (cam_rec)                                                                                     \
    k_pre_bwd<D, A, true><<<blocks, 256, 0, st>>>(gp, cams, ws, sz, gr, accumulate, a, cam_rec);   \
  else                                                                                             \
    k_pre_bwd<D, A, false><<<blocks, 256, 0, st>>>(gp, cams, ws, sz, gr, accumulate, a, nullptr);
#define GSR_PRE_BWD(D)      \
  if (adam) {               \
    GSR_PRE_BWD_C(D, true)  \
  } else {                  \
    GSR_PRE_BWD_C(D, false) \
  }
  switch (sh_degree) {
    case 0: GSR_PRE_BWD(0) break;
    case 1: GSR_PRE_BWD(1) break;
    case 2: GSR_PRE_BWD(2) break;
    default: GSR_PRE_BWD(3) break;
  }
#undef GSR_PRE_BWD
#undef GSR_PRE_BWD_C
}

void launch_step_inc(int32_t *step, hipStream_t st) { k_step_inc<<<1, 64, 0, st>>>(step); }

void launch_adam(const MutPtrs &g, const AdamArgs &a, int64_t n, int sh_degree, hipStream_t st) {
  const int64_t K = (int64_t)(sh_degree + 1) * (sh_degree + 1);
  AdamSegs s;
  s.s[0] = {a.p.mean, g.mean, a.m.mean, a.v.mean, 3 * n, a.lr[0]};
  s.s[1] = {a.p.log_scale, g.log_scale, a.m.log_scale, a.v.log_scale, 3 * n, a.lr[1]};
  s.s[2] = {a.p.quat, g.quat, a.m.quat, a.v.quat, 4 * n, a.lr[2]};
  s.s[3] = {a.p.opacity_logit, g.opacity_logit, a.m.opacity_logit, a.v.opacity_logit, n, a.lr[3]};
  s.s[4] = {a.p.sh, g.sh, a.m.sh, a.v.sh, 3 * n, a.lr[4]};
  s.s[5] = {a.p.sh + 3 * n, g.sh + 3 * n, a.m.sh + 3 * n, a.v.sh + 3 * n, (K - 1) * 3 * n, a.lr[5]};
  const int64_t total = (11 + 3 * K) * n;
  if (total == 0) return;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 16384);
  k_adam<<<(unsigned)blocks, 256, 0, st>>>(s, a.beta1, a.beta2, a.eps, a.step, total);
}

}  // namespace gsr

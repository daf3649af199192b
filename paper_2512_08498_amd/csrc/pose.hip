// Camera-pose gradients and the rig parameterisation of the poses.
//
// The paper updates camera parameters jointly with the Gaussians, with the
// SH colour detached from that update (Sec. 3.3, "Optimization"), and links
// the rig's cameras rigidly: T_i^t = T_m^t T_{i->m} (Sec. 3.1, Eq. 3).  The
// per-Gaussian backward leaves each record's pose gradient (12 floats: dL/dR
// row-major, dL/dt) in a per-record buffer; here those are summed per view
// in a fixed order (one workgroup per 2048 consecutive records, then one
// block per view over the workgroups' partials), so the result does not
// depend on scheduling.  The rig kernels compose the views' poses from the
// central and relative transforms and carry the views' gradients back to
// them.
#include "kernels.hpp"
#include "util.hpp"

namespace gsr {

namespace {

constexpr int kCamPer = 8;                               // records per thread
constexpr uint32_t kCamChunk = 256u * (uint32_t)kCamPer;  // records per workgroup
constexpr int kCamGroup = 32;                            // views combined per LDS round

// Partials [block][view][12] of the records [block * 2048, +2048).  Thread
// t owns records i * 256 + t of the chunk (i = 0..7, so every load is
// coalesced) and loads all of them first; per view it adds its matching
// records in ascending i, each wave sums its lanes with the packed DPP
// butterfly, and the four waves' sums are added in wave order.
__global__ __launch_bounds__(256) void k_cam_reduce(const float4 *__restrict__ cam_rec,
                                                    const uint32_t *__restrict__ rec_view,
                                                    const uint32_t *__restrict__ scalars, int n_views,
                                                    float *__restrict__ part) {
  if (scalars[kOverflow]) return;
  const uint32_t nrec = scalars[kNumRecords];
  const uint32_t base = blockIdx.x * kCamChunk;
  if (base >= nrec) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  uint32_t vw[kCamPer];
  float4 x[kCamPer][3];
#pragma unroll
  for (int i = 0; i < kCamPer; ++i) {
    const uint32_t r = base + (uint32_t)i * 256u + (uint32_t)tid;
    const bool ok = r < nrec;
    vw[i] = ok ? rec_view[r] : 0xFFFFFFFFu;
#pragma unroll
    for (int k = 0; k < 3; ++k) x[i][k] = ok ? cam_rec[(size_t)r * 3 + k] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  __shared__ float lds[4][kCamGroup][12];
  float *out = part + (size_t)blockIdx.x * (size_t)n_views * 12;
  for (int g0 = 0; g0 < n_views; g0 += kCamGroup) {
    const int gn = n_views - g0 < kCamGroup ? n_views - g0 : kCamGroup;
    for (int j = 0; j < gn; ++j) {
      const uint32_t v = (uint32_t)(g0 + j);
      float a[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) a[k] = 0.0f;
      bool hit = false;
#pragma unroll
      for (int i = 0; i < kCamPer; ++i) {
        const bool m = vw[i] == v;
        hit |= m;
        a[0] += m ? x[i][0].x : 0.f; a[1] += m ? x[i][0].y : 0.f; a[2] += m ? x[i][0].z : 0.f;
        a[3] += m ? x[i][0].w : 0.f; a[4] += m ? x[i][1].x : 0.f; a[5] += m ? x[i][1].y : 0.f;
        a[6] += m ? x[i][1].z : 0.f; a[7] += m ? x[i][1].w : 0.f; a[8] += m ? x[i][2].x : 0.f;
        a[9] += m ? x[i][2].y : 0.f; a[10] += m ? x[i][2].z : 0.f; a[11] += m ? x[i][2].w : 0.f;
      }
      if (__ballot(hit) == 0) {
        if (lane < 12) lds[w][j][lane] = 0.0f;
        continue;
      }
      const float lo[9] = {a[0], a[1], a[2], a[3], a[4], a[5], a[6], a[7], a[8]};
      const float hi[9] = {a[9], a[10], a[11], 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      const float s = wave_sum9_packed(lo);
      const float t = wave_sum9_packed(hi);
      if (lane < 8) lds[w][j][lane] = s;
      if (lane == 32) lds[w][j][8] = s;
      if (lane < 3) lds[w][j][9 + lane] = t;
    }
    __syncthreads();
    for (int e = tid; e < gn * 12; e += 256) {
      const int j = e / 12, k = e % 12;
      out[(size_t)(g0 + j) * 12 + k] = (lds[0][j][k] + lds[1][j][k]) + (lds[2][j][k] + lds[3][j][k]);
    }
    __syncthreads();
  }
}

// One block per view: value k of the view summed over the chunks, chunk b
// by slice b mod 16 in ascending b, then the 16 slices in order.
__global__ __launch_bounds__(192) void k_cam_final(const float *__restrict__ part,
                                                   const uint32_t *__restrict__ scalars, int n_views,
                                                   float *__restrict__ out, int accumulate) {
  if (scalars[kOverflow]) return;
  const uint32_t nrec = scalars[kNumRecords];
  const uint32_t nb = (nrec + kCamChunk - 1) / kCamChunk;
  const int v = blockIdx.x;
  const int k = threadIdx.x % 12, s = threadIdx.x / 12;
  float acc = 0.0f;
#pragma unroll 4
  for (uint32_t b = (uint32_t)s; b < nb; b += 16u) acc += part[((size_t)b * n_views + v) * 12 + k];
  __shared__ float red[16][12];
  red[s][k] = acc;
  __syncthreads();
  if (threadIdx.x < 12) {
    float t = 0.0f;
#pragma unroll
    for (int j = 0; j < 16; ++j) t += red[j][threadIdx.x];
    float *o = out + (size_t)v * 12 + threadIdx.x;
    *o = accumulate ? *o + t : t;
  }
}

// T_v = T_m^{f(v)} T_{c(v)->m}: R_v = R_m R_r, t_v = R_m t_r + t_m.
__global__ __launch_bounds__(64) void k_rig_compose(const float *__restrict__ central,
                                                    const float *__restrict__ relative, RigIdx ri, Cam *cams) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= ri.n_views) return;
  const float *m = central + 12 * ri.frame[v];
  const float *r = relative + 12 * ri.cam[v];
  float R[9], t[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) R[3 * i + j] = (m[3 * i] * r[j] + m[3 * i + 1] * r[3 + j]) + m[3 * i + 2] * r[6 + j];
    t[i] = ((m[3 * i] * r[9] + m[3 * i + 1] * r[10]) + m[3 * i + 2] * r[11]) + m[9 + i];
  }
  Cam &c = cams[v];
#pragma unroll
  for (int k = 0; k < 9; ++k) c.R[k] = R[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) c.t[k] = t[k];
}

// Gradient of a left perturbation T <- exp(xi^) T, xi = (rho, phi), from the
// matrix gradient (G, g) of T = (R, t): dL/drho = g,
// dL/dphi = sum_j R_col_j x G_col_j + t x g.
__device__ __forceinline__ void tangent(const float *T, const float G[12], float *xi) {
  float ph[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const float r0 = T[j], r1 = T[3 + j], r2 = T[6 + j];
    const float g0 = G[j], g1 = G[3 + j], g2 = G[6 + j];
    ph[0] += r1 * g2 - r2 * g1;
    ph[1] += r2 * g0 - r0 * g2;
    ph[2] += r0 * g1 - r1 * g0;
  }
  ph[0] += T[10] * G[11] - T[11] * G[10];
  ph[1] += T[11] * G[9] - T[9] * G[11];
  ph[2] += T[9] * G[10] - T[10] * G[9];
  xi[0] = G[9];
  xi[1] = G[10];
  xi[2] = G[11];
  xi[3] = ph[0];
  xi[4] = ph[1];
  xi[5] = ph[2];
}

// One thread per rig transform (frames first, then cameras), each summing
// its views' contributions in view order.  The views' indices and gradients
// are staged through LDS, 256 views at a time, so the per-view loop reads
// no global memory but the other factor's pose.
constexpr int kRigStage = 256;

__global__ __launch_bounds__(256) void k_rig_grads(const float *__restrict__ central,
                                                   const float *__restrict__ relative,
                                                   const float *__restrict__ view_grads, RigIdx ri,
                                                   float *__restrict__ d_central, float *__restrict__ d_relative,
                                                   float *__restrict__ xi_central, float *__restrict__ xi_relative) {
  __shared__ float sg[kRigStage][12];
  __shared__ int sf[kRigStage], sc[kRigStage];
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = item < ri.n_frames + ri.n_cams;
  const bool is_central = item < ri.n_frames;
  const int id = is_central ? item : item - ri.n_frames;
  float G[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) G[k] = 0.0f;
  for (int v0 = 0; v0 < ri.n_views; v0 += kRigStage) {
    const int nv = ri.n_views - v0 < kRigStage ? ri.n_views - v0 : kRigStage;
    __syncthreads();
    for (int e = threadIdx.x; e < nv * 12; e += blockDim.x) sg[e / 12][e % 12] = view_grads[(size_t)v0 * 12 + e];
    for (int e = threadIdx.x; e < nv; e += blockDim.x) {
      sf[e] = ri.frame[v0 + e];
      sc[e] = ri.cam[v0 + e];
    }
    __syncthreads();
    if (!active) continue;
    for (int j = 0; j < nv; ++j) {
      if ((is_central ? sf[j] : sc[j]) != id) continue;
      const float *gv = sg[j];
      if (is_central) {
        // R_v = R_m R_r, t_v = R_m t_r + t_m:  dR_m = G_R R_r^T + g t_r^T, dt_m = g
        const float *r = relative + 12 * sc[j];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
#pragma unroll
          for (int c = 0; c < 3; ++c)
            G[3 * i + c] += ((gv[3 * i] * r[3 * c] + gv[3 * i + 1] * r[3 * c + 1]) + gv[3 * i + 2] * r[3 * c + 2]) +
                            gv[9 + i] * r[9 + c];
          G[9 + i] += gv[9 + i];
        }
      } else {
        // dR_r = R_m^T G_R, dt_r = R_m^T g
        const float *m = central + 12 * sf[j];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
#pragma unroll
          for (int c = 0; c < 3; ++c) G[3 * i + c] += (m[i] * gv[c] + m[3 + i] * gv[3 + c]) + m[6 + i] * gv[6 + c];
          G[9 + i] += (m[i] * gv[9] + m[3 + i] * gv[10]) + m[6 + i] * gv[11];
        }
      }
    }
  }
  if (!active) return;
  float *dst = is_central ? d_central + 12 * id : d_relative + 12 * id;
#pragma unroll
  for (int k = 0; k < 12; ++k) dst[k] = G[k];
  float *xo = is_central ? xi_central : xi_relative;
  if (xo) tangent(is_central ? central + 12 * id : relative + 12 * id, G, xo + 6 * id);
}

}  // namespace

uint32_t cam_chunks(uint32_t cap_rec) { return (cap_rec + kCamChunk - 1) / kCamChunk; }

void launch_cam_grads(const Ws &ws, const Sizes &sz, const float4 *cam_rec, float *cam_part, float *out,
                      int accumulate, hipStream_t st) {
  if (sz.n_views == 0) return;
  const uint32_t nb = cam_chunks(sz.cap_rec);
  if (nb > 0) k_cam_reduce<<<nb, 256, 0, st>>>(cam_rec, ws.rec_view, ws.scalars, sz.n_views, cam_part);
  k_cam_final<<<(unsigned)sz.n_views, 192, 0, st>>>(cam_part, ws.scalars, sz.n_views, out, accumulate);
}

void launch_rig_compose(const float *central, const float *relative, const RigIdx &ri, Cam *cams, hipStream_t st) {
  if (ri.n_views == 0) return;
  k_rig_compose<<<(unsigned)((ri.n_views + 63) / 64), 64, 0, st>>>(central, relative, ri, cams);
}

void launch_rig_grads(const float *central, const float *relative, const float *view_grads, const RigIdx &ri,
                      float *d_central, float *d_relative, float *xi_central, float *xi_relative, hipStream_t st) {
  const int items = ri.n_frames + ri.n_cams;
  if (items == 0) return;
  k_rig_grads<<<(unsigned)((items + 255) / 256), 256, 0, st>>>(central, relative, view_grads, ri, d_central,
                                                              d_relative, xi_central, xi_relative);
}

}  // namespace gsr

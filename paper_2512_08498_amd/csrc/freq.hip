// Frequency-based scheduling (Sec. 3.3, "Frequency-based Scheduling",
// Eqs. 9-12): the frequency significance X(I) = sum over bins of the
// channel 2-norm of the unnormalised 2D DFT, for a batch of planar RGB images
// of arbitrary sizes; the n x n box downsampling of the LOD levels; and the
// per-frame ratios, level updates and ratio-weighted frame draws.
//
// X takes two passes over HBM.  Row pass: one workgroup per image row packs
// the red and green rows into one complex FFT (z = R + iG; R and G are
// separated by the Hermitian symmetry of real inputs) and the blue row into a
// second, and writes the half spectrum j = 0..W/2 of each channel transposed
// (column-major per channel), so the column pass reads contiguous columns.
// Consecutive rows run on one XCD, so the transposed 8-byte writes of
// neighbouring rows meet in the same L2.  Column pass: one workgroup per
// half-spectrum column FFTs the three channels' columns, adds |F|^2 over the
// channels per bin, and sums the square roots; columns 1..ceil(W/2)-1 count
// twice (their mirror W - j has the same magnitudes).  A last pass sums each
// image's columns in order.
//
// The FFT is Stockham's self-sorting mixed-radix form (radices 2, 3, 4, 5,
// 7 and the composites 8, 9, 15, 16, 20, 25, 27, planned for the fewest
// stages), one stage per radix over all sequences of the workgroup at once
// (the two packed rows, or the three channels' columns), in one LDS buffer:
// every thread loads and transforms its butterflies in registers, then
// stores them after a barrier.  The twiddles exp(-2 pi i t / N) come from a
// table per transform length computed in double precision at plan time.
#include <cfloat>

#include "kernels.hpp"
#include "util.hpp"

namespace gsr {

namespace {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i
__device__ __forceinline__ float2 cmi(float2 a) { return make_float2(a.y, -a.x); }

// a / d for 0 <= a < 2^24, d >= 1, from a float reciprocal with one
// correction step each way (the float quotient is off by at most one).
__device__ __forceinline__ int fdiv(int a, int d, float inv) {
  int q = (int)((float)a * inv);
  q -= (q * d > a) ? 1 : 0;
  q += ((q + 1) * d <= a) ? 1 : 0;
  return q;
}

// exp(-2 pi i k / P) for k = 1 .. P - 1 (the forward sign).
template <int P>
struct Roots;
template <>
struct Roots<3> {
  static __device__ __forceinline__ float2 w(int k) {
    return k == 1 ? make_float2(-0.5f, -0.8660254037844386f) : make_float2(-0.5f, 0.8660254037844386f);
  }
};
template <>
struct Roots<5> {
  static __device__ __forceinline__ float2 w(int k) {
    switch (k) {
      case 1: return make_float2(0.30901699437494742f, -0.95105651629515357f);
      case 2: return make_float2(-0.80901699437494742f, -0.58778525229247313f);
      case 3: return make_float2(-0.80901699437494742f, 0.58778525229247313f);
      default: return make_float2(0.30901699437494742f, 0.95105651629515357f);
    }
  }
};
template <>
struct Roots<7> {
  static __device__ __forceinline__ float2 w(int k) {
    switch (k) {
      case 1: return make_float2(0.62348980185873353f, -0.78183148246802981f);
      case 2: return make_float2(-0.22252093395631440f, -0.97492791218182361f);
      case 3: return make_float2(-0.90096886790241913f, -0.43388373911755812f);
      case 4: return make_float2(-0.90096886790241913f, 0.43388373911755812f);
      case 5: return make_float2(-0.22252093395631440f, 0.97492791218182361f);
      default: return make_float2(0.62348980185873353f, 0.78183148246802981f);
    }
  }
};

// Composite radices P = A B, done in registers as B DFTs of size A, the
// twiddles exp(-2 pi i a b / P), then A DFTs of size B (Cooley-Tukey with
// n = B n1 + n2, k = k1 + A k2), so one Stockham stage covers two factors.
template <int P>
struct Split {
  static constexpr int A = 1, B = P;
};
template <> struct Split<8> { static constexpr int A = 4, B = 2; };
template <> struct Split<9> { static constexpr int A = 3, B = 3; };
template <> struct Split<15> { static constexpr int A = 3, B = 5; };
template <> struct Split<16> { static constexpr int A = 4, B = 4; };
template <> struct Split<20> { static constexpr int A = 4, B = 5; };
template <> struct Split<25> { static constexpr int A = 5, B = 5; };
template <> struct Split<27> { static constexpr int A = 3, B = 9; };

// cos and sin at compile time: Taylor series in double on |x| <= pi (30
// terms, far below float resolution).
constexpr double ct_sin(double x) {
  double t = x, s = x;
  for (int k = 1; k < 30; ++k) {
    t *= -x * x / (double)((2 * k) * (2 * k + 1));
    s += t;
  }
  return s;
}
constexpr double ct_cos(double x) {
  double t = 1.0, s = 1.0;
  for (int k = 1; k < 30; ++k) {
    t *= -x * x / (double)((2 * k - 1) * (2 * k));
    s += t;
  }
  return s;
}

// cos and sin of 2 pi m / P, m = 0 .. P - 1.
template <int P>
struct TwiddleTable {
  float c[P], s[P];
  constexpr TwiddleTable() : c(), s() {
    constexpr double kPi = 3.14159265358979323846;
    for (int m = 0; m < P; ++m) {
      double x = 2.0 * kPi * m / P;
      if (x > kPi) x -= 2.0 * kPi;
      c[m] = (float)ct_cos(x);
      s[m] = (float)ct_sin(x);
    }
  }
};

template <int P>
__device__ __forceinline__ void dft(float2 *v);

template <int P>
__device__ __forceinline__ void dft_composite(float2 *v) {
  constexpr int A = Split<P>::A, B = Split<P>::B;
  constexpr TwiddleTable<P> tw{};
  float2 t[P];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    float2 u[A];
#pragma unroll
    for (int a = 0; a < A; ++a) u[a] = v[b + B * a];
    dft<A>(u);
#pragma unroll
    for (int a = 0; a < A; ++a) {
      const int m = (a * b) % P;  // u exp(-2 pi i m / P) = u (c - i s)
      t[a * B + b] = m == 0 ? u[a]
                            : make_float2(u[a].x * tw.c[m] + u[a].y * tw.s[m], u[a].y * tw.c[m] - u[a].x * tw.s[m]);
    }
  }
#pragma unroll
  for (int a = 0; a < A; ++a) dft<B>(t + a * B);
#pragma unroll
  for (int a = 0; a < A; ++a)
#pragma unroll
    for (int b = 0; b < B; ++b) v[a + A * b] = t[a * B + b];
}

// In-register radix-P DFT with the forward sign.  Radices 3 and 5 use the
// symmetric forms: with s_k = x_k + x_{P-k} and d_k = x_k - x_{P-k},
// X_q = x_0 + sum_k cos(2 pi k q / P) s_k - i sum_k sin(2 pi k q / P) d_k.
template <int P>
__device__ __forceinline__ void dft(float2 *v) {
  if constexpr (Split<P>::A > 1) {
    dft_composite<P>(v);
  } else if constexpr (P == 3) {
    constexpr float s1 = 0.86602540378443865f;  // sin(2 pi / 3)
    const float2 s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
    const float2 a = make_float2(v[0].x - 0.5f * s.x, v[0].y - 0.5f * s.y);
    const float2 b = make_float2(s1 * d.y, -s1 * d.x);  // -i sin(2 pi / 3) d
    v[0] = cadd(v[0], s);
    v[1] = cadd(a, b);
    v[2] = csub(a, b);
  } else if constexpr (P == 5) {
    constexpr float c1 = 0.30901699437494742f, c2 = -0.80901699437494742f;  // cos(2 pi / 5), cos(4 pi / 5)
    constexpr float s1 = 0.95105651629515357f, s2 = 0.58778525229247313f;   // sin(2 pi / 5), sin(4 pi / 5)
    const float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    const float2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    const float2 a1 = make_float2(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
    const float2 a2 = make_float2(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
    const float2 b1 = make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y);
    const float2 b2 = make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y);
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd(a1, cmi(b1));
    v[4] = csub(a1, cmi(b1));
    v[2] = cadd(a2, cmi(b2));
    v[3] = csub(a2, cmi(b2));
  } else if constexpr (P == 2) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (P == 4) {
    const float2 a = v[0], b = v[1], c = v[2], d = v[3];
    const float2 s0 = cadd(a, c), s1 = csub(a, c), s2 = cadd(b, d), s3 = cmi(csub(b, d));
    v[0] = cadd(s0, s2);
    v[1] = cadd(s1, s3);
    v[2] = csub(s0, s2);
    v[3] = csub(s1, s3);
  } else {
    float2 o[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
      float2 acc = v[0];
#pragma unroll
      for (int r = 1; r < P; ++r) {
        const int e = (q * r) % P;
        acc = cadd(acc, e == 0 ? v[r] : cmul(v[r], Roots<P>::w(e)));
      }
      o[q] = acc;
    }
#pragma unroll
    for (int q = 0; q < P; ++q) v[q] = o[q];
  }
}

constexpr int kRowThreads = 256;                // row pass: two sequences of length W
constexpr int kColThreads = 256;                // column pass: three sequences of length H
constexpr int kRowMaxElems = 2 * 2560;
constexpr int kColMaxElems = 3 * 2560;

// One radix-P Stockham stage over `cnt` sequences of length N stored one
// after the other in buf.  Butterfly b (sequence b / m, index j = b mod m,
// m = N / P) reads elements j + r m, multiplies by the twiddles
// exp(-2 pi i k r / (Ns P)) (k = j mod Ns; table entry k r N / (Ns P)),
// transforms, and writes (j / Ns) Ns P + k + q Ns.  All butterflies of the
// thread are loaded and transformed before the barrier, then stored, so one
// LDS buffer suffices.  Not inlined: each radix then gets its own register
// allocation (71 to 113 VGPRs), where inlining all five into the stage loop
// made the kernels allocate for their union (241 VGPRs, two waves per SIMD
// instead of three).
template <int P, int T, int MAXE>
__device__ __attribute__((noinline)) void fft_stage(float2 *buf, int N, int cnt, int Ns, const float2 *tw) {
  constexpr int kMaxB = (MAXE / P + T - 1) / T;
  const int m = N / P;
  const int total = cnt * m;
  const int tstep = N / (Ns * P);
  const float inv_ns = 1.0f / (float)Ns;
  const bool first = Ns == 1;  // k = 0: no twiddles, no division
  float2 v[kMaxB][P];
  int dst[kMaxB];
#pragma unroll
  for (int i = 0; i < kMaxB; ++i) {
    const int b = threadIdx.x + i * T;
    if (b < total) {
      const int seq = (b >= m ? 1 : 0) + (b >= 2 * m ? 1 : 0);  // cnt <= 3
      const int j = b - seq * m;
      const int jq = first ? j : fdiv(j, Ns, inv_ns);
      const int k = j - jq * Ns;
      const float2 *src = buf + seq * N + j;
#pragma unroll
      for (int r = 0; r < P; ++r) v[i][r] = src[r * m];
      if (!first) {
#pragma unroll
        for (int r = 1; r < P; ++r) v[i][r] = cmul(v[i][r], tw[k * r * tstep]);
      }
      dft<P>(v[i]);
      dst[i] = seq * N + jq * Ns * P + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kMaxB; ++i) {
    const int b = threadIdx.x + i * T;
    if (b < total) {
#pragma unroll
      for (int q = 0; q < P; ++q) buf[dst[i] + q * Ns] = v[i][q];
    }
  }
  __syncthreads();
}

// Forward DFTs, in place, of cnt sequences of length N in LDS (cnt * N <=
// MAXE) by a workgroup of T threads; tw is the length-N table
// exp(-2 pi i t / N), also in LDS.  Every thread must call it.
template <int T, int MAXE>
__device__ __forceinline__ void fft_lds(float2 *buf, int N, int cnt, const float2 *tw, const uint8_t *__restrict__ fac,
                                        int nfac) {
  int Ns = 1;
  for (int s = 0; s < nfac; ++s) {
    switch (fac[s]) {
      case 27: fft_stage<27, T, MAXE>(buf, N, cnt, Ns, tw); break;
      case 25: fft_stage<25, T, MAXE>(buf, N, cnt, Ns, tw); break;
      case 20: fft_stage<20, T, MAXE>(buf, N, cnt, Ns, tw); break;
      case 16: fft_stage<16, T, MAXE>(buf, N, cnt, Ns, tw); break;
      case 15: fft_stage<15, T, MAXE>(buf, N, cnt, Ns, tw); break;
      case 9: fft_stage<9, T, MAXE>(buf, N, cnt, Ns, tw); break;
      case 8: fft_stage<8, T, MAXE>(buf, N, cnt, Ns, tw); break;
      case 4: fft_stage<4, T, MAXE>(buf, N, cnt, Ns, tw); break;
      case 2: fft_stage<2, T, MAXE>(buf, N, cnt, Ns, tw); break;
      case 3: fft_stage<3, T, MAXE>(buf, N, cnt, Ns, tw); break;
      case 5: fft_stage<5, T, MAXE>(buf, N, cnt, Ns, tw); break;
      default: fft_stage<7, T, MAXE>(buf, N, cnt, Ns, tw); break;
    }
    Ns *= fac[s];
  }
}

__device__ __forceinline__ int find_image(const FreqImg *imgs, int n, int64_t idx, bool rows) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((rows ? imgs[mid].row_base : imgs[mid].col_base) <= idx) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Deterministic sum over a workgroup of NW waves: butterfly per wave, then
// the waves in order; the result is valid in every thread.
template <int NW>
__device__ __forceinline__ float block_sum(float x, float *red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  float t = red[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) t += red[w];
  return t;
}

__global__ __launch_bounds__(kRowThreads) void k_fft_rows(const float *__restrict__ images, const FreqImg *__restrict__ imgs,
                                                  int n_imgs, int64_t n_rows, const float2 *__restrict__ tw_all,
                                                  float2 *__restrict__ inter) {
  extern __shared__ float2 lds[];
  const int64_t row = xcd_tile(blockIdx.x, gridDim.x);
  if (row >= n_rows) return;
  const FreqImg *ip = imgs + find_image(imgs, n_imgs, row, true);
  const FreqImg im = *ip;
  const int i = (int)(row - im.row_base), W = im.w, H = im.h, half = W / 2 + 1;
  const float *R = images + im.pix_off + (int64_t)i * W;
  const float *G = R + (int64_t)W * H, *B = G + (int64_t)W * H;
  // sequence 0: R + iG, sequence 1: B; then the twiddle table
  float2 *tw = lds + 2 * W;
  const float2 *twg = tw_all + im.tw_w;
  for (int x = threadIdx.x; x < W; x += blockDim.x) {
    lds[x] = make_float2(R[x], G[x]);
    lds[W + x] = make_float2(B[x], 0.0f);
    tw[x] = twg[x];
  }
  __syncthreads();
  fft_lds<kRowThreads, kRowMaxElems>(lds, W, 2, tw, ip->fac_w, im.nfac_w);
  float2 *out = inter + im.inter_off;
  for (int j = threadIdx.x; j < half; j += blockDim.x) {
    const float2 p = lds[j], q = lds[j == 0 ? 0 : W - j];
    // F_R = (Z(j) + conj Z(-j)) / 2,  F_G = (Z(j) - conj Z(-j)) / 2i
    out[((int64_t)0 * half + j) * H + i] = make_float2(0.5f * (p.x + q.x), 0.5f * (p.y - q.y));
    out[((int64_t)1 * half + j) * H + i] = make_float2(0.5f * (p.y + q.y), -0.5f * (p.x - q.x));
    out[((int64_t)2 * half + j) * H + i] = lds[W + j];
  }
}

constexpr int kMaxBinsPerThread = (2560 + kColThreads - 1) / kColThreads;  // H <= 2560

__global__ __launch_bounds__(kColThreads) void k_fft_cols(const FreqImg *__restrict__ imgs, int n_imgs, int64_t n_cols,
                                                  const float2 *__restrict__ tw_all,
                                                  const float2 *__restrict__ inter, float *__restrict__ col_sum) {
  extern __shared__ float2 lds[];
  __shared__ float red[kColThreads / 64];
  const int64_t col = blockIdx.x;
  if (col >= n_cols) return;
  const FreqImg *ip = imgs + find_image(imgs, n_imgs, col, false);
  const FreqImg im = *ip;
  const int j = (int)(col - im.col_base), W = im.w, H = im.h, half = W / 2 + 1;
  float2 *tw = lds + 3 * H;
  const float2 *twg = tw_all + im.tw_h;
  for (int k = threadIdx.x; k < H; k += blockDim.x) tw[k] = twg[k];
  for (int c = 0; c < 3; ++c) {
    const float2 *src = inter + im.inter_off + ((int64_t)c * half + j) * H;
    for (int k = threadIdx.x; k < H; k += blockDim.x) lds[c * H + k] = src[k];
  }
  __syncthreads();
  fft_lds<kColThreads, kColMaxElems>(lds, H, 3, tw, ip->fac_h, im.nfac_h);
  float s = 0.0f;
#pragma unroll
  for (int t = 0; t < kMaxBinsPerThread; ++t) {
    const int k = threadIdx.x + t * kColThreads;
    if (k < H) {
      const float2 a = lds[k], b = lds[H + k], c = lds[2 * H + k];
      s += sqrtf((a.x * a.x + a.y * a.y) + (b.x * b.x + b.y * b.y) + (c.x * c.x + c.y * c.y));
    }
  }
  const float total = block_sum<kColThreads / 64>(s, red);
  if (threadIdx.x == 0) {
    const bool single = j == 0 || (W % 2 == 0 && j == W / 2);
    col_sum[col] = single ? total : 2.0f * total;
  }
}

// X of each image: its columns' sums in column order (thread t takes the
// columns t mod 256 in order, then the fixed block sum).
__global__ __launch_bounds__(256) void k_freq_final(const FreqImg *__restrict__ imgs,
                                                    const float *__restrict__ col_sum, float *__restrict__ X) {
  __shared__ float red[4];
  const FreqImg im = imgs[blockIdx.x];
  const int half = im.w / 2 + 1;
  float s = 0.0f;
  for (int j = threadIdx.x; j < half; j += blockDim.x) s += col_sum[im.col_base + j];
  const float total = block_sum<4>(s, red);
  if (threadIdx.x == 0) X[blockIdx.x] = total;
}

// Box average over n x n blocks; one thread per output value, the block's
// values added row by row.
__global__ __launch_bounds__(256) void k_downsample(const float *__restrict__ src, int W, int H, int n,
                                                    float *__restrict__ dst) {
  const int w = W / n, h = H / n;
  const int64_t total = 3ll * w * h;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int x = (int)(idx % w);
  const int y = (int)((idx / w) % h);
  const int c = (int)(idx / ((int64_t)w * h));
  const float *p = src + ((int64_t)c * H + (int64_t)y * n) * W + (int64_t)x * n;
  float s = 0.0f;
  for (int dy = 0; dy < n; ++dy)
    for (int dx = 0; dx < n; ++dx) s += p[(int64_t)dy * W + dx];
  dst[idx] = s / (float)(n * n);
}

// Ratios, level updates and frame draws of one scheduling step (single
// workgroup; the prefix sums of the weights are taken by one thread in frame
// order, in float32, so the draws are reproducible bit for bit).
__global__ __launch_bounds__(256) void k_freq_schedule(const float *__restrict__ x_gt,
                                                       const float *__restrict__ x_gt_level,
                                                       const float *__restrict__ x_render, int F, float tau_f,
                                                       int32_t *__restrict__ levels, const float *__restrict__ u,
                                                       int n_picks, float *__restrict__ r_out,
                                                       float *__restrict__ rp_out, int32_t *__restrict__ picks) {
  extern __shared__ float cdf[];
  const float cap = FLT_MAX / (float)(2 * F);  // F capped weights cannot overflow
  for (int f = threadIdx.x; f < F; f += blockDim.x) {
    const float r = x_gt[f] / x_render[f];
    const float rp = x_gt_level ? x_gt_level[f] / x_render[f] : __builtin_nanf("");
    if (r_out) r_out[f] = r;
    if (rp_out) rp_out[f] = rp;
    if (levels && rp < tau_f && levels[f] > 0) levels[f] -= 1;
    cdf[f] = isnan(r) ? 0.0f : fmaxf(fminf(r, cap), 0.0f);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float acc = 0.0f;
    for (int f = 0; f < F; ++f) {
      acc = acc + cdf[f];
      cdf[f] = acc;
    }
  }
  __syncthreads();
  if (!picks) return;
  const float total = cdf[F - 1];
  for (int b = threadIdx.x; b < n_picks; b += blockDim.x) {
    const float ub = u[b];
    int f;
    if (!(total > 0.0f)) {
      f = (int)(ub * (float)F);
      f = f < F - 1 ? f : F - 1;
      f = f > 0 ? f : 0;
    } else {
      const float target = ub * total;
      int lo = 0, hi = F - 1;  // first f with cdf[f] > target, else F - 1
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cdf[mid] > target) hi = mid;
        else lo = mid + 1;
      }
      f = lo;
    }
    picks[b] = f;
  }
}

}  // namespace

void launch_freq_significance(const float *images, const FreqImg *imgs, int n_imgs, int64_t n_rows, int64_t n_cols,
                              int max_w, int max_h, const float2 *tw, float2 *inter, float *col_sum, float *X,
                              hipStream_t st) {
  if (n_imgs == 0) return;
  const uint32_t grid = tile_grid((uint32_t)n_rows);
  k_fft_rows<<<grid, kRowThreads, (size_t)3 * max_w * sizeof(float2), st>>>(images, imgs, n_imgs, n_rows, tw, inter);
  k_fft_cols<<<(unsigned)n_cols, kColThreads, (size_t)4 * max_h * sizeof(float2), st>>>(imgs, n_imgs, n_cols, tw,
                                                                                        inter, col_sum);
  k_freq_final<<<(unsigned)n_imgs, 256, 0, st>>>(imgs, col_sum, X);
}

void launch_downsample(const float *src, int W, int H, int n, float *dst, hipStream_t st) {
  const int64_t total = 3ll * (W / n) * (H / n);
  if (total == 0) return;
  k_downsample<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(src, W, H, n, dst);
}

void launch_freq_schedule(const float *x_gt, const float *x_gt_level, const float *x_render, int F, float tau_f,
                          int32_t *levels, const float *u, int n_picks, float *r, float *rp, int32_t *picks,
                          hipStream_t st) {
  if (F == 0) return;
  k_freq_schedule<<<1, 256, (size_t)F * sizeof(float), st>>>(x_gt, x_gt_level, x_render, F, tau_f, levels, u,
                                                             n_picks, r, rp, picks);
}

}  // namespace gsr

// Learned screener: per-camera features and a 4-layer BF16 MLP with its
// training step (forward, loss, backward, Adam), all on the GPU.
//
// Features (55 per camera) come from the scene stage's intermediate data:
//   * the diagonal block Z_ii of the reduced camera matrix (Sec. 5.2): log10
//     of its diagonal and its 36 correlations, row-major upper triangle;
//   * log(1 + count) of the camera's observations in 8 track-length bins
//     (2, 3, 4, 5, 6-7, 8-10, 11-15, >= 16);
//   * the mean over its observations of the largest angle between its ray to
//     the point and another track camera's ray;
//   * log(1 + number of cameras sharing a point with it).
//
// MLP: 55 -> 256 -> 256 -> 256 -> 45, ReLU, linear output.  Parameters are
// one FP32 master vector (per layer W out x in row-major, then b); every
// product rounds its operands to BF16 and accumulates in FP32 on
// v_mfma_f32_16x16x16_bf16.  Hidden activations are stored in BF16.
#include <algorithm>

#include "ucov_internal.h"
#include "../../include/ucov.h"

namespace ucov {

namespace {

constexpr int kIn = 55, kHid = 256, kOut = 45;

// ---------------------------------------------------------------------------
// features
// ---------------------------------------------------------------------------

__device__ inline int track_bin(int len) {
  return len >= 16 ? 7 : len >= 11 ? 6 : len >= 8 ? 5 : len >= 6 ? 4 : (len >= 2 ? len - 2 : 0);
}

// One thread per observation slot: its track-length bin, its largest
// triangulation angle, accumulated per camera.
__global__ void k_feat_obs(SceneDev sc, const int64_t *ptr_p, const int32_t *slot_cam,
                           const int32_t *slot_pt, int32_t *hist, double *ang) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= ptr_p[sc.m]) return;
  const int j = slot_pt[a], c = slot_cam[a];
  const int64_t p0 = ptr_p[j], p1 = ptr_p[j + 1];
  const double X0 = sc.pts[3 * (int64_t)j], X1 = sc.pts[3 * (int64_t)j + 1],
               X2 = sc.pts[3 * (int64_t)j + 2];
  const double *Cc = sc.cams + 9 * (int64_t)c + 3;
  double r0 = X0 - Cc[0], r1 = X1 - Cc[1], r2 = X2 - Cc[2];
  const double inv = 1.0 / sqrt(r0 * r0 + r1 * r1 + r2 * r2);
  r0 *= inv;
  r1 *= inv;
  r2 *= inv;
  double best = 0.0;
  for (int64_t b = p0; b < p1; ++b) {
    if (b == a) continue;
    const double *Ck = sc.cams + 9 * (int64_t)slot_cam[b] + 3;
    const double s0 = X0 - Ck[0], s1 = X1 - Ck[1], s2 = X2 - Ck[2];
    const double d = (r0 * s0 + r1 * s1 + r2 * s2) / sqrt(s0 * s0 + s1 * s1 + s2 * s2);
    best = fmax(best, acos(fmin(1.0, fmax(-1.0, d))));
  }
  atomicAdd(&hist[8 * (int64_t)c + track_bin((int)(p1 - p0))], 1);
  atomicAdd(&ang[c], best);
}

// Cameras sharing a point: one thread per non-empty camera-pair bin.
__global__ void k_feat_covis(const int2 *nzlist, const int64_t *nzcount, int32_t *covis) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nzcount[0]) return;
  const int2 ik = nzlist[e];
  if (ik.x == ik.y) return;
  atomicAdd(&covis[ik.x], 1);
  atomicAdd(&covis[ik.y], 1);
}

__global__ void k_feat_finish(int n, const double *zdiag, const int32_t *hist, const double *ang,
                              const int32_t *covis, float *feat) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double *z = zdiag + 81 * (int64_t)i;
  float *f = feat + (int64_t)kIn * i;
  int k = 0;
  for (int a = 0; a < 9; ++a)
    for (int b = a; b < 9; ++b)
      f[k++] = (float)(a == b ? log10(z[10 * a]) : z[9 * a + b] / sqrt(z[10 * a] * z[10 * b]));
  int cnt = 0;
  for (int b = 0; b < 8; ++b) {
    const int h = hist[8 * (int64_t)i + b];
    cnt += h;
    f[45 + b] = (float)log1p((double)h);
  }
  f[53] = (float)(cnt > 0 ? ang[i] / cnt : 0.0);
  f[54] = (float)log1p((double)covis[i]);
}

// ---------------------------------------------------------------------------
// BF16 MFMA GEMM
//
// C[M x N] = op(A) op(B) with op(A)[m][k] = A[m*lda + k] (TA = false) or
// A[k*lda + m] (TA = true) and op(B)[k][n] = B[n*ldb + k] (TB = true) or
// B[k*ldb + n] (TB = false).  A and B are float or bf16 (ushort) in memory
// and are rounded to BF16 on their way into LDS.  64 x 64 tile per workgroup
// of 4 waves, each wave a 32 x 32 quarter as 2 x 2 MFMA 16 x 16 tiles; K in
// steps of 32.
// ---------------------------------------------------------------------------

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ inline unsigned short to_bf16(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (unsigned short)(u >> 16);
}
__device__ inline float from_bf16(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

template <class T>
__device__ inline float load_f(const T *p, int64_t i);
template <>
__device__ inline float load_f<float>(const float *p, int64_t i) { return p[i]; }
template <>
__device__ inline float load_f<unsigned short>(const unsigned short *p, int64_t i) {
  return from_bf16(p[i]);
}

enum Epi { kStoreF32 = 0, kBiasReluBf16 = 1, kBiasF32 = 2, kReluMaskBf16 = 3 };

struct MlpGemm {
  int M, N, K;
  const void *A;
  int64_t lda;
  const void *B;
  int64_t ldb;
  void *C;
  int64_t ldc;
  const float *bias;            // per column n (kBiasReluBf16, kBiasF32)
  const unsigned short *mask;   // kReluMaskBf16: C = acc * [mask > 0], mask ld = ldc
};

constexpr int kTM = 64, kTK = 32, kLdsK = kTK + 8;

template <class TAe, class TBe, bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_mlp_gemm(MlpGemm g) {
  __shared__ unsigned short As[kTM * kLdsK];  // [m][k]
  __shared__ unsigned short Bs[kTM * kLdsK];  // [n][k]
  const int m0 = blockIdx.x * kTM, n0 = blockIdx.y * kTM;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = (wid >> 1) * 32, wn = (wid & 1) * 32;
  const TAe *A = static_cast<const TAe *>(g.A);
  const TBe *B = static_cast<const TBe *>(g.B);
  floatx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < g.K; k0 += kTK) {
    // 64 x 32 elements of each operand, 8 per thread
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = tid * 8 + e;
      int r, k;
      if (!TA) {  // contiguous along k
        r = idx / kTK;
        k = idx % kTK;
      } else {    // contiguous along m
        k = idx / kTM;
        r = idx % kTM;
      }
      const int gm = m0 + r, gk = k0 + k;
      float v = 0.f;
      if (gm < g.M && gk < g.K)
        v = load_f<TAe>(A, TA ? (int64_t)gk * g.lda + gm : (int64_t)gm * g.lda + gk);
      As[r * kLdsK + k] = to_bf16(v);
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = tid * 8 + e;
      int c, k;
      if (TB) {   // contiguous along k
        c = idx / kTK;
        k = idx % kTK;
      } else {    // contiguous along n
        k = idx / kTM;
        c = idx % kTM;
      }
      const int gn = n0 + c, gk = k0 + k;
      float v = 0.f;
      if (gn < g.N && gk < g.K)
        v = load_f<TBe>(B, TB ? (int64_t)gn * g.ldb + gk : (int64_t)gk * g.ldb + gn);
      Bs[c * kLdsK + k] = to_bf16(v);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kTK; ks += 16) {
      const int kk = ks + 4 * (lane >> 4);
      bf16x4 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const unsigned short *pa = As + (wm + 16 * i + (lane & 15)) * kLdsK + kk;
        const unsigned short *pb = Bs + (wn + 16 * i + (lane & 15)) * kLdsK + kk;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          a[i][q] = (short)pa[q];
          b[i][q] = (short)pb[q];
        }
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // D[4 (lane / 16) + v][lane % 16] of each 16 x 16 tile
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = m0 + wm + 16 * i + 4 * (lane >> 4) + v;
        const int gn = n0 + wn + 16 * j + (lane & 15);
        if (gm >= g.M || gn >= g.N) continue;
        float x = acc[i][j][v];
        const int64_t o = (int64_t)gm * g.ldc + gn;
        if (EPI == kStoreF32) {
          static_cast<float *>(g.C)[o] = x;
        } else if (EPI == kBiasF32) {
          static_cast<float *>(g.C)[o] = x + g.bias[gn];
        } else if (EPI == kBiasReluBf16) {
          static_cast<unsigned short *>(g.C)[o] = to_bf16(fmaxf(x + g.bias[gn], 0.f));
        } else {
          const bool on = from_bf16(g.mask[o]) > 0.f;
          static_cast<unsigned short *>(g.C)[o] = to_bf16(on ? x : 0.f);
        }
      }
}

template <class TAe, class TBe, bool TA, bool TB, int EPI>
void gemm_launch(const MlpGemm &g, hipStream_t st) {
  const dim3 grid((g.M + kTM - 1) / kTM, (g.N + kTM - 1) / kTM);
  hipLaunchKernelGGL((k_mlp_gemm<TAe, TBe, TA, TB, EPI>), grid, dim3(256), 0, st, g);
}

// ---------------------------------------------------------------------------
// loss, bias gradient, Adam, label transforms
// ---------------------------------------------------------------------------

// dY = 2 (Y - T) / (B * 45); loss += sum (Y - T)^2 / (B * 45)
__global__ __launch_bounds__(256) void k_mse(int64_t count, const float *y, const float *t,
                                             float *dy, double *loss) {
  __shared__ double red[4];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (i < count) {
    const float d = y[i] - t[i];
    dy[i] = 2.f * d / (float)count;
    s = (double)d * d;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, (red[0] + red[1] + red[2] + red[3]) / (double)count);
}

// db[n] = sum_b D[b][n], D float or bf16, one thread per column, rows strided
template <class T>
__global__ void k_colsum(int rows, int cols, const T *d, float *db) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += load_f<T>(d, (int64_t)r * cols + c);
  db[c] = s;
}

__global__ void k_adam(int64_t n, float *p, const float *g, float *m, float *v, float lr,
                       float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

__global__ void k_loss_out(const double *acc, float *out) { *out = (float)*acc; }

// xs = (x - mean) / std per feature (identity when mean is null)
__global__ void k_standardize(int64_t count, const float *x, const float *mean, const float *stdv,
                              float *xs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int f = (int)(i % kIn);
  xs[i] = mean ? (x[i] - mean[f]) / stdv[f] : x[i];
}

// Per camera: b_a, the standard deviations of the block-diagonal estimate
// (Z_ii)^-1, from the camera's 45 Z_ii features (log10 of the diagonal, then
// the correlations, row-major upper triangle).  With C the correlation
// matrix, ((Z_ii)^-1)_aa = (C^-1)_aa / Z_aa; C is taken with kScaleRidge
// added to its diagonal, which keeps it positive definite although its
// entries are rounded to FP32 (at most ~6e-8 each, below 1e-6 in norm) and
// bounds b for a nearly singular block.  ((C + ridge I)^-1)_aa is the squared
// norm of column a of R^-1 for the Cholesky factor R R^T.
constexpr double kScaleRidge = 1e-6;

__global__ void k_block_scale(int64_t n, const float *feat, double *b, DevStatus *ds) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float *f = feat + (int64_t)kIn * i;
  double C[9][9], R[9][9];
  int k = 0;
  for (int a = 0; a < 9; ++a)
    for (int c = a; c < 9; ++c, ++k) C[a][c] = a == c ? 1.0 + kScaleRidge : (double)f[k];
  bool ok = true;
  for (int a = 0; a < 9; ++a)
    for (int c = 0; c <= a; ++c) {
      double s = C[c][a];
      for (int q = 0; q < c; ++q) s -= R[a][q] * R[c][q];
      if (a == c) {
        if (!(s > 0.0)) {
          ok = false;
          s = 1.0;
        }
        R[a][a] = sqrt(s);
      } else {
        R[a][c] = s / R[c][c];
      }
    }
  if (!ok) report_error(ds, UCOV_EINVAL, (int)i);
  // R^-1 (lower), overwriting C's lower triangle
  for (int c = 0; c < 9; ++c) {
    C[c][c] = 1.0 / R[c][c];
    for (int a = c + 1; a < 9; ++a) {
      double s = 0.0;
      for (int q = c; q < a; ++q) s += R[a][q] * C[q][c];
      C[a][c] = -s / R[a][a];
    }
  }
  k = 0;
  for (int a = 0; a < 9; ++a) {
    double q = 0.0;
    for (int r = a; r < 9; ++r) q += C[r][a] * C[r][a];
    b[9 * i + a] = sqrt(q) * pow(10.0, -0.5 * (double)f[k]);
    k += 9 - a;
  }
}

// Covariances -> standardised log-Cholesky parameters of D^-1 S D^-1 with the
// per-camera D_a = s_a b_a, standardised and (clip) clipped to +-kLabelClip:
// a camera that the other cameras barely constrain has a normalised
// covariance many orders of magnitude above the rest, whose raw parameters
// would dominate the loss.
constexpr double kLabelClip = 6.0;

__global__ void k_labels(int64_t n, const double *cov, const double *b, const double *s_glob,
                         const float *mean, const float *stdv, bool clip, float *lab,
                         DevStatus *ds) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double L[9][9], D[9];
  for (int a = 0; a < 9; ++a) D[a] = s_glob[a] * b[9 * i + a];
  const double *S = cov + 81 * i;
  for (int a = 0; a < 9; ++a)
    for (int c = 0; c <= a; ++c) {
      double s = S[9 * a + c] / (D[a] * D[c]);
      for (int k = 0; k < c; ++k) s -= L[a][k] * L[c][k];
      if (a == c) {
        if (!(s > 0.0)) {
          report_error(ds, UCOV_EINVAL, (int)i);
          s = 1.0;
        }
        L[a][a] = sqrt(s);
      } else {
        L[a][c] = s / L[c][c];
      }
    }
  int k = 0;
  for (int a = 0; a < 9; ++a)
    for (int c = 0; c <= a; ++c, ++k) {
      const double v = a == c ? log(L[a][a]) : L[a][c];
      const double z = (v - mean[k]) / stdv[k];
      lab[45 * i + k] = (float)(clip ? fmin(fmax(z, -kLabelClip), kLabelClip) : z);
    }
}

// Network outputs -> covariances D L L^T D (D_a = s_a b_a per camera) and
// their spread trace(L L^T)
__global__ void k_predicted_cov(int64_t n, const float *y, const double *b, const double *s_glob,
                                const float *mean, const float *stdv, double *cov,
                                double *spread) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double L[9][9], D[9];
  for (int a = 0; a < 9; ++a) D[a] = s_glob[a] * b[9 * i + a];
  int k = 0;
  for (int a = 0; a < 9; ++a)
    for (int c = 0; c < 9; ++c) L[a][c] = 0.0;
  for (int a = 0; a < 9; ++a)
    for (int c = 0; c <= a; ++c, ++k) {
      const double v = (double)mean[k] + (double)stdv[k] * (double)y[45 * i + k];
      L[a][c] = a == c ? exp(v) : v;
    }
  double tr = 0.0;
  for (int a = 0; a < 9; ++a)
    for (int c = 0; c < 9; ++c) {
      double s = 0.0;
      for (int q = 0; q <= (a < c ? a : c); ++q) s += L[a][q] * L[c][q];
      if (a == c) tr += s;
      if (cov) cov[81 * i + 9 * a + c] = D[a] * s * D[c];
    }
  if (spread) spread[i] = tr;
}

// ---------------------------------------------------------------------------
// standardisation statistics of a training set
// ---------------------------------------------------------------------------
constexpr int kStatThreads = 256;

// Fixed-order sum over the workgroup: each thread its strided share, then a
// tree in LDS (the same bits on every call).
__device__ inline double block_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = kStatThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// One workgroup per column c of x (n x cols, row-major FP32): mean and the
// standard deviation with n - 1 in the denominator, at least 1e-6.
__global__ __launch_bounds__(kStatThreads) void k_col_stats(int64_t n, int cols, const float *x,
                                                          float *mean, float *stdv) {
  __shared__ double red[kStatThreads];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kStatThreads) s += (double)x[i * cols + c];
  const double mu = block_sum(s, red) / (double)n;
  double q = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kStatThreads) {
    const double d = (double)x[i * cols + c] - mu;
    q += d * d;
  }
  const double var = block_sum(q, red) / (double)(n - 1);
  if (threadIdx.x == 0) {
    mean[c] = (float)mu;
    stdv[c] = fmaxf((float)sqrt(var), 1e-6f);
  }
}

// Order-preserving unsigned key of a double.
__device__ inline uint64_t order_key(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// The value of rank `rank` (0-based, ascending) among n keys, found digit by
// digit (8 bits at a time, from the top) with LDS histograms: the counts, and
// so the result, do not depend on the order of the atomic increments.
template <typename KeyFn>
__device__ uint64_t select_key(int64_t n, int64_t rank, KeyFn key, int32_t *hist, uint64_t *sh) {
  uint64_t prefix = 0;
  for (int shift = 56; shift >= 0; shift -= 8) {
    const uint64_t hi_mask = shift == 56 ? 0 : ~((1ull << (shift + 8)) - 1);
    for (int d = threadIdx.x; d < 256; d += blockDim.x) hist[d] = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
      const uint64_t k = key(i);
      if ((k & hi_mask) == prefix) atomicAdd(&hist[(k >> shift) & 255u], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int d = 0;
      while (d < 255 && rank >= hist[d]) rank -= hist[d++];
      sh[0] = prefix | ((uint64_t)d << shift);
      sh[1] = (uint64_t)rank;
    }
    __syncthreads();
    prefix = sh[0];
    rank = (int64_t)sh[1];
    __syncthreads();
  }
  return prefix;
}

__device__ inline double key_value(uint64_t k) {
  const uint64_t b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double((long long)b);
}

// One workgroup per column c of x (n x cols, row-major FP32): the lower
// median m (rank (n - 1) / 2) and 1.4826 times the lower median of |x - m|
// (the median absolute deviation, scaled to a normal distribution's
// standard deviation), at least 1e-6.
__global__ __launch_bounds__(kStatThreads) void k_col_robust(int64_t n, int cols, const float *x,
                                                           float *center, float *spread) {
  __shared__ int32_t hist[256];
  __shared__ uint64_t sh[2];
  const int c = blockIdx.x;
  const int64_t rank = (n - 1) / 2;
  const double m = key_value(select_key(
      n, rank, [&](int64_t i) { return order_key((double)x[i * cols + c]); }, hist, sh));
  const double mad = key_value(select_key(
      n, rank, [&](int64_t i) { return order_key(fabs((double)x[i * cols + c] - m)); }, hist,
      sh));
  if (threadIdx.x == 0) {
    center[c] = (float)m;
    spread[c] = fmaxf((float)(1.4826 * mad), 1e-6f);
  }
}

// One workgroup per diagonal entry a: s[a] = sqrt of the lower median (the
// value of rank (n - 1) / 2 in ascending order) over the n blocks of the
// variance ratio cov[81 i + 10 a] / b[9 i + a]^2, found bit by bit on the
// order-preserving keys.
__global__ __launch_bounds__(kStatThreads) void k_diag_median(int64_t n, const double *cov,
                                                            const double *b, double *s_glob) {
  __shared__ double red[kStatThreads];
  const int a = blockIdx.x;
  uint64_t prefix = 0;
  int64_t rank = (n - 1) / 2;  // rank among the values that share the prefix
  for (int bit = 63; bit >= 0; --bit) {
    const uint64_t hi_mask = bit == 63 ? 0 : ~((1ull << (bit + 1)) - 1);
    int64_t cnt = 0;  // values with the prefix and a 0 at this bit
    for (int64_t i = threadIdx.x; i < n; i += kStatThreads) {
      const double bi = b[9 * i + a];
      const uint64_t k = order_key(cov[81 * i + 10 * a] / (bi * bi));
      cnt += ((k & hi_mask) == prefix) && !((k >> bit) & 1ull);
    }
    const int64_t zeros = (int64_t)block_sum((double)cnt, red);
    if (rank >= zeros) {
      rank -= zeros;
      prefix |= 1ull << bit;
    }
  }
  if (threadIdx.x == 0) {
    const uint64_t v = (prefix >> 63) ? (prefix & 0x7fffffffffffffffull) : ~prefix;
    s_glob[a] = sqrt(__longlong_as_double((long long)v));
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

void launch_col_stats(int64_t n, int cols, const float *x, float *mean, float *stdv,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_col_stats, dim3(cols), dim3(kStatThreads), 0, st, n, cols, x, mean, stdv);
}

void launch_col_robust(int64_t n, int cols, const float *x, float *center, float *spread,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_col_robust, dim3(cols), dim3(kStatThreads), 0, st, n, cols, x, center,
                     spread);
}

void launch_block_scale(int64_t n, const float *feat, double *b, DevStatus *ds, hipStream_t st) {
  hipLaunchKernelGGL(k_block_scale, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, n, feat, b,
                     ds);
}

void launch_diag_median(int64_t n, const double *cov, const double *b, double *s_glob,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_diag_median, dim3(9), dim3(kStatThreads), 0, st, n, cov, b, s_glob);
}

void launch_screener_features(const SceneDev &sc, const SceneWork &w, int32_t *hist,
                              double *ang, int32_t *covis, float *feat, hipStream_t st) {
  const int64_t n = sc.n;
  fill_i32(hist, 0, 8 * n, st);
  fill_f64(ang, 0.0, n, st);
  fill_i32(covis, 0, n, st);
  const int64_t t = sc.t;
  hipLaunchKernelGGL(k_feat_obs, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, sc, w.ptr_p,
                     w.slot_cam, w.slot_pt, hist, ang);
  const int64_t nb = n * (n + 1) / 2;
  hipLaunchKernelGGL(k_feat_covis, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, w.nzlist,
                     w.nzcount, covis);
  hipLaunchKernelGGL(k_feat_finish, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, (int)n,
                     w.zdiag, hist, ang, covis, feat);
}

int64_t mlp_param_count() {
  return (int64_t)kHid * kIn + kHid + 2 * ((int64_t)kHid * kHid + kHid) + (int64_t)kOut * kHid +
         kOut;
}

size_t mlp_workspace_bytes(int64_t batch) {
  // H1, H2, H3, dA (2) in BF16; Y, dY and the standardised input in FP32;
  // the loss accumulator
  return 2 * (size_t)batch * kHid * 5 + 4 * (size_t)batch * kOut * 2 + 4 * (size_t)batch * kIn +
         64;
}

namespace {

struct MlpView {
  const float *W[4], *b[4];
  int in[4], out[4];
};

MlpView view(const float *p) {
  MlpView v;
  const int dims[5] = {kIn, kHid, kHid, kHid, kOut};
  int64_t k = 0;
  for (int l = 0; l < 4; ++l) {
    v.in[l] = dims[l];
    v.out[l] = dims[l + 1];
    v.W[l] = p + k;
    k += (int64_t)dims[l] * dims[l + 1];
    v.b[l] = p + k;
    k += dims[l + 1];
  }
  return v;
}

struct MlpWork {
  unsigned short *H[3], *dA[2];
  float *Y, *dY, *Xs;
  double *loss;
};

MlpWork carve(void *ws, int64_t batch) {
  MlpWork w;
  char *c = static_cast<char *>(ws);
  const size_t hb = 2 * (size_t)batch * kHid;
  for (int i = 0; i < 3; ++i, c += hb) w.H[i] = reinterpret_cast<unsigned short *>(c);
  for (int i = 0; i < 2; ++i, c += hb) w.dA[i] = reinterpret_cast<unsigned short *>(c);
  w.Y = reinterpret_cast<float *>(c);
  c += 4 * (size_t)batch * kOut;
  w.dY = reinterpret_cast<float *>(c);
  c += 4 * (size_t)batch * kOut;
  w.Xs = reinterpret_cast<float *>(c);
  c += 4 * (size_t)batch * kIn;
  w.loss = reinterpret_cast<double *>((reinterpret_cast<uintptr_t>(c) + 7) & ~uintptr_t(7));
  return w;
}

MlpGemm gemm_args(int M, int N, int K, const void *A, int64_t lda, const void *B, int64_t ldb,
                  void *C, int64_t ldc) {
  MlpGemm g{};
  g.M = M;
  g.N = N;
  g.K = K;
  g.A = A;
  g.lda = lda;
  g.B = B;
  g.ldb = ldb;
  g.C = C;
  g.ldc = ldc;
  return g;
}

void forward(const MlpView &v, const MlpWork &w, int64_t batch, const float *x,
             const float *mean, const float *stdv, float *y, hipStream_t st) {
  const int B = (int)batch;
  const int64_t cnt = batch * kIn;
  hipLaunchKernelGGL(k_standardize, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, cnt, x,
                     mean, stdv, w.Xs);
  MlpGemm g = gemm_args(B, kHid, kIn, w.Xs, kIn, v.W[0], kIn, w.H[0], kHid);
  g.bias = v.b[0];
  gemm_launch<float, float, false, true, kBiasReluBf16>(g, st);
  for (int l = 1; l < 3; ++l) {
    g = gemm_args(B, kHid, kHid, w.H[l - 1], kHid, v.W[l], kHid, w.H[l], kHid);
    g.bias = v.b[l];
    gemm_launch<unsigned short, float, false, true, kBiasReluBf16>(g, st);
  }
  g = gemm_args(B, kOut, kHid, w.H[2], kHid, v.W[3], kHid, y, kOut);
  g.bias = v.b[3];
  gemm_launch<unsigned short, float, false, true, kBiasF32>(g, st);
}

// Gradient of the mean squared error into grad (flat, same layout as the
// parameters); loss accumulated into w.loss.
void backward(const MlpView &v, const MlpWork &w, float *grad, int64_t batch,
              const float *target, hipStream_t st) {
  const int B = (int)batch;
  const int64_t cnt = batch * kOut;
  fill_f64(w.loss, 0.0, 1, st);
  hipLaunchKernelGGL(k_mse, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, cnt, w.Y,
                     target, w.dY, w.loss);
  MlpView gv = view(grad);
  // layer 4: dW4 = dY^T H3, db4, dA3 = (dY W4) * [H3 > 0]
  gemm_launch<float, unsigned short, true, false, kStoreF32>(
      gemm_args(kOut, kHid, B, w.dY, kOut, w.H[2], kHid, const_cast<float *>(gv.W[3]), kHid), st);
  hipLaunchKernelGGL(k_colsum<float>, dim3(1), dim3(64), 0, st, B, kOut, w.dY,
                     const_cast<float *>(gv.b[3]));
  MlpGemm g = gemm_args(B, kHid, kOut, w.dY, kOut, v.W[3], kHid, w.dA[0], kHid);
  g.mask = w.H[2];
  gemm_launch<float, float, false, false, kReluMaskBf16>(g, st);
  // layers 3 and 2
  int cur = 0;
  for (int l = 2; l >= 1; --l) {
    const unsigned short *dA = w.dA[cur];
    gemm_launch<unsigned short, unsigned short, true, false, kStoreF32>(
        gemm_args(kHid, kHid, B, dA, kHid, w.H[l - 1], kHid, const_cast<float *>(gv.W[l]), kHid),
        st);
    hipLaunchKernelGGL(k_colsum<unsigned short>, dim3(kHid / 64), dim3(64), 0, st, B, kHid, dA,
                       const_cast<float *>(gv.b[l]));
    g = gemm_args(B, kHid, kHid, dA, kHid, v.W[l], kHid, w.dA[1 - cur], kHid);
    g.mask = w.H[l - 1];
    gemm_launch<unsigned short, float, false, false, kReluMaskBf16>(g, st);
    cur = 1 - cur;
  }
  // layer 1: dW1 = dA1^T Xs, db1
  g = gemm_args(kHid, kIn, B, w.dA[cur], kHid, w.Xs, kIn, const_cast<float *>(gv.W[0]), kIn);
  gemm_launch<unsigned short, float, true, false, kStoreF32>(g, st);
  hipLaunchKernelGGL(k_colsum<unsigned short>, dim3(kHid / 64), dim3(64), 0, st, B, kHid,
                     w.dA[cur], const_cast<float *>(gv.b[0]));
}

}  // namespace

void mlp_forward(const float *params, int64_t batch, const float *x, const float *mean,
                 const float *stdv, float *y, void *ws, hipStream_t st) {
  forward(view(params), carve(ws, batch), batch, x, mean, stdv, y, st);
}

void mlp_gradient(const float *params, int64_t batch, const float *x, const float *mean,
                  const float *stdv, const float *target, float *grad, float *loss, void *ws,
                  hipStream_t st) {
  const MlpView v = view(params);
  const MlpWork w = carve(ws, batch);
  forward(v, w, batch, x, mean, stdv, w.Y, st);
  backward(v, w, grad, batch, target, st);
  if (loss) hipLaunchKernelGGL(k_loss_out, dim3(1), dim3(1), 0, st, w.loss, loss);
}

void mlp_adam(int64_t n, float *params, const float *grad, float *m, float *v, float lr,
              int64_t step, hipStream_t st) {
  const float c1 = 1.f - powf(0.9f, (float)step), c2 = 1.f - powf(0.999f, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, params, grad,
                     m, v, lr, c1, c2);
}

void launch_labels(int64_t n, const double *cov, const double *b, const double *s_glob,
                   const float *mean, const float *stdv, bool clip, float *lab, DevStatus *ds,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_labels, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, n, cov, b, s_glob,
                     mean, stdv, clip, lab, ds);
}

void launch_predicted_cov(int64_t n, const float *y, const double *b, const double *s_glob,
                          const float *mean, const float *stdv, double *cov, double *spread,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_predicted_cov, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, n, y, b,
                     s_glob, mean, stdv, cov, spread);
}

}  // namespace ucov

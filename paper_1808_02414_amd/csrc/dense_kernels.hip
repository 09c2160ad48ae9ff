// Dense stage of the camera covariance (step a4): the inverse Cholesky
// factor of the Jacobi-scaled, gauge-regularised camera matrix and the
// per-camera covariance blocks read from it.
//
// With A_s = S (Z + a QQ^T) S = L L^T we need only the diagonal 9x9 blocks
// of A_s^-1 = L^-T L^-1, i.e. column-block inner products of L^-1.  L^-1 is
// produced by one recursion that interleaves the factorisation and the
// triangular inversion (2 N^3 / 3 flops in total):
//
//   [A11      ]        L11^-1 <- recurse(A11)
//   [A21  A22 ]  ->    T      <- A21 L11^-T            (= L21)
//                      A22    <- A22 - T T^T
//                      A21    <- T L11^-1
//                      L22^-1 <- recurse(A22)
//                      A21    <- -L22^-1 A21           (= (L^-1)21)
//
// The leaves are 64x64 blocks factored and inverted in LDS by one workgroup;
// the products run on FP64 MFMA (v_mfma_f64_16x16x4f64) in 64x64 output tiles.
#include "ucov_internal.h"
#include "../../include/ucov.h"

namespace ucov {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

enum KMode { kFull = 0, kLeN = 1, kGeN = 2, kLeM = 3 };

// ---------------------------------------------------------------------------
// C = alpha op(A) op(B) + beta C, 64x64 tile per workgroup, M, N, K multiples
// of 64.  BT: B is stored N x K and used transposed (C = A B^T); otherwise
// B is K x N.  LOWER: only tiles on or below the diagonal are computed.
// kmode restricts the K range to the nonzero part of a triangular operand:
//   kLeN  k < (tile_n + 1) * 64  (B lower triangular, used transposed)
//   kGeN  k >= tile_n * 64       (B lower triangular)
//   kLeM  k < (tile_m + 1) * 64  (A lower triangular)
// MFMA operand layout (16x16x4, 64 lanes): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; the accumulator holds D[4*v + l/16][l%16], v = 0..3.
// ---------------------------------------------------------------------------
constexpr int kKc = 16;     // K chunk staged in LDS
constexpr int kLdsPad = 4;  // row padding of the LDS tiles (doubles)

template <bool BT, bool LOWER>
__global__ __launch_bounds__(256) void k_gemm64(int64_t K, const double *__restrict__ A,
                                               int64_t lda, const double *__restrict__ B,
                                               int64_t ldb, double *__restrict__ C, int64_t ldc,
                                               double alpha, double beta, int kmode) {
  const int tm = blockIdx.x, tn = blockIdx.y;
  if (LOWER && tn > tm) return;
  int64_t kb = 0, ke = K;
  if (kmode == kLeN) ke = min(K, (int64_t)(tn + 1) * 64);
  else if (kmode == kGeN) kb = (int64_t)tn * 64;
  else if (kmode == kLeM) ke = min(K, (int64_t)(tm + 1) * 64);

  __shared__ double As[kKc][64 + kLdsPad];
  __shared__ double Bs[kKc][64 + kLdsPad];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  const int la_k = tid >> 4, la_m = (tid & 15) * 4;  // A (and B^T) loader
  const int lb_n = tid >> 2, lb_k = (tid & 3) * 4;   // B (K x N) loader
  const double *pa = A + (int64_t)tm * 64 + la_m + la_k * lda;
  const double *pb = BT ? B + (int64_t)tn * 64 + la_m + la_k * ldb
                        : B + lb_k + ((int64_t)tn * 64 + lb_n) * ldb;
  double ra[4], rb[4];
  auto load = [&](int64_t k0) {
    const double2 a01 = *reinterpret_cast<const double2 *>(pa + k0 * lda);
    const double2 a23 = *reinterpret_cast<const double2 *>(pa + k0 * lda + 2);
    ra[0] = a01.x; ra[1] = a01.y; ra[2] = a23.x; ra[3] = a23.y;
    if (BT) {
      const double2 b01 = *reinterpret_cast<const double2 *>(pb + k0 * ldb);
      const double2 b23 = *reinterpret_cast<const double2 *>(pb + k0 * ldb + 2);
      rb[0] = b01.x; rb[1] = b01.y; rb[2] = b23.x; rb[3] = b23.y;
    } else {
      const double2 b01 = *reinterpret_cast<const double2 *>(pb + k0);
      const double2 b23 = *reinterpret_cast<const double2 *>(pb + k0 + 2);
      rb[0] = b01.x; rb[1] = b01.y; rb[2] = b23.x; rb[3] = b23.y;
    }
  };
  if (kb < ke) load(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += kKc) {
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) As[la_k][la_m + v] = ra[v];
    if (BT) {
#pragma unroll
      for (int v = 0; v < 4; ++v) Bs[la_k][la_m + v] = rb[v];
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) Bs[lb_k + v][lb_n] = rb[v];
    }
    __syncthreads();
    if (k0 + kKc < ke) load(k0 + kKc);  // prefetch the next chunk during the MFMAs
#pragma unroll
    for (int kk = 0; kk < kKc / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      const int c = lane & 15;
      const double a0 = As[kr][wm * 32 + c], a1 = As[kr][wm * 32 + 16 + c];
      const double b0 = Bs[kr][wn * 32 + c], b1 = Bs[kr][wn * 32 + 16 + c];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int64_t col = (int64_t)tn * 64 + wn * 32 + bj * 16 + (lane & 15);
      const int64_t row = (int64_t)tm * 64 + wm * 32 + bi * 16 + (lane >> 4);
      double *pc = C + row + col * ldc;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double x = alpha * acc[bi][bj][v];
        pc[4 * v] = beta == 0.0 ? x : x + beta * pc[4 * v];
      }
    }
}

// ---------------------------------------------------------------------------
// 64x64 leaf: Cholesky factor L of the lower triangle and its inverse, in
// LDS; writes L^-1 (lower) and zeros above the diagonal of the tile.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_leaf64(double *A, int64_t lda, int64_t o,
                                               DevStatus *ds) {
  __shared__ double Ls[64][65];
  __shared__ double Xs[64][65];
  __shared__ double dg[64];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  double *T = A + o + o * lda;
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    Ls[r][c] = r >= c ? T[r + (int64_t)c * lda] : 0.0;
    Xs[r][c] = r == c ? 1.0 : 0.0;
  }
  __syncthreads();
  // symmetric Gaussian elimination: after step j, column j holds L[:, j] L[j][j]
  for (int j = 0; j < 64; ++j) {
    const double piv = Ls[j][j];
    if (tid == 0 && !(piv > 0.0)) report_error(ds, UCOV_EGAUGE, (int)((o + j) / 9));
    const double inv = 1.0 / piv;
    const double lr = Ls[lane][j];
    for (int c = j + 1 + wid; c < 64; c += 4) {
      if (lane >= c) Ls[lane][c] -= lr * Ls[c][j] * inv;
    }
    __syncthreads();
  }
  if (tid < 64) dg[tid] = sqrt(Ls[tid][tid]);
  __syncthreads();
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    if (r > c) Ls[r][c] /= dg[c];
    else if (r == c) Ls[r][c] = dg[c];
  }
  __syncthreads();
  // X = L^-1 by forward elimination on the identity: with y_j final,
  // y_r -= (L[r][j] / L[j][j]) y_j for r > j; finally x_r = y_r / L[r][r].
  for (int j = 0; j < 63; ++j) {
    const double f = (lane > j) ? Ls[lane][j] / Ls[j][j] : 0.0;
    for (int c = wid; c <= j; c += 4) {
      if (lane > j) Xs[lane][c] -= f * Xs[j][c];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    T[r + (int64_t)c * lda] = r >= c ? Xs[r][c] / Ls[r][r] : 0.0;
  }
}

// copy an m x n block
__global__ void k_copy(int64_t m, int64_t n, const double *src, int64_t lds, double *dst,
                       int64_t ldd) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r < m && c < n) dst[r + c * ldd] = src[r + c * lds];
}

__global__ void k_pad_identity(int64_t N, int64_t Np, double *a, int64_t lda) {
  const int64_t c = blockIdx.x;
  const int64_t r0 = c > N ? c : N;
  for (int64_t r = r0 + threadIdx.x; r < Np; r += blockDim.x)
    a[r + c * lda] = (r == c) ? 1.0 : 0.0;
}

__global__ void k_scale_dense(int64_t N, const double *z, int64_t ldz, const double *q,
                              const double *s, const double *alpha, double *a, int64_t lda) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r >= N) return;  // both triangles are written; the factorisation reads the lower one
  double g = 0.0;
#pragma unroll
  for (int k = 0; k < 7; ++k) g += q[k * N + r] * q[k * N + c];
  a[r + c * lda] = s[r] * (z[r + c * ldz] + (*alpha) * g) * s[c];
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// One workgroup per camera: (A_s^-1)_ii = sum over rows r >= 9i of the outer
// products of row r of L^-1 restricted to the camera's 9 columns.
__global__ __launch_bounds__(256) void k_extract(int64_t N, const double *linv, int64_t ld,
                                                const double *s, const double *q,
                                                const double *alpha, double *cov) {
  const int64_t i = blockIdx.x;
  const int64_t c0 = 9 * i;
  double acc[45];
#pragma unroll
  for (int k = 0; k < 45; ++k) acc[k] = 0.0;
  for (int64_t r = c0 + threadIdx.x; r < N; r += blockDim.x) {
    // only the lower triangle of linv is defined: a camera's columns may
    // straddle two tiles, whose upper-right part is never written
    double v[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) v[c] = r >= c0 + c ? linv[r + (c0 + c) * ld] : 0.0;
    int idx = 0;
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
      for (int b = a; b < 9; ++b) acc[idx++] += v[a] * v[b];
  }
  __shared__ double part[4][45];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 45; ++k) {
    const double v = wave_sum(acc[k]);
    if (lane == 0) part[wid][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 81) {
    const int a0 = threadIdx.x / 9, b0 = threadIdx.x % 9;
    const int a = a0 < b0 ? a0 : b0, b = a0 < b0 ? b0 : a0;
    const int idx = a * 9 - a * (a - 1) / 2 + (b - a);
    const double x = part[0][idx] + part[1][idx] + part[2][idx] + part[3][idx];
    double g = 0.0;
#pragma unroll
    for (int k = 0; k < 7; ++k) g += q[k * N + c0 + a0] * q[k * N + c0 + b0];
    cov[81 * i + threadIdx.x] = s[c0 + a0] * x * s[c0 + b0] - g / (*alpha);
  }
}

template <bool BT, bool LOWER>
void gemm(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda, const double *B,
          int64_t ldb, double *C, int64_t ldc, double alpha, double beta, int kmode,
          hipStream_t st) {
  dim3 grid((unsigned)(M / 64), (unsigned)(N / 64));
  hipLaunchKernelGGL((k_gemm64<BT, LOWER>), grid, dim3(256), 0, st, K, A, lda, B, ldb, C, ldc,
                     alpha, beta, kmode);
}

void recurse(double *A, int64_t lda, int64_t o, int64_t n, double *T, int64_t ldt,
             DevStatus *ds, hipStream_t st) {
  if (n == 64) {
    hipLaunchKernelGGL(k_leaf64, dim3(1), dim3(256), 0, st, A, lda, o, ds);
    return;
  }
  const int64_t tiles = n / 64;
  const int64_t n1 = (tiles / 2) * 64, n2 = n - n1;
  recurse(A, lda, o, n1, T, ldt, ds, st);
  double *A11 = A + o + o * lda;
  double *A21 = A + (o + n1) + o * lda;
  double *A22 = A + (o + n1) + (o + n1) * lda;
  gemm<true, false>(n2, n1, n1, A21, lda, A11, lda, T, ldt, 1.0, 0.0, kLeN, st);
  gemm<true, true>(n2, n2, n1, T, ldt, T, ldt, A22, lda, -1.0, 1.0, kFull, st);
  gemm<false, false>(n2, n1, n1, T, ldt, A11, lda, A21, lda, 1.0, 0.0, kGeN, st);
  recurse(A, lda, o + n1, n2, T, ldt, ds, st);
  gemm<false, false>(n2, n1, n2, A22, lda, A21, lda, T, ldt, -1.0, 0.0, kLeM, st);
  hipLaunchKernelGGL(k_copy, dim3((unsigned)((n2 + 255) / 256), (unsigned)n1), dim3(256), 0,
                     st, n2, n1, T, ldt, A21, lda);
}

}  // namespace

void launch_scale_dense(int64_t N, const double *z, int64_t ldz, const double *q,
                        const double *s, const double *alpha, double *a, int64_t lda,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_scale_dense, dim3((unsigned)((N + 255) / 256), (unsigned)N), dim3(256),
                     0, st, N, z, ldz, q, s, alpha, a, lda);
}

void launch_pad_identity(int64_t N, int64_t Np, double *a, int64_t lda, hipStream_t st) {
  if (Np == N) return;
  hipLaunchKernelGGL(k_pad_identity, dim3((unsigned)Np), dim3(64), 0, st, N, Np, a, lda);
}

void spd_lower_inverse_fp64(double *a, int64_t lda, int64_t Np, double *tmp, int64_t ldt,
                            DevStatus *ds, hipStream_t st) {
  recurse(a, lda, 0, Np, tmp, ldt, ds, st);
}

void launch_extract(int64_t N, const double *linv, int64_t ld, const double *s,
                    const double *q, const double *alpha, double *cov, hipStream_t st) {
  hipLaunchKernelGGL(k_extract, dim3((unsigned)(N / 9)), dim3(256), 0, st, N, linv, ld, s, q,
                     alpha, cov);
}

}  // namespace ucov

// Split-BF16 products on BF16 MFMA: the Newton-Schulz correction X <- X + X R
// of the mixed-precision inverse, with X R formed from 8-bit slices of X and
// R whose products sum exactly in FP32 (Ozaki-style error-free splitting).
//
// Every entry of X is written relative to a power of two 2^e_m that bounds
// its row m (every entry of R relative to one per column c) as S fixed-point
// slices of 8 significant bits,
//   x 2^-e = s_0 + s_1 + ... + s_{S-1} + t,   s_i = q_i 2^(-8(i+1)),
// with integers |q_0| <= 256, |q_i| <= 128 (i > 0) from rounding to nearest,
// and |t| <= 2^(-8S-1): each slice is exact in BF16 (8 significant bits).
// The product of slice i of X and slice j of R is an integer multiple of
// 2^(-8(g+2)), g = i + j, at most 2^16 units per term for g = 0 and 2^15 for
// g > 0 (|q_0| <= 256, |q_i| <= 128), so the FP32 sum of the g + 1 pairs of
// group g over a K chunk of 64 terms stays below 2^24 units (g = 3: 4 pairs,
// 64 terms, 2^15 + 2^14 + 2^14 + 2^15 per k: 96 Ki units per k, 6 Mi in all)
// and is exact whatever order the MFMA adds in.  Pairs with i + j < S are kept and the exact chunk sums are added
// in FP64, so the product carries only the dropped slice terms: about
// 2^(-8S) relative to the row and column bounds, independent of K.
#include <hip/hip_runtime.h>

#include "ucov_internal.h"

namespace ucov {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kSTile = 64;      // output tile of a workgroup
constexpr int kKs = 32;        // K of one MFMA and of one LDS stage
constexpr int kFlushK = 64;    // K between the FP64 flushes of the exact FP32 sums
constexpr int kLdsRow = kKs + 8;  // LDS row pitch in BF16 (16-byte aligned rows)
constexpr int kNoExp = -1100;  // exponent of an all-zero row or column

inline unsigned blocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// Bound exponent of |x|: |x| < 2^e.
__device__ inline int bound_exp(double x) { return x == 0.0 ? kNoExp : ilogb(x) + 1; }

__global__ void k_fill_exp(int64_t n, int *e) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) e[i] = kNoExp;
}

// e[m] = bound exponent of row m of the n x n column-major a; each thread a
// row and one of 64 interleaved column sets (the maximum is order-free).
__global__ __launch_bounds__(256) void k_exp_rows(int64_t n, const double *a, int64_t lda,
                                                 int *e) {
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= n) return;
  int best = kNoExp;
  for (int64_t c = blockIdx.y; c < n; c += gridDim.y) best = max(best, bound_exp(a[m + c * lda]));
  atomicMax(&e[m], best);
}

// e[c] = bound exponent of column c, one workgroup per column.
__global__ __launch_bounds__(256) void k_exp_cols(int64_t n, const double *a, int64_t lda,
                                                 int *e) {
  const int64_t c = blockIdx.x;
  int best = kNoExp;
  for (int64_t m = threadIdx.x; m < n; m += 256) best = max(best, bound_exp(a[m + c * lda]));
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) best = max(best, __shfl_xor(best, d, 64));
  __shared__ int part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) e[c] = max(max(part[0], part[1]), max(part[2], part[3]));
}

// BF16 bits of a float that BF16 holds exactly.
__device__ inline unsigned short exact_bf16(float f) { return (unsigned short)(__float_as_uint(f) >> 16); }

// The S slices of x 2^-e (see the file comment).
template <int S>
__device__ inline void split(double x, int e, unsigned short q[S]) {
  double v = e == kNoExp ? 0.0 : ldexp(x, -e);
#pragma unroll
  for (int i = 0; i < S; ++i) {
    const double sc = ldexp(1.0, 8 * (i + 1));
    const double s = rint(v * sc) / sc;
    q[i] = exact_bf16((float)s);
    v -= s;
  }
}

// Slices of the rows of X: out[i][m][k] (row-major n x n per slice, K
// contiguous for the MFMA operand loads).  Each thread one row m and 8
// consecutive k (column reads coalesced across the wave).
template <int S>
__global__ __launch_bounds__(256) void k_split_rows(int64_t n, const double *x, int64_t ldx,
                                                   const int *e, unsigned short *out) {
  const int64_t m = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int64_t k0 = (int64_t)blockIdx.y * 32 + (threadIdx.x >> 6) * 8;
  if (m >= n || k0 >= n) return;
  const int em = e[m];
  unsigned short q[8][S];
#pragma unroll
  for (int u = 0; u < 8; ++u) split<S>(x[m + (k0 + u) * ldx], em, q[u]);
#pragma unroll
  for (int i = 0; i < S; ++i) {
    uint4 w;
    w.x = q[0][i] | ((unsigned)q[1][i] << 16);
    w.y = q[2][i] | ((unsigned)q[3][i] << 16);
    w.z = q[4][i] | ((unsigned)q[5][i] << 16);
    w.w = q[6][i] | ((unsigned)q[7][i] << 16);
    *reinterpret_cast<uint4 *>(out + (size_t)i * n * n + m * n + k0) = w;
  }
}

// Slices of the columns of R: out[j][c][k] (column-major like R).
template <int S>
__global__ __launch_bounds__(256) void k_split_cols(int64_t n, const double *r, int64_t ldr,
                                                   const int *e, unsigned short *out) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (k >= n) return;
  unsigned short q[S];
  split<S>(r[k + c * ldr], e[c], q);
#pragma unroll
  for (int j = 0; j < S; ++j) out[(size_t)j * n * n + c * n + k] = q[j];
}

// x (in place, n x n column-major) += 2^(ex[m] + er[c]) sum_{i+j<S} A_i B_j
// for the 64 x 64 tile (blockIdx.x, blockIdx.y): 4 waves, each a 32 x 32
// quarter as 2 x 2 tiles of v_mfma_f32_16x16x32_bf16 (lane l supplies row
// l % 16, k = 8 (l / 16) .. + 7 of either operand; accumulator register v
// holds row 4 (l / 16) + v, column l % 16).  One FP32 accumulator set per
// group g = i + j, flushed into FP64 every kFlushK.  The tile of x is read
// and written by the same thread only, and the operands come from the
// slices, so the update in place is race-free.
template <int S>
__global__ __launch_bounds__(256, 2) void k_gemm_bf16x(int64_t n, const unsigned short *as,
                                                   const unsigned short *bs, const int *ex,
                                                   const int *er, double *x, int64_t ldx) {
  __shared__ __attribute__((aligned(16))) unsigned short sa[S][kSTile * kLdsRow];
  __shared__ __attribute__((aligned(16))) unsigned short sb[S][kSTile * kLdsRow];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = (wid >> 1) * 32, wn = (wid & 1) * 32;
  const int64_t m0 = (int64_t)blockIdx.x * kSTile, n0 = (int64_t)blockIdx.y * kSTile;
  const size_t slice = (size_t)n * n;
  // loader: thread -> row (or column) tid / 4 of the tile, 8 k at (tid % 4) * 8;
  // the next stage's slices wait in registers while the MFMAs run
  const int lr = tid >> 2, lk = (tid & 3) * 8;
  const unsigned short *pa = as + (m0 + lr) * n + lk;
  const unsigned short *pb = bs + (n0 + lr) * n + lk;
  uint4 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
#define UCOV_SPLIT_LOAD(k0)                                                        \
  do {                                                                             \
    ra0 = *reinterpret_cast<const uint4 *>(pa + (k0));                             \
    rb0 = *reinterpret_cast<const uint4 *>(pb + (k0));                             \
    ra1 = *reinterpret_cast<const uint4 *>(pa + slice + (k0));                     \
    rb1 = *reinterpret_cast<const uint4 *>(pb + slice + (k0));                     \
    if (S > 2) {                                                                   \
      ra2 = *reinterpret_cast<const uint4 *>(pa + 2 * slice + (k0));               \
      rb2 = *reinterpret_cast<const uint4 *>(pb + 2 * slice + (k0));               \
    }                                                                              \
    if (S > 3) {                                                                   \
      ra3 = *reinterpret_cast<const uint4 *>(pa + 3 * slice + (k0));               \
      rb3 = *reinterpret_cast<const uint4 *>(pb + 3 * slice + (k0));               \
    }                                                                              \
  } while (0)
  f4 acc[S][2][2];
  double sum[2][2][4];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
#pragma unroll
      for (int g = 0; g < S; ++g) acc[g][bi][bj] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) sum[bi][bj][v] = 0.0;
    }
  UCOV_SPLIT_LOAD(0);
  for (int64_t k0 = 0; k0 < n; k0 += kKs) {
    __syncthreads();
    {
      const int o = lr * kLdsRow + lk;
      *reinterpret_cast<uint4 *>(&sa[0][o]) = ra0;
      *reinterpret_cast<uint4 *>(&sb[0][o]) = rb0;
      *reinterpret_cast<uint4 *>(&sa[1][o]) = ra1;
      *reinterpret_cast<uint4 *>(&sb[1][o]) = rb1;
      if (S > 2) {
        *reinterpret_cast<uint4 *>(&sa[S > 2 ? 2 : 0][o]) = ra2;
        *reinterpret_cast<uint4 *>(&sb[S > 2 ? 2 : 0][o]) = rb2;
      }
      if (S > 3) {
        *reinterpret_cast<uint4 *>(&sa[S > 3 ? 3 : 0][o]) = ra3;
        *reinterpret_cast<uint4 *>(&sb[S > 3 ? 3 : 0][o]) = rb3;
      }
    }
    __syncthreads();
    if (k0 + kKs < n) UCOV_SPLIT_LOAD(k0 + kKs);
    // the slices of R for this k-step, then slice by slice of X: pair (i, j)
    // of group i + j (only i + j < S)
    const int kq = 8 * (lane >> 4);
    bf16x8 fb[S][2];
#pragma unroll
    for (int j = 0; j < S; ++j)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        fb[j][b] = *reinterpret_cast<const bf16x8 *>(&sb[j][(wn + 16 * b + (lane & 15)) * kLdsRow + kq]);
#pragma unroll
    for (int i = 0; i < S; ++i) {
      bf16x8 fa[2];
#pragma unroll
      for (int b = 0; b < 2; ++b)
        fa[b] = *reinterpret_cast<const bf16x8 *>(&sa[i][(wm + 16 * b + (lane & 15)) * kLdsRow + kq]);
#pragma unroll
      for (int j = 0; j + i < S; ++j)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
            acc[i + j][bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                fa[bi], fb[j][bj], acc[i + j][bi][bj], 0, 0, 0);
    }
    if ((k0 + kKs) % kFlushK == 0 || k0 + kKs >= n) {
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double t = 0.0;
#pragma unroll
            for (int g = 0; g < S; ++g) t += (double)acc[g][bi][bj][v];
            sum[bi][bj][v] += t;
#pragma unroll
            for (int g = 0; g < S; ++g) acc[g][bi][bj][v] = 0.f;
          }
    }
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm + 16 * bi + 4 * (lane >> 4) + v;
        const int64_t col = n0 + wn + 16 * bj + (lane & 15);
        const int e = ex[row] + er[col];
        if (ex[row] == kNoExp || er[col] == kNoExp) continue;
        x[row + col * ldx] += ldexp(sum[bi][bj][v], e);
      }
#undef UCOV_SPLIT_LOAD
}

// The same product on 128 x 128 tiles (three slices only): 8 waves, each a
// 32 x 64 part as 2 x 4 MFMA tiles, which halves the slice panels each tile
// streams past the L2 and reads a quarter fewer LDS bytes per MFMA; all A
// fragments of a step stay in registers while the B slices go by (about 240
// registers, two waves per SIMD, one workgroup per CU).  n is a multiple of
// 64, so the last tile row or column may be half outside: its loads repeat
// the first half (in bounds) and its stores are skipped.
constexpr int kBTile = 128;
constexpr int64_t kBigSplitN = 512;  // from this size the 128 x 128 tiles

__global__ __launch_bounds__(512, 1) void k_gemm_bf16x3_big(int64_t n, const unsigned short *as,
                                                         const unsigned short *bs,
                                                         const int *ex, const int *er,
                                                         double *x, int64_t ldx) {
  constexpr int S = 3;
  __shared__ __attribute__((aligned(16))) unsigned short sa[S][kBTile * kLdsRow];
  __shared__ __attribute__((aligned(16))) unsigned short sb[S][kBTile * kLdsRow];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = (wid >> 1) * 32, wn = (wid & 1) * 64;
  const int64_t m0 = (int64_t)blockIdx.x * kBTile, n0 = (int64_t)blockIdx.y * kBTile;
  const size_t slice = (size_t)n * n;
  // loader: thread -> row tid / 4 of the tile, 8 k at (tid % 4) * 8
  const int lr = tid >> 2, lk = (tid & 3) * 8;
  const int64_t ar = m0 + lr < n ? m0 + lr : m0 + lr - 64;  // in bounds
  const int64_t br = n0 + lr < n ? n0 + lr : n0 + lr - 64;
  const unsigned short *pa = as + ar * n + lk;
  const unsigned short *pb = bs + br * n + lk;
  uint4 ra0, ra1, ra2, rb0, rb1, rb2;
#define UCOV_SPLIT_LOAD3(k0)                                         \
  do {                                                               \
    ra0 = *reinterpret_cast<const uint4 *>(pa + (k0));               \
    rb0 = *reinterpret_cast<const uint4 *>(pb + (k0));               \
    ra1 = *reinterpret_cast<const uint4 *>(pa + slice + (k0));       \
    rb1 = *reinterpret_cast<const uint4 *>(pb + slice + (k0));       \
    ra2 = *reinterpret_cast<const uint4 *>(pa + 2 * slice + (k0));   \
    rb2 = *reinterpret_cast<const uint4 *>(pb + 2 * slice + (k0));   \
  } while (0)
  f4 acc[S][2][4];
  double sum[2][4][4];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
#pragma unroll
      for (int g = 0; g < S; ++g) acc[g][bi][bj] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) sum[bi][bj][v] = 0.0;
    }
  UCOV_SPLIT_LOAD3(0);
  for (int64_t k0 = 0; k0 < n; k0 += kKs) {
    __syncthreads();
    {
      const int o = lr * kLdsRow + lk;
      *reinterpret_cast<uint4 *>(&sa[0][o]) = ra0;
      *reinterpret_cast<uint4 *>(&sb[0][o]) = rb0;
      *reinterpret_cast<uint4 *>(&sa[1][o]) = ra1;
      *reinterpret_cast<uint4 *>(&sb[1][o]) = rb1;
      *reinterpret_cast<uint4 *>(&sa[2][o]) = ra2;
      *reinterpret_cast<uint4 *>(&sb[2][o]) = rb2;
    }
    __syncthreads();
    if (k0 + kKs < n) UCOV_SPLIT_LOAD3(k0 + kKs);
    const int kq = 8 * (lane >> 4);
    bf16x8 fa[S][2];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        fa[i][b] = *reinterpret_cast<const bf16x8 *>(&sa[i][(wm + 16 * b + (lane & 15)) * kLdsRow + kq]);
#pragma unroll
    for (int j = 0; j < S; ++j) {
      bf16x8 fb[4];
#pragma unroll
      for (int b = 0; b < 4; ++b)
        fb[b] = *reinterpret_cast<const bf16x8 *>(&sb[j][(wn + 16 * b + (lane & 15)) * kLdsRow + kq]);
#pragma unroll
      for (int i = 0; i + j < S; ++i)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 4; ++bj)
            acc[i + j][bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i][bi], fb[bj],
                                                                         acc[i + j][bi][bj], 0, 0, 0);
    }
    if ((k0 + kKs) % kFlushK == 0 || k0 + kKs >= n) {
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double t = 0.0;
#pragma unroll
            for (int g = 0; g < S; ++g) t += (double)acc[g][bi][bj][v];
            sum[bi][bj][v] += t;
#pragma unroll
            for (int g = 0; g < S; ++g) acc[g][bi][bj][v] = 0.f;
          }
    }
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm + 16 * bi + 4 * (lane >> 4) + v;
        const int64_t col = n0 + wn + 16 * bj + (lane & 15);
        if (row >= n || col >= n) continue;
        if (ex[row] == kNoExp || er[col] == kNoExp) continue;
        x[row + col * ldx] += ldexp(sum[bi][bj][v], ex[row] + er[col]);
      }
#undef UCOV_SPLIT_LOAD3
}

}  // namespace

int split_bf16_slices(int64_t n) { return n > kSplitSmallN ? 4 : 3; }

size_t split_bf16_scratch(int64_t n) {
  return 2 * (size_t)split_bf16_slices(n) * n * n * 2 + 8 * (size_t)n;
}

namespace {

template <int S>
void update(int64_t n, double *x, const double *r, void *scratch, hipStream_t st) {
  unsigned short *as = static_cast<unsigned short *>(scratch);
  unsigned short *bs = as + (size_t)S * n * n;
  int *ex = reinterpret_cast<int *>(bs + (size_t)S * n * n);
  int *er = ex + n;
  hipLaunchKernelGGL(k_fill_exp, dim3(blocks(n, 256)), dim3(256), 0, st, n, ex);
  hipLaunchKernelGGL(k_exp_rows, dim3(blocks(n, 256), 64), dim3(256), 0, st, n, x, n, ex);
  hipLaunchKernelGGL(k_exp_cols, dim3((unsigned)n), dim3(256), 0, st, n, r, n, er);
  hipLaunchKernelGGL((k_split_rows<S>), dim3(blocks(n, 64), blocks(n, 32)), dim3(256), 0, st, n,
                     x, n, ex, as);
  hipLaunchKernelGGL((k_split_cols<S>), dim3(blocks(n, 256), (unsigned)n), dim3(256), 0, st, n,
                     r, n, er, bs);
  if (S == 3 && n >= kBigSplitN) {
    const unsigned t = blocks(n, kBTile);
    hipLaunchKernelGGL(k_gemm_bf16x3_big, dim3(t, t), dim3(512), 0, st, n, as, bs, ex, er, x, n);
    return;
  }
  hipLaunchKernelGGL((k_gemm_bf16x<S>), dim3((unsigned)(n / kSTile), (unsigned)(n / kSTile)),
                     dim3(256), 0, st, n, as, bs, ex, er, x, n);
}

}  // namespace

void split_bf16_update(int64_t n, double *x, const double *r, void *scratch, hipStream_t st) {
  if (split_bf16_slices(n) == 4) update<4>(n, x, r, scratch, st);
  else update<3>(n, x, r, scratch, st);
}

}  // namespace ucov

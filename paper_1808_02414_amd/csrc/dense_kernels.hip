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
//                      A22    <- A22 - T T^T       } one launch
//                      T2     <- T L11^-1          }
//                      L22^-1 <- recurse(A22)
//                      A21    <- -L22^-1 T2            (= (L^-1)21)
//
// Leaves of 128 (or 64) are factored and inverted by one workgroup in LDS;
// every product runs on MFMA.  The recursion is generic over the element
// type: FP64 (v_mfma_f64_16x16x4f64) for the plain path, FP32
// (v_mfma_f32_16x16x4f32) for the initial inverse of the mixed path, which
// Newton-Schulz steps with FP64 residuals then refine (see ucov_api.hip).
#include <algorithm>
#include <type_traits>
#include <utility>

#include <string>
#include <vector>

#include "ucov_internal.h"
#include "../../include/ucov.h"

namespace ucov {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// MFMA 16x16x4 of the element type.  Operand layout (64 lanes): lane l
// supplies A[l%16][l/16] and B[l/16][l%16].  Accumulator register v of lane l
// holds D[row(l, v)][l%16] with row = 4*v + l/16 for FP64 and
// row = 4*(l/16) + v for FP32 (the two instructions interleave rows
// differently).
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef d4 acc_t;
  typedef double2 vec2;
  __device__ static acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <>
struct Mfma<float> {
  typedef f4 acc_t;
  typedef float2 vec2;
  __device__ static acc_t zero() { return acc_t{0.0f, 0.0f, 0.0f, 0.0f}; }
  __device__ static acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

enum KMode { kFull = 0, kLeN = 1, kGeN = 2, kLeM = 3, kGeMN = 4 };

// ---------------------------------------------------------------------------
// C = alpha op(A) op(B) + beta C, 64x64 tile per workgroup, M, N, K multiples
// of 64.  AT: A is stored K x M and used transposed; BT: B is stored N x K
// and used transposed; otherwise A is M x K and B is K x N (column-major).
// LOWER: only tiles on or below the diagonal are computed.  kmode restricts
// the K range to the nonzero part of a triangular operand (tile granular;
// the upper part of diagonal tiles of a triangular operand is zero):
//   kLeN  k < (tile_n + 1) * 64  (B lower triangular, used transposed)
//   kGeN  k >= tile_n * 64       (B lower triangular)
//   kLeM  k < (tile_m + 1) * 64  (A lower triangular)
//   kGeMN k >= max(tile_m, tile_n) * 64  (A^T B with A, B lower triangular)
// Measured on MI355X: single-buffered LDS with a register prefetch and 4
// waves/SIMD occupancy beats double buffering and die-aware tile orders for
// these tiles.  Products large enough for at least kBigTiles tiles of
// 128 x 128 run on the 8-wave kernel below instead (square FP64 products:
// 60-65 against 48-50 TFLOP/s from n = 3456 up; at n = 2304 the 64 x 64
// tiles win, 46 against 42).
// ---------------------------------------------------------------------------
constexpr int kKc = 16;  // K chunk staged in LDS
constexpr int kPad = 4;  // row padding of the LDS tiles

template <typename T>
struct GemmArgs {
  int64_t M, N, K;
  const T *A;
  int64_t lda;
  const T *B;
  int64_t ldb;
  T *C;
  int64_t ldc;
  T alpha, beta;
  int kmode;
};

template <typename T, bool AT, bool BT, bool LOWER>
__device__ inline void gemm_tile(const GemmArgs<T> &g, int tm, int tn) {
  typedef Mfma<T> MF;
  typedef typename MF::vec2 V2;
  if (LOWER && tn > tm) return;
  const int64_t K = g.K, lda = g.lda, ldb = g.ldb, ldc = g.ldc;
  const T *__restrict__ A = g.A;
  const T *__restrict__ B = g.B;
  T *__restrict__ C = g.C;
  const int kmode = g.kmode;
  int64_t kb = 0, ke = K;
  if (kmode == kLeN) ke = min(K, (int64_t)(tn + 1) * 64);
  else if (kmode == kGeN) kb = (int64_t)tn * 64;
  else if (kmode == kLeM) ke = min(K, (int64_t)(tm + 1) * 64);
  else if (kmode == kGeMN) kb = (int64_t)max(tm, tn) * 64;

  __shared__ T As[kKc][64 + kPad];
  __shared__ T Bs[kKc][64 + kPad];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  typename MF::acc_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = MF::zero();

  // loaders: 4 consecutive elements per thread per chunk
  const int lt_k = tid >> 4, lt_m = (tid & 15) * 4;  // K-major tile (M contiguous)
  const int lc_m = tid >> 2, lc_k = (tid & 3) * 4;   // M-major tile (K contiguous)
  const T *pa = AT ? A + lc_k + ((int64_t)tm * 64 + lc_m) * lda
                   : A + (int64_t)tm * 64 + lt_m + lt_k * lda;
  const T *pb = BT ? B + (int64_t)tn * 64 + lt_m + lt_k * ldb
                   : B + lc_k + ((int64_t)tn * 64 + lc_m) * ldb;
  T ra[4], rb[4];
  auto load = [&](int64_t k0) {
    const T *qa = AT ? pa + k0 : pa + k0 * lda;
    const V2 a01 = *reinterpret_cast<const V2 *>(qa);
    const V2 a23 = *reinterpret_cast<const V2 *>(qa + 2);
    ra[0] = a01.x; ra[1] = a01.y; ra[2] = a23.x; ra[3] = a23.y;
    const T *qb = BT ? pb + k0 * ldb : pb + k0;
    const V2 b01 = *reinterpret_cast<const V2 *>(qb);
    const V2 b23 = *reinterpret_cast<const V2 *>(qb + 2);
    rb[0] = b01.x; rb[1] = b01.y; rb[2] = b23.x; rb[3] = b23.y;
  };
  if (kb < ke) load(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += kKc) {
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (AT) As[lc_k + v][lc_m] = ra[v];
      else As[lt_k][lt_m + v] = ra[v];
      if (BT) Bs[lt_k][lt_m + v] = rb[v];
      else Bs[lc_k + v][lc_m] = rb[v];
    }
    __syncthreads();
    if (k0 + kKc < ke) load(k0 + kKc);  // prefetch the next chunk during the MFMAs
#pragma unroll
    for (int kk = 0; kk < kKc / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      const int c = lane & 15;
      const T a0 = As[kr][wm * 32 + c], a1 = As[kr][wm * 32 + 16 + c];
      const T b0 = Bs[kr][wn * 32 + c], b1 = Bs[kr][wn * 32 + 16 + c];
      acc[0][0] = MF::mma(a0, b0, acc[0][0]);
      acc[0][1] = MF::mma(a0, b1, acc[0][1]);
      acc[1][0] = MF::mma(a1, b0, acc[1][0]);
      acc[1][1] = MF::mma(a1, b1, acc[1][1]);
    }
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int64_t col = (int64_t)tn * 64 + wn * 32 + bj * 16 + (lane & 15);
      const int64_t row0 = (int64_t)tm * 64 + wm * 32 + bi * 16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        T *pc = C + row0 + MF::row(lane, v) + col * ldc;
        const T x = g.alpha * acc[bi][bj][v];
        *pc = g.beta == T(0) ? x : x + g.beta * (*pc);
      }
    }
}

// ---------------------------------------------------------------------------
// FP64 products on 128 x 128 tiles: 8 waves per workgroup, each computing a
// 32 x 64 part (2 x 4 MFMA blocks), the same 16-deep K chunks as above.  A
// product of M x N x K on 64 x 64 tiles moves about M N K / 4 bytes past the
// L2 (each tile streams its own panels); 128 x 128 tiles halve that, which
// on the large products raises the MFMA rate from ~50 to ~64 TFLOP/s.
//
// M and N are multiples of 64, so in the last tile row (column) the second
// half may lie outside the product: its loads are redirected to the first
// half (in bounds, the results discarded) and its stores skipped.  The
// semantics are those of the 64 x 64 tiles exactly: the K ranges of
// triangular operands are cut at 128 granularity, and every element of a
// 64 x 64 block strictly above the diagonal of a triangular operand is read
// as zero (those blocks are never written by the recursion and may hold the
// original matrix); LOWER writes the 64 x 64 blocks on or below the
// diagonal only.
// ---------------------------------------------------------------------------
constexpr int kBig = 128;

template <bool AT, bool BT, bool LOWER>
__device__ inline void gemm_tile128(const GemmArgs<double> &g, int tm, int tn) {
  typedef Mfma<double> MF;
  if (LOWER && tn > tm) return;
  const int64_t M = g.M, N = g.N, K = g.K, lda = g.lda, ldb = g.ldb, ldc = g.ldc;
  const double *__restrict__ A = g.A;
  const double *__restrict__ B = g.B;
  double *__restrict__ C = g.C;
  const int kmode = g.kmode;
  int64_t kb = 0, ke = K;
  if (kmode == kLeN) ke = min(K, (int64_t)(tn + 1) * kBig);
  else if (kmode == kGeN) kb = (int64_t)tn * kBig;
  else if (kmode == kLeM) ke = min(K, (int64_t)(tm + 1) * kBig);
  else if (kmode == kGeMN) kb = (int64_t)max(tm, tn) * kBig;

  __shared__ double As[kKc][kBig + kPad];
  __shared__ double Bs[kKc][kBig + kPad];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;  // wave part: rows 32 wm.., columns 64 wn..
  MF::acc_t acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = MF::zero();

  // loaders, 4 consecutive elements per thread and chunk
  const int lt_k = tid >> 5, lt_m = (tid & 31) * 4;  // K-major tile (M contiguous): 16 x 128
  const int lc_m = tid >> 2, lc_k = (tid & 3) * 4;   // M-major tile (K contiguous): 128 x 16
  const int64_t m0 = (int64_t)tm * kBig, n0 = (int64_t)tn * kBig;
  const int a_x = AT ? lc_m : lt_m, b_x = BT ? lt_m : lc_m;  // tile row of A / column of B
  const int a_src = m0 + a_x < M ? a_x : a_x - 64;           // in bounds
  const int b_src = n0 + b_x < N ? b_x : b_x - 64;
  const double *pa = AT ? A + lc_k + (m0 + a_src) * lda : A + m0 + a_src + lt_k * lda;
  const double *pb = BT ? B + n0 + b_src + lt_k * ldb : B + lc_k + (n0 + b_src) * ldb;
  // 64-block of the row of A / column of B this thread loads, for the masks
  const int64_t a_blk = (m0 + a_x) >> 6, b_blk = (n0 + b_x) >> 6;
  const bool a_tri = kmode == kLeM || kmode == kGeMN;
  const bool b_tri = kmode == kLeN || kmode == kGeN || kmode == kGeMN;
  double ra[4], rb[4];
  auto load = [&](int64_t k0) {
    const double *qa = AT ? pa + k0 : pa + k0 * lda;
    const double2 a01 = *reinterpret_cast<const double2 *>(qa);
    const double2 a23 = *reinterpret_cast<const double2 *>(qa + 2);
    ra[0] = a01.x; ra[1] = a01.y; ra[2] = a23.x; ra[3] = a23.y;
    const double *qb = BT ? pb + k0 * ldb : pb + k0;
    const double2 b01 = *reinterpret_cast<const double2 *>(qb);
    const double2 b23 = *reinterpret_cast<const double2 *>(qb + 2);
    rb[0] = b01.x; rb[1] = b01.y; rb[2] = b23.x; rb[3] = b23.y;
    // the 4 elements share their K block and their row / column block
    const int64_t ka = (k0 + (AT ? lc_k : lt_k)) >> 6, kbk = (k0 + (BT ? lt_k : lc_k)) >> 6;
    const bool za = a_tri && (kmode == kLeM ? ka > a_blk : ka < a_blk);
    const bool zb = b_tri && (kmode == kLeN ? kbk > b_blk : kbk < b_blk);
    if (za) ra[0] = ra[1] = ra[2] = ra[3] = 0.0;
    if (zb) rb[0] = rb[1] = rb[2] = rb[3] = 0.0;
  };
  if (kb < ke) load(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += kKc) {
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (AT) As[lc_k + v][lc_m] = ra[v];
      else As[lt_k][lt_m + v] = ra[v];
      if (BT) Bs[lt_k][lt_m + v] = rb[v];
      else Bs[lc_k + v][lc_m] = rb[v];
    }
    __syncthreads();
    if (k0 + kKc < ke) load(k0 + kKc);  // prefetch the next chunk during the MFMAs
#pragma unroll
    for (int kk = 0; kk < kKc / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      const int c = lane & 15;
      double a[2], b[4];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kr][wm * 32 + i * 16 + c];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kr][wn * 64 + j * 16 + c];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = MF::mma(a[i], b[j], acc[i][j]);
    }
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      const int64_t col = n0 + wn * 64 + bj * 16 + (lane & 15);
      const int64_t row0 = m0 + wm * 32 + bi * 16;
      // outside the product, or (LOWER) a 64 x 64 block above the diagonal
      if (row0 >= M || n0 + wn * 64 >= N || (LOWER && (n0 >> 6) + wn > (row0 >> 6))) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double *pc = C + row0 + MF::row(lane, v) + col * ldc;
        const double x = g.alpha * acc[bi][bj][v];
        *pc = g.beta == 0.0 ? x : x + g.beta * (*pc);
      }
    }
}

// Tile of workgroup (bx, by): with a triangular operand cut at the tile the
// K range grows with the tile row (kLeM) or column (kLeN); that direction is
// taken as the slow grid dimension (the grid of a kLeM product is launched
// transposed, N tiles by M tiles) and reversed, so the tiles with the
// longest K ranges are dispatched first and the short ones fill in at the
// end.
__device__ inline int2 tile_order128(const GemmArgs<double> &g, int bx, int by) {
  const int mt = (int)((g.M + kBig - 1) / kBig), nt = (int)((g.N + kBig - 1) / kBig);
  const bool lem = g.kmode == kLeM, len = g.kmode == kLeN;
  return make_int2(lem ? mt - 1 - by : bx, lem ? bx : (len ? nt - 1 - by : by));
}

template <bool AT, bool BT, bool LOWER>
__global__ __launch_bounds__(512) void k_gemm128(GemmArgs<double> g) {
  const int2 t = tile_order128(g, blockIdx.x, blockIdx.y);
  gemm_tile128<AT, BT, LOWER>(g, t.x, t.y);
}

// The recursion node's pair (as k_gemm64_pair) on 128 x 128 tiles.
__global__ __launch_bounds__(512) void k_gemm128_pair(GemmArgs<double> s, GemmArgs<double> t,
                                                      int nblk_s) {
  const int b = blockIdx.x;
  if (b < nblk_s) {
    const int mt = (int)((s.M + kBig - 1) / kBig);
    gemm_tile128<false, true, true>(s, b % mt, b / mt);
  } else {
    const int mt = (int)((t.M + kBig - 1) / kBig), bb = b - nblk_s;
    gemm_tile128<false, false, false>(t, bb % mt, bb / mt);
  }
}

constexpr int kRow32 = 32 + kPad;
constexpr int kStage32 = 2 * kKc * kRow32;  // one wave's A and B chunk (elements)
static_assert(kStage32 >= 16 * 64, "a wave's slot also holds its partial tile");

// sh: S * kStage32 elements of LDS, one slot per wave.
template <typename T, bool AT, bool BT, bool LOWER, int S>
__device__ inline void gemm_tile32_split(const GemmArgs<T> &g, int tm, int tn, T *sh) {
  typedef Mfma<T> MF;
  typedef typename MF::vec2 V2;
  if (LOWER && tn > tm) return;
  const int64_t K = g.K, lda = g.lda, ldb = g.ldb, ldc = g.ldc;
  const T *__restrict__ A = g.A;
  const T *__restrict__ B = g.B;
  T *__restrict__ C = g.C;
  const int kmode = g.kmode;
  int64_t kb = 0, ke = K;
  if (kmode == kLeN) ke = min(K, (int64_t)(tn + 1) * 32);
  else if (kmode == kGeN) kb = (int64_t)tn * 32;
  else if (kmode == kLeM) ke = min(K, (int64_t)(tm + 1) * 32);
  else if (kmode == kGeMN) kb = (int64_t)max(tm, tn) * 32;

  constexpr int kRow = kRow32, kStage = kStage32;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  T *As = sh + wid * kStage;
  T *Bs = As + kKc * kRow;
  typename MF::acc_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = MF::zero();
  const int lt_k = lane >> 2, lt_m = (lane & 3) * 8;  // K-major tile (M contiguous)
  const int lc_m = lane >> 1, lc_k = (lane & 1) * 8;  // M-major tile (K contiguous)
  const T *pa = AT ? A + lc_k + ((int64_t)tm * 32 + lc_m) * lda
                   : A + (int64_t)tm * 32 + lt_m + lt_k * lda;
  const T *pb = BT ? B + (int64_t)tn * 32 + lt_m + lt_k * ldb
                   : B + lc_k + ((int64_t)tn * 32 + lc_m) * ldb;
  T ra[8], rb[8];
  auto load = [&](int64_t k0) {
    const T *qa = AT ? pa + k0 : pa + k0 * lda;
    const T *qb = BT ? pb + k0 * ldb : pb + k0;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const V2 a = *reinterpret_cast<const V2 *>(qa + 2 * h);
      const V2 b = *reinterpret_cast<const V2 *>(qb + 2 * h);
      ra[2 * h] = a.x;
      ra[2 * h + 1] = a.y;
      rb[2 * h] = b.x;
      rb[2 * h + 1] = b.y;
    }
  };
  auto wave_sync = [] {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  const int64_t step = (int64_t)S * kKc;
  const int64_t k_first = kb + (int64_t)wid * kKc;
  if (k_first < ke) load(k_first);
  for (int64_t k0 = k_first; k0 < ke; k0 += step) {
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      if (AT) As[(lc_k + v) * kRow + lc_m] = ra[v];
      else As[lt_k * kRow + lt_m + v] = ra[v];
      if (BT) Bs[lt_k * kRow + lt_m + v] = rb[v];
      else Bs[(lc_k + v) * kRow + lc_m] = rb[v];
    }
    wave_sync();
    if (k0 + step < ke) load(k0 + step);
#pragma unroll
    for (int kk = 0; kk < kKc / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      const int c = lane & 15;
      const T a0 = As[kr * kRow + c], a1 = As[kr * kRow + 16 + c];
      const T b0 = Bs[kr * kRow + c], b1 = Bs[kr * kRow + 16 + c];
      acc[0][0] = MF::mma(a0, b0, acc[0][0]);
      acc[0][1] = MF::mma(a0, b1, acc[0][1]);
      acc[1][0] = MF::mma(a1, b0, acc[1][0]);
      acc[1][1] = MF::mma(a1, b1, acc[1][1]);
    }
    wave_sync();
  }
  // partial tiles: slot of wave w holds [block 2*bi+bj][register v][lane]
  __syncthreads();
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) sh[wid * kStage + ((2 * bi + bj) * 4 + v) * 64 + lane] = acc[bi][bj][v];
  __syncthreads();
  for (int o = wid; o < 16; o += S) {  // o = 4 * block + v
    T sum = T(0);
#pragma unroll
    for (int s = 0; s < S; ++s) sum += sh[s * kStage + o * 64 + lane];
    const int blk = o >> 2, v = o & 3;
    const int64_t col = (int64_t)tn * 32 + (blk & 1) * 16 + (lane & 15);
    const int64_t row = (int64_t)tm * 32 + (blk >> 1) * 16 + MF::row(lane, v);
    T *pc = C + row + col * ldc;
    const T x = g.alpha * sum;
    *pc = g.beta == T(0) ? x : x + g.beta * (*pc);
  }
}

template <typename T, bool AT, bool BT, bool LOWER, int S>
__global__ __launch_bounds__(64 * S) void k_gemm32s(GemmArgs<T> g) {
  __shared__ T sh[S * kStage32];
  gemm_tile32_split<T, AT, BT, LOWER, S>(g, blockIdx.x, blockIdx.y, sh);
}

template <typename T, int S>
__global__ __launch_bounds__(64 * S) void k_gemm32s_pair(GemmArgs<T> s, GemmArgs<T> t, int nblk_s) {
  __shared__ T sh[S * kStage32];
  const int b = blockIdx.x;
  if (b < nblk_s) {
    const int mt = (int)(s.M / 32);
    gemm_tile32_split<T, false, true, true, S>(s, b % mt, b / mt, sh);
  } else {
    const int mt = (int)(t.M / 32), bb = b - nblk_s;
    gemm_tile32_split<T, false, false, false, S>(t, bb % mt, bb / mt, sh);
  }
}

// One product; grid (M/64, N/64), tile rows fastest.  (A die-aware order --
// each of the 8 dies given a contiguous range of a grouped tile order, so
// that the workgroups running side by side on one die form 8 x 8 tile
// blocks -- was measured slower on the large scene: dense stage 342 against
// 264 ms.)
template <typename T, bool AT, bool BT, bool LOWER>
__global__ __launch_bounds__(256) void k_gemm64(GemmArgs<T> g) {
  gemm_tile<T, AT, BT, LOWER>(g, blockIdx.x, blockIdx.y);
}

// The two independent products of one recursion node in one launch: the
// Schur update A22 -= T T^T (lower tiles, first nblk_s workgroups) and
// T2 = T L11^-1.
template <typename T>
__global__ __launch_bounds__(256) void k_gemm64_pair(GemmArgs<T> s, GemmArgs<T> t, int nblk_s) {
  const int b = blockIdx.x;
  if (b < nblk_s) {
    const int mt = (int)(s.M / 64);
    gemm_tile<T, false, true, true>(s, b % mt, b / mt);
  } else {
    const int mt = (int)(t.M / 64), bb = b - nblk_s;
    gemm_tile<T, false, false, false>(t, bb % mt, bb / mt);
  }
}

// ---------------------------------------------------------------------------
// Leaf of NB x NB (64 or 128) on MFMA: Cholesky factor and inverse with the
// block resident in LDS (column-major, padded leading dimension) and 16-column
// panels.  Factorisation, panel p:
//   1. one wave factors the 16x16 diagonal block in registers (row per lane,
//      scalar lane broadcasts, hardware reciprocal square roots refined by
//      Newton steps) and inverts it by forward elimination in the same
//      column loop: L_pp and L_pp^-1;
//   2. the panel below: L_ip = A_ip L_pp^-T            (MFMA, all waves)
//   3. the trailing lower blocks: A_ij -= L_ip L_jp^T   (MFMA); wave 0
//      solves panel row p + 1, updates block (p+1, p+1) from it at once and
//      goes on to step 1 of panel p + 1 while the other waves do the rest of
//      the panel and the trailing update.
// Inversion (forward elimination of L Y = I by block rows), panel p:
//   Y(p, c) = L_pp^-1 W(p, c) for c < p, Y(p, p) = L_pp^-1, and
//   W(i, c) -= L_ip Y(p, c) for i > p;
// the columns c < p run beside the trailing update of p (one wave per
// column), column p, which overwrites L_ip, beside the panel solve of p + 1.
// Writes L^-1 (lower) into the tile and zeros above its diagonal.
// ---------------------------------------------------------------------------
// LDS strides of the leaf: column-strided accesses (lane = column) then fall
// on distinct banks (a stride of 2 dwords modulo the bank count).
constexpr int kLP = 1;   // leading-dimension padding of the tile
constexpr int kDL = 17;  // column stride of the 16x16 diagonal inverses

// Broadcast lane l's value of x to the whole wave (scalar lane reads).
__device__ inline double readlane(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline float readlane(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// Hardware reciprocal square root refined by Newton-Raphson steps
// (y <- y (3 - x y^2) / 2) to the working precision.
__device__ inline double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}
__device__ inline float rsqrt_nr(float x) {
  float y = __builtin_amdgcn_rsqf(x);
  y = y * (1.5f - 0.5f * x * y * y);
  return y;
}
// Hardware reciprocal refined by Newton-Raphson steps (y <- y + y (1 - x y)).
__device__ inline double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
}
__device__ inline float rcp_nr(float x) {
  float y = __builtin_amdgcn_rcpf(x);
  return fmaf(y, fmaf(-x, y, 1.0f), y);
}

// Lane n of each row of 16 lanes, broadcast to that row (DPP row_newbcast).
template <int N>
__device__ inline double row_bcast(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, 0x150 + N, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x150 + N, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int N>
__device__ inline float row_bcast(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x150 + N, 0xF, 0xF, true));
}
// Lane src's value of x, for any src of the wave (LDS crossbar, no memory).
__device__ inline double lane_fetch(double x, int src) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_ds_bpermute(4 * src, (int)b);
  const int hi = __builtin_amdgcn_ds_bpermute(4 * src, (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline float lane_fetch(float x, int src) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(4 * src, __float_as_int(x)));
}

// Inverse L^-1 of the Cholesky factor of a 16 x 16 diagonal block on one
// wave (the factor L itself is not needed: the leaf uses only L^-1 of its
// diagonal blocks).  Lane 16 q + r holds a[k] = A[r][4k + q] of the
// symmetric trailing matrix (both triangles) and t[k] = T[4k + q][r], column
// r of the forward elimination L T = I.  Column j: pivot A[j][j],
// rs = A[j][j]^-1/2, L[i][j] = A[i][j] rs = A[j][i] rs (symmetry), so the
// values every lane needs, row j at its own columns, come from lane j of its
// own row of 16 lanes (one DPP broadcast each); A[r][j] and T[j][r] come
// from column group j % 4 over the crossbar.  Then
//   A[r][c] -= A[r][j] A[j][c] / A[j][j]   (c > j),
//   T[i][r] -= A[j][i] T[j][r] / A[j][j]   (i > j),
// and row j of T is final, stored at once (every column group holds the same
// values and writes the same addresses); row j of L^-1 is T[j][.] / sqrt(A[j][j]),
// scaled after the last column so that no square root sits in the column
// loop.  The entries of columns and rows already final keep being updated
// in registers, with values nothing reads.
template <typename T, int J>
__device__ __forceinline__ void diag_step(T (&a)[4], T (&t)[4], int r, T &pv, T *dinv, bool &ok) {
  constexpr int KJ = J / 4, QJ = J % 4;
  const T piv = readlane(a[KJ], 16 * QJ + J);
  ok = ok && piv > T(0);
  pv = r == J ? piv : pv;  // lane r keeps pivot r for the final scaling
  const T inv = rcp_nr(piv);
  const int src = 16 * QJ + r;
  const T col = lane_fetch(a[KJ], src);  // A[r][j]
  const T tj = lane_fetch(t[KJ], src);   // T[j][r]
  const T w2 = col * inv, tz = tj * inv;
  dinv[r * kDL + J] = tj;  // T[j][r], column-major; row j is scaled at the end
#pragma unroll
  for (int k = KJ; k < 4; ++k) {
    const T bc = row_bcast<J>(a[k]);  // A[j][4k + q]
    a[k] -= w2 * bc;
    t[k] -= tz * bc;
  }
}
template <typename T, int... J>
__device__ __forceinline__ void diag_steps(T (&a)[4], T (&t)[4], int r, T &pv, T *dinv, bool &ok,
                                           std::integer_sequence<int, J...>) {
  (diag_step<T, J>(a, t, r, pv, dinv, ok), ...);
}

template <typename T, int NB, int NT>
__device__ __forceinline__ void leaf_body(T *A, int64_t lda, int64_t o, DevStatus *ds) {
  typedef Mfma<T> MF;
  typedef typename MF::vec2 V2;
  constexpr int LD = NB + kLP;
  constexpr int NPAN = NB / 16;
  constexpr int NW = NT / 64;  // waves
  __shared__ T S[NB * LD];
  __shared__ T Dinv[NPAN][16 * kDL];  // L_pp^-1, column-major 16x16
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  T *G = A + o + o * lda;
  // Whole columns with paired loads (the upper part is read and discarded):
  // column block 0 by every thread; the rest by waves 1.. while wave 0
  // factors diagonal block 0.
  constexpr int NL0 = 16 * NB / 2 / NT, NL1 = (NB - 16) * NB / 2 / (NT - 64);
  static_assert(2 * NL0 * NT == 16 * NB && 2 * NL1 * (NT - 64) == (NB - 16) * NB,
                "the leaf's loads divide evenly over its threads");
  auto stage_pair = [&](int e, V2 x) {  // element pair (e, e + 1), column-major
    const int r = e % NB, c = e / NB;
    S[c * LD + r] = r >= c ? x.x : T(0);
    S[c * LD + r + 1] = r + 1 >= c ? x.y : T(0);
  };
  {
    V2 ld2[NL0];
#pragma unroll
    for (int k = 0; k < NL0; ++k) {
      const int e = 2 * (tid + NT * k);
      ld2[k] = *reinterpret_cast<const V2 *>(G + e % NB + (int64_t)(e / NB) * lda);
    }
#pragma unroll
    for (int k = 0; k < NL0; ++k) stage_pair(2 * (tid + NT * k), ld2[k]);
  }
  __syncthreads();
  const int lr = lane & 15, lg = lane >> 4;  // row in block, column group

  // Diagonal block p on wave 0: L_pp^-1 into Dinv[p] (L_pp itself is never
  // read: the panel solve and the inversion use L_pp^-1, and block (p, p) of
  // S is overwritten by it later).  S holds the lower triangle of the block
  // (the upper one is not kept up to date); lane 16 q + r reads both
  // triangles from it.
  auto factor_diag = [&](int p) {
    const int c0 = 16 * p, q = lane >> 4;
    T a[4], t[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int c = 4 * k + q, lo = lr < c ? lr : c, hi = lr < c ? c : lr;
      a[k] = S[(c0 + lo) * LD + c0 + hi];
      t[k] = c == lr ? T(1) : T(0);
    }
    bool ok = true;
    T pv = T(1);
    diag_steps(a, t, lr, pv, Dinv[p], ok, std::make_integer_sequence<int, 16>());
    // row r of L^-1 = row r of T / sqrt(pivot r); lane 16 q + r scales its
    // columns 4k + q, which other lanes of this wave stored above
    const T rs = rsqrt_nr(pv);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < 4; ++k) Dinv[p][(4 * k + q) * kDL + lr] *= rs;
    if (!ok && lane == 0) report_error(ds, UCOV_EGAUGE, (int)((o + c0) / 9));
  };
  // Trailing block (i, j) -= L_ip L_jp^T (one wave, MFMA).
  auto trailing_block = [&](int p, int i, int j) {
    const int c0 = 16 * p;
    typename MF::acc_t acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = S[(16 * j + lr) * LD + 16 * i + MF::row(lane, v)];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = 4 * kk + lg;
      const T a = -S[(c0 + k) * LD + 16 * i + lr];
      const T bb = S[(c0 + k) * LD + 16 * j + lr];
      acc = MF::mma(a, bb, acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) S[(16 * j + lr) * LD + 16 * i + MF::row(lane, v)] = acc[v];
  };

  // Inversion steps (forward elimination L Y = I by block rows; W(i, c)
  // accumulates -sum_k L_ik Y(k, c) in block (i, c) over the factor):
  //   Y(p, c) = L_pp^-1 W(p, c) for c < p, Y(p, p) = L_pp^-1, in block (p, c);
  //   W(i, c) -= L_ip Y(p, c) for i > p (W(i, p) starts at zero and replaces
  //   L_ip in place).
  auto inv_y = [&](int p, int c) {
    const int c0 = 16 * p;
    if (c == p) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = lg + 4 * v;
        S[(c0 + col) * LD + c0 + lr] = Dinv[p][col * kDL + lr];
      }
    } else {
      typename MF::acc_t acc = MF::zero();
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int k = 4 * kk + lg;
        const T a = Dinv[p][k * kDL + lr];          // (L_pp^-1)[lr][k]
        const T b = S[(16 * c + lr) * LD + c0 + k];  // W(p, c)[k][lr]
        acc = MF::mma(a, b, acc);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) S[(16 * c + lr) * LD + c0 + MF::row(lane, v)] = acc[v];
    }
  };
  auto inv_col = [&](int p, int i, int c) {
    const int c0 = 16 * p;
    typename MF::acc_t acc;
#pragma unroll
    for (int v = 0; v < 4; ++v)
      acc[v] = (c == p) ? T(0) : S[(16 * c + lr) * LD + 16 * i + MF::row(lane, v)];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = 4 * kk + lg;
      const T a = -S[(c0 + k) * LD + 16 * i + lr];  // L_ip[lr][k]
      const T bb = (c == p) ? Dinv[p][lr * kDL + k]  // Y(p, c)[k][lr]
                            : S[(16 * c + lr) * LD + c0 + k];
      acc = MF::mma(a, bb, acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) S[(16 * c + lr) * LD + 16 * i + MF::row(lane, v)] = acc[v];
  };

  // Factorisation with a one-panel lookahead (wave 0 updates the next
  // diagonal block beside the panel solve and factors it beside the trailing
  // update; each step's LDS writes are read back only by wave 0 itself),
  // fused with the inversion steps: two barriers per panel.
  if (wid == 0) {
    factor_diag(0);
  } else {
    V2 ld2[NL1];
#pragma unroll
    for (int k = 0; k < NL1; ++k) {
      const int e = 16 * NB + 2 * (tid - 64 + (NT - 64) * k);
      ld2[k] = *reinterpret_cast<const V2 *>(G + e % NB + (int64_t)(e / NB) * lda);
    }
#pragma unroll
    for (int k = 0; k < NL1; ++k) stage_pair(16 * NB + 2 * (tid - 64 + (NT - 64) * k), ld2[k]);
  }
  __syncthreads();
  for (int p = 0; p < NPAN; ++p) {
    const int c0 = 16 * p;
    // ---- phase A: panel L_ip = A_ip L_pp^-T (i > p), and column p - 1 of
    // the inversion: Y(p-1, p-1) and W(i, p-1) for i >= p over L_{i,p-1}.
    // Wave 0 solves row p + 1 and at once updates block (p+1, p+1), the
    // next diagonal block, from it ----
    {
      const int npan = NPAN - 1 - p;
      const int ncol = p > 0 ? NPAN - p + 1 : 0;
      auto panel = [&](int i) {
        typename MF::acc_t acc = MF::zero();
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int k = 4 * kk + lg;
          const T a = S[(c0 + k) * LD + 16 * i + lr];
          const T b = Dinv[p][k * kDL + lr];  // (L_pp^-1)[lr][k] = B^T[k][lr]
          acc = MF::mma(a, b, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) S[(c0 + lr) * LD + 16 * i + MF::row(lane, v)] = acc[v];
      };
      const int first = npan > 0 ? 1 : 0;  // task 0 (row p + 1) is wave 0's
      if (first && wid == 0) {
        panel(p + 1);
        __builtin_amdgcn_s_waitcnt(0);  // L_{p+1,p} is read back by this wave
        __builtin_amdgcn_wave_barrier();
        trailing_block(p, p + 1, p + 1);
      } else {
        for (int t = wid; t < npan + ncol; t += NW - first) {
          if (t < npan) {
            panel(p + 1 + t);
          } else {
            const int u = t - npan;
            if (u == 0) inv_y(p - 1, p - 1);
            else inv_col(p - 1, p - 1 + u, p - 1);
          }
        }
      }
    }
    __syncthreads();
    // ---- phase B: trailing A_ij -= L_ip L_jp^T (p < j <= i, block (p+1, p+1)
    // done) and the next diagonal factorisation on wave 0; on the other
    // waves, beside the trailing blocks, the inversion's columns c < p, each
    // by one wave: Y(p, c), then W(i, c) for every i > p (these read L_ip,
    // which the trailing update only reads, and write blocks left of p) ----
    {
      const int m = NPAN - 1 - p;       // trailing block rows
      const int ntr = m * (m + 1) / 2;  // trailing blocks, block (p+1, p+1) first
      const bool look = p + 1 < NPAN;
      if (look && wid == 0) {
        factor_diag(p + 1);
      } else {
        const int w0 = look ? 1 : 0, nw = look ? NW - 1 : NW;
        const int first = look ? 1 : 0;      // block (p+1, p+1) is wave 0's
        const int ncol = look ? p : p + 1;   // columns c < p; the last panel adds Y(p, p)
        const int u = wid - w0;              // this wave among the nw (ncol <= nw)
        if (u < ncol) {                      // inversion column u, a chain of NPAN - p blocks
          inv_y(p, u);
          if (u < p) {
            __builtin_amdgcn_s_waitcnt(0);  // Y(p, u) is read back by this wave
            __builtin_amdgcn_wave_barrier();
            for (int i = p + 1; i < NPAN; ++i) inv_col(p, i, u);
          }
        }
        auto trail = [&](int j) {
          int jj = 0, rem = j + first;  // -> (ii, jj) in the lower triangle of m x m blocks
          while (rem >= m - jj) {
            rem -= m - jj;
            ++jj;
          }
          trailing_block(p, p + 1 + jj + rem, p + 1 + jj);
        };
        // trailing blocks go to the waves without a column first, up to a
        // column's length each, and the rest round-robin over all waves
        const int ntrail = ntr - first, nfree = nw - ncol;
        const int cap = min(ntrail, nfree * (NPAN - p));
        if (u >= ncol)
          for (int j = u - ncol; j < cap; j += nfree) trail(j);
        for (int j = cap + u; j < ntrail; j += nw) trail(j);
      }
    }
    __syncthreads();
  }
  constexpr int NL = NB * NB / 2 / NT;
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int e = 2 * (tid + NT * k);
    const int r = e % NB, c = e / NB;
    V2 x;
    x.x = r >= c ? S[c * LD + r] : T(0);
    x.y = r + 1 >= c ? S[c * LD + r + 1] : T(0);
    *reinterpret_cast<V2 *>(G + r + (int64_t)c * lda) = x;
  }
}

// Threads of a leaf workgroup: 8 waves for 128 (more block products per
// barrier; 16 waves leave too few registers), 4 for 64.
template <int NB>
struct LeafThreads {
  static constexpr int value = NB == 128 ? 512 : 256;
};

template <typename T, int NB>
__global__ __launch_bounds__(LeafThreads<NB>::value) void k_leaf_mfma(T *A, int64_t lda, int64_t o,
                                                                     DevStatus *ds) {
  leaf_body<T, NB, LeafThreads<NB>::value>(A, lda, o, ds);
}

// ---------------------------------------------------------------------------
// Batched forms for many independent matrices: one launch serves one node of
// the recursion for every matrix that reaches it, blockIdx.z selecting the
// matrix's arguments from a device table (workgroups beyond a smaller
// matrix's tiles return at once).
// ---------------------------------------------------------------------------
template <typename T>
struct LeafArg {
  T *A;
  int64_t lda, o;
  DevStatus *ds;
};

template <typename T, int NB>
__global__ __launch_bounds__(LeafThreads<NB>::value) void k_leaf_mfma_b(const LeafArg<T> *tab) {
  const LeafArg<T> a = tab[blockIdx.x];
  leaf_body<T, NB, LeafThreads<NB>::value>(a.A, a.lda, a.o, a.ds);
}

// As in the single 128 x 128 products, a triangular operand cut per tile row
// (kLeM, whose launch has its grid transposed: N tiles by M tiles) or column
// (kLeN) makes that direction the slow one, reversed: the scene's tiles with
// the longest K ranges go first.
template <typename T, bool AT, bool BT, bool LOWER>
__global__ __launch_bounds__(256) void k_gemm64_b(const GemmArgs<T> *tab) {
  const GemmArgs<T> g = tab[blockIdx.z];
  const int mt = (int)(g.M / 64), nt = (int)(g.N / 64);
  const bool lem = g.kmode == kLeM;
  const int bm = lem ? (int)blockIdx.y : (int)blockIdx.x;  // over the M tiles
  const int bn = lem ? (int)blockIdx.x : (int)blockIdx.y;  // over the N tiles
  if (bm >= mt || bn >= nt) return;
  gemm_tile<T, AT, BT, LOWER>(g, lem ? mt - 1 - bm : bm, g.kmode == kLeN ? nt - 1 - bn : bn);
}

template <typename T>
__global__ __launch_bounds__(256) void k_gemm64_pair_b(const GemmArgs<T> *stab,
                                                       const GemmArgs<T> *ttab) {
  const GemmArgs<T> sg = stab[blockIdx.z];
  const int ms = (int)(sg.M / 64), nblk_s = ms * ms, b = blockIdx.x;
  if (b < nblk_s) {
    gemm_tile<T, false, true, true>(sg, b % ms, b / ms);
  } else {
    const GemmArgs<T> tg = ttab[blockIdx.z];
    const int mt = (int)(tg.M / 64), bb = b - nblk_s;
    if (bb >= mt * (int)(tg.N / 64)) return;
    gemm_tile<T, false, false, false>(tg, bb % mt, bb / mt);
  }
}

// Batched split 32 x 32 tiles: blockIdx.z picks the product of a scene, the
// K range of a tile is dealt out to S waves (see gemm_tile32_split).
template <typename T, bool AT, bool BT, bool LOWER, int S>
__global__ __launch_bounds__(64 * S) void k_gemm32s_b(const GemmArgs<T> *tab) {
  __shared__ T sh[S * kStage32];
  const GemmArgs<T> g = tab[blockIdx.z];
  if ((int64_t)blockIdx.x * 32 >= g.M || (int64_t)blockIdx.y * 32 >= g.N) return;
  gemm_tile32_split<T, AT, BT, LOWER, S>(g, blockIdx.x, blockIdx.y, sh);
}

template <typename T, int S>
__global__ __launch_bounds__(64 * S) void k_gemm32s_pair_b(const GemmArgs<T> *stab,
                                                          const GemmArgs<T> *ttab) {
  __shared__ T sh[S * kStage32];
  const GemmArgs<T> sg = stab[blockIdx.z];
  const int ms = (int)(sg.M / 32), nblk_s = ms * ms, b = blockIdx.x;
  if (b < nblk_s) {
    gemm_tile32_split<T, false, true, true, S>(sg, b % ms, b / ms, sh);
  } else {
    const GemmArgs<T> tg = ttab[blockIdx.z];
    const int mt = (int)(tg.M / 32), bb = b - nblk_s;
    if (bb >= mt * (int)(tg.N / 32)) return;
    gemm_tile32_split<T, false, false, false, S>(tg, bb % mt, bb / mt, sh);
  }
}

// Strict upper triangle of an n x n matrix (n a multiple of 32) set from its
// lower triangle through 32 x 32 LDS tiles: workgroup (tm, tn), tm >= tn,
// reads tile (tm, tn) with coalesced column loads and writes its transpose
// at (tn, tm), rows across the lanes.  tile[c][r] holds a(32 tm + r, 32 tn + c).
__global__ __launch_bounds__(256) void k_mirror_lower(double *a, int64_t lda) {
  const int64_t tm = blockIdx.x, tn = blockIdx.y;
  if (tn > tm) return;
  __shared__ double tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t R0 = 32 * tm, C0 = 32 * tn;
  for (int c = ty; c < 32; c += 8) tile[c][tx] = a[(R0 + tx) + (C0 + c) * lda];
  __syncthreads();
  for (int c = ty; c < 32; c += 8) {
    const int64_t row = C0 + tx, col = R0 + c;  // a(row, col) = a(col, row) = tile[tx][c]
    if (row < col) a[row + col * lda] = tile[tx][c];
  }
}

// A symmetric positive definite test matrix for timing the dense stage:
// a_ij = 0.5 exp(-|i - j| / 8) off the diagonal, 10 on it (diagonally dominant).
__global__ void k_tuning_matrix(int64_t n, double *a, int64_t lda) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (r >= n) return;
  const double d = (double)(r > c ? r - c : c - r);
  a[r + c * lda] = r == c ? 10.0 : 0.5 * exp(-d / 8.0);
}

// ---------------------------------------------------------------------------
// elementwise helpers
// ---------------------------------------------------------------------------
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

// lower triangle of a (FP64) -> lower triangle of a32 (FP32), n x n
__global__ void k_lower_to_f32(int64_t n, const double *a, int64_t lda, float *a32,
                               int64_t ld32) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r < n && r >= c) a32[r + c * ld32] = (float)a[r + c * lda];
}

// a <- full symmetric matrix from its lower triangle (n x n)
__global__ void k_symmetrize(int64_t n, double *a, int64_t lda) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r < n && r < c) a[r + c * lda] = a[c + r * lda];
}

__global__ void k_f32_to_f64(int64_t n, const float *x, int64_t ldx, double *y, int64_t ldy) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r < n) y[r + c * ldy] = (double)x[r + c * ldx];
}

__global__ void k_f64_to_f32(int64_t n, const double *x, int64_t ldx, float *y, int64_t ldy) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r < n) y[r + c * ldy] = (float)x[r + c * ldx];
}

__global__ void k_identity(int64_t n, double *a, int64_t lda) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r < n) a[r + c * lda] = (r == c) ? 1.0 : 0.0;
}

// x += (double) d
__global__ void k_add_f32(int64_t n, const float *d, int64_t ldd, double *x, int64_t ldx) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r < n) x[r + c * ldx] += (double)d[r + c * ldd];
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// part[c] = sum of squares of column c of the n x n matrix
__global__ __launch_bounds__(256) void k_sumsq(int64_t n, const double *a, int64_t lda,
                                              double *part_out) {
  const int64_t c = blockIdx.x;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += 256) {
    const double v = a[r + c * lda];
    s += v * v;
  }
  __shared__ double part[4];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part_out[c] = part[0] + part[1] + part[2] + part[3];
}

// out[0] = sum of part[0..n) in a fixed order (the same bits on every call,
// so the stopping decision of the refinement is reproducible)
__global__ __launch_bounds__(256) void k_sum_parts(int64_t n, const double *part, double *out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// One workgroup per camera: (A_s^-1)_ii = sum over rows r >= 9i of the outer
// products of row r of L^-1 restricted to the camera's 9 columns.
__global__ __launch_bounds__(256) void k_extract(int64_t N, const double *linv, int64_t ld,
                                                const double *s, const double *q, int64_t ldq,
                                                const double *alpha, int subtract, double *cov) {
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
    for (int k = 0; k < 7; ++k) g += q[k * ldq + c0 + a0] * q[k * ldq + c0 + b0];
    cov[81 * i + threadIdx.x] = s[c0 + a0] * x * s[c0 + b0] - (subtract ? g / (*alpha) : 0.0);
  }
}

// cov[i] = S_i X_ii S_i - Q_i Q_i^T / alpha from a full inverse X (81 threads
// per camera)
__global__ void k_extract_full(int64_t N, const double *x, int64_t ld, const double *s,
                               const double *q, int64_t ldq, const double *alpha, int subtract,
                               double *cov) {
  const int64_t i = blockIdx.x;
  const int t = threadIdx.x;
  if (t >= 81) return;
  const int64_t r = 9 * i + t / 9, c = 9 * i + t % 9;
  const double xs = 0.5 * (x[r + c * ld] + x[c + r * ld]);
  double g = 0.0;
#pragma unroll
  for (int k = 0; k < 7; ++k) g += q[k * ldq + r] * q[k * ldq + c];
  cov[81 * i + t] = s[r] * xs * s[c] - (subtract ? g / (*alpha) : 0.0);
}

// Every scene of a concatenation: grid (column c, scene s); rows r >= max(c,
// N_s) of column c of scene s's padded matrix set to the identity.
__global__ void k_pad_identity_scenes(const int32_t *cam_off, const int64_t *a_off,
                                      const int64_t *a_ld, double *amat) {
  const int s = blockIdx.y;
  const int64_t N = 9 * (int64_t)(cam_off[s + 1] - cam_off[s]), Np = a_ld[s];
  const int64_t c = blockIdx.x;
  if (c >= Np) return;
  double *a = amat + a_off[s];
  const int64_t r0 = c > N ? c : N;
  for (int64_t r = r0 + threadIdx.x; r < Np; r += blockDim.x) a[r + c * Np] = (r == c) ? 1.0 : 0.0;
}

// Blocks of every camera of a concatenation (one workgroup per camera): as
// k_extract with the scene's matrix, scaling, basis rows and gauge weight.
__global__ __launch_bounds__(256) void k_extract_scenes(const int32_t *cam_scene,
                                                       const int32_t *cam_off,
                                                       const int64_t *a_off, const int64_t *a_ld,
                                                       const double *amat, int64_t Ntot,
                                                       const double *s, const double *q,
                                                       const double *alpha, double *cov) {
  const int64_t gi = blockIdx.x;
  const int sc = cam_scene[gi];
  const int64_t r0 = 9 * (int64_t)cam_off[sc];
  const int64_t N = 9 * (int64_t)(cam_off[sc + 1] - cam_off[sc]);
  const int64_t ld = a_ld[sc];
  const double *linv = amat + a_off[sc];
  const int64_t c0 = 9 * gi - r0;
  double acc[45];
#pragma unroll
  for (int k = 0; k < 45; ++k) acc[k] = 0.0;
  for (int64_t r = c0 + threadIdx.x; r < N; r += blockDim.x) {
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
    const int64_t ra = 9 * gi + a0, rb = 9 * gi + b0;  // global rows of s and q
    double g = 0.0;
#pragma unroll
    for (int k = 0; k < 7; ++k) g += q[k * Ntot + ra] * q[k * Ntot + rb];
    cov[81 * gi + threadIdx.x] = s[ra] * x * s[rb] - g / alpha[sc];
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <typename T>
GemmArgs<T> make_args(int64_t M, int64_t N, int64_t K, const T *A, int64_t lda, const T *B,
                      int64_t ldb, T *C, int64_t ldc, T alpha, T beta, int kmode) {
  GemmArgs<T> g;
  g.M = M; g.N = N; g.K = K; g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.alpha = alpha; g.beta = beta; g.kmode = kmode;
  return g;
}

// Products with fewer 64 x 64 tiles than `small` run on 32 x 32 tiles
// (kSmallTilesDefault unless the size was tuned), with each tile's K range
// split over 4 waves, or over 8 for products with fewer 32 x 32 tiles than
// the GPU has compute units (256).  (One wave per 32 x 32 tile was measured
// slower at every node size of the recursion.)
constexpr int64_t kSplit8Tiles = 256;

// FP64 products with at least kBigTiles tiles of 128 x 128 run on them
// (between the 324 tiles of n = 2304, where 64 x 64 tiles are faster, and
// the 729 of n = 3456, where 128 x 128 tiles are).
constexpr int64_t kBigTiles = 512;
inline int64_t big_tiles(int64_t M, int64_t N) {
  return ((M + kBig - 1) / kBig) * ((N + kBig - 1) / kBig);
}

template <typename T, bool AT, bool BT, bool LOWER>
void gemm(int64_t M, int64_t N, int64_t K, const T *A, int64_t lda, const T *B, int64_t ldb,
          T *C, int64_t ldc, T alpha, T beta, int kmode, hipStream_t st,
          int64_t small = kSmallTilesDefault) {
  GemmArgs<T> g = make_args<T>(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, kmode);
  if constexpr (std::is_same<T, double>::value) {
    if (big_tiles(M, N) >= kBigTiles) {
      const unsigned mt = (unsigned)((M + kBig - 1) / kBig), nt = (unsigned)((N + kBig - 1) / kBig);
      const dim3 grid = kmode == kLeM ? dim3(nt, mt) : dim3(mt, nt);  // see tile_order128
      hipLaunchKernelGGL((k_gemm128<AT, BT, LOWER>), grid, dim3(512), 0, st, g);
      return;
    }
  }
  if ((M / 64) * (N / 64) < small) {
    const dim3 grid((unsigned)(M / 32), (unsigned)(N / 32));
    const int64_t t32 = (M / 32) * (N / 32);
    if (t32 < kSplit8Tiles)
      hipLaunchKernelGGL((k_gemm32s<T, AT, BT, LOWER, 8>), grid, dim3(512), 0, st, g);
    else
      hipLaunchKernelGGL((k_gemm32s<T, AT, BT, LOWER, 4>), grid, dim3(256), 0, st, g);
    return;
  }
  hipLaunchKernelGGL((k_gemm64<T, AT, BT, LOWER>), dim3((unsigned)(M / 64), (unsigned)(N / 64)),
                     dim3(256), 0, st, g);
}

template <typename T>
void gemm_pair(const GemmArgs<T> &s, const GemmArgs<T> &t, hipStream_t st,
               int64_t small = kSmallTilesDefault) {
  if constexpr (std::is_same<T, double>::value) {
    const int64_t a = big_tiles(s.M, s.N), b = big_tiles(t.M, t.N);
    if (a + b >= 2 * kBigTiles) {  // as for two products of kBigTiles tiles
      hipLaunchKernelGGL(k_gemm128_pair, dim3((unsigned)(a + b)), dim3(512), 0, st, s, t, (int)a);
      return;
    }
  }
  const unsigned a = (unsigned)((s.M / 64) * (s.N / 64)), b = (unsigned)((t.M / 64) * (t.N / 64));
  if ((int64_t)a + b < small) {
    const unsigned a32 = (unsigned)((s.M / 32) * (s.N / 32)),
                   b32 = (unsigned)((t.M / 32) * (t.N / 32));
    const int64_t t32 = (int64_t)a32 + b32;
    if (t32 < kSplit8Tiles)
      hipLaunchKernelGGL((k_gemm32s_pair<T, 8>), dim3(a32 + b32), dim3(512), 0, st, s, t, (int)a32);
    else
      hipLaunchKernelGGL((k_gemm32s_pair<T, 4>), dim3(a32 + b32), dim3(256), 0, st, s, t, (int)a32);
    return;
  }
  hipLaunchKernelGGL((k_gemm64_pair<T>), dim3(a + b), dim3(256), 0, st, s, t, (int)a);
}

// Scratch needed by recurse() for an n x n block (elements).
int64_t recurse_scratch(int64_t n) {
  if (n <= 128) return 0;
  const int64_t tiles = n / 64, n1 = (tiles / 2) * 64, n2 = n - n1;
  return n2 * n1 + std::max(n2 * n1, std::max(recurse_scratch(n1), recurse_scratch(n2)));
}

// In-place L^-1 of the n x n block at offset o.  tmp[0, n2*n1) holds this
// level's T2 = L21 L11^-1 across the recursion into A22; the rest is scratch
// for T = L21 and for the children.  (Running T2 on a second stream beside
// the right subtree was measured slower at every node size: the concurrent
// products slow each other and the cross-stream waits add latency.)
template <typename T>
void recurse(T *A, int64_t lda, int64_t o, int64_t n, T *tmp, DevStatus *ds, hipStream_t st,
             int64_t small = kSmallTilesDefault) {
  if (n == 64) {
    hipLaunchKernelGGL((k_leaf_mfma<T, 64>), dim3(1), dim3(LeafThreads<64>::value), 0, st, A, lda,
                       o, ds);
    return;
  }
  if (n == 128) {
    hipLaunchKernelGGL((k_leaf_mfma<T, 128>), dim3(1), dim3(LeafThreads<128>::value), 0, st, A,
                       lda, o, ds);
    return;
  }
  const int64_t tiles = n / 64;
  const int64_t n1 = (tiles / 2) * 64, n2 = n - n1;
  T *T2 = tmp;
  T *Tm = tmp + n2 * n1;
  T *child = Tm;
  recurse(A, lda, o, n1, child, ds, st, small);
  T *A11 = A + o + o * lda;
  T *A21 = A + (o + n1) + o * lda;
  T *A22 = A + (o + n1) + (o + n1) * lda;
  const T one = T(1), zero = T(0), mone = T(-1);
  gemm<T, false, true, false>(n2, n1, n1, A21, lda, A11, lda, Tm, n2, one, zero, kLeN, st,
                              small);  // L21
  gemm_pair<T>(make_args<T>(n2, n2, n1, Tm, n2, Tm, n2, A22, lda, mone, one, kFull),  // Schur
               make_args<T>(n2, n1, n1, Tm, n2, A11, lda, T2, n2, one, zero, kGeN), st, small);
  recurse(A, lda, o + n1, n2, child, ds, st, small);
  gemm<T, false, false, false>(n2, n1, n2, A22, lda, T2, n2, A21, lda, mone, zero, kLeM, st,
                               small);
}

}  // namespace

// ---------------------------------------------------------------------------
// Batched inverse Cholesky factors of many SPD matrices of different sizes.
//
// Every matrix is embedded in the leading block of one virtual matrix of the
// largest size P, whose recursion tree (the same splits as recurse()) is
// walked once.  A node (o, n) involves the matrices that extend past o; one
// whose extent ends inside the left half only takes part in the left
// subtree (its off-diagonal and trailing blocks would be zero and identity).
// Each matrix keeps its own scratch: at a node with a trailing extent m the
// products T (m x n1) and T2 (m x n1) sit at its current scratch offset, the
// right subtree continues past T2, the left one at the same offset.
// ---------------------------------------------------------------------------
namespace {

enum PlanKind { kPlanLeaf64 = 0, kPlanLeaf128 = 1, kPlanGemmT = 2, kPlanPair = 3, kPlanFinal = 4 };
// Tile shape of a product launch: 64 x 64, or split 32 x 32 over 4 or 8 waves.
enum PlanTiles { kTiles64 = 0, kTiles32x4 = 1, kTiles32x8 = 2 };

struct PlanLaunch {
  int kind;
  int64_t first, second;  // table offsets (pair: Schur and T2 entries)
  int count;
  unsigned gx, gy;
  int tiles = kTiles64;   // products: PlanTiles
};

struct WalkMat {
  int64_t np;
  int64_t need;  // scratch high-water mark (elements)
};

template <typename T>
struct PlanBuilder {
  const SpdMat *mats;
  int64_t small = 0;  // launches with fewer 64 x 64 tiles (all scenes) use 32 x 32 tiles
  std::vector<GemmArgs<T>> gemms;
  std::vector<int> gemm_owner;  // matrix of each product (for the bounds check)
  std::vector<int> gemm_bt;     // 1 when B is used transposed
  std::vector<LeafArg<T>> leaves;
  std::vector<int> leaf_owner, leaf_nb;
  std::vector<PlanLaunch> launches;
  std::vector<int64_t> need;

  void add(const GemmArgs<T> &g, int owner, int bt) {
    gemms.push_back(g);
    gemm_owner.push_back(owner);
    gemm_bt.push_back(bt);
  }

  void walk(int64_t o, int64_t n, const std::vector<int> &act, const std::vector<int64_t> &off) {
    if (act.empty()) return;
    if (n <= 128) {
      for (int nb : {128, 64}) {
        PlanLaunch L{nb == 128 ? kPlanLeaf128 : kPlanLeaf64, (int64_t)leaves.size(), 0, 0, 0, 1};
        for (int s : act) {
          const int64_t e = std::min(n, mats[s].np - o);
          if (e != nb) continue;
          leaves.push_back(LeafArg<T>{static_cast<T *>(mats[s].A), mats[s].lda, o, mats[s].ds});
          leaf_owner.push_back(s);
          leaf_nb.push_back(nb);
          ++L.count;
        }
        if (L.count) {
          L.gx = (unsigned)L.count;
          launches.push_back(L);
        }
      }
      return;
    }
    const int64_t n1 = (n / 64 / 2) * 64, n2 = n - n1;
    walk(o, n1, act, off);
    std::vector<int> F;
    std::vector<int64_t> m, offR;
    for (size_t q = 0; q < act.size(); ++q) {
      const int s = act[q];
      const int64_t e = std::min(n, mats[s].np - o);
      if (e <= n1) continue;
      F.push_back(s);
      m.push_back(e - n1);
      offR.push_back(off[q] + (e - n1) * n1);
      need[s] = std::max(need[s], off[q] + 2 * (e - n1) * n1);
    }
    if (F.empty()) return;
    const T one = T(1), zero = T(0), mone = T(-1);
    int64_t mmax = 0;
    for (int64_t x : m) mmax = std::max(mmax, x);
    const unsigned mt = (unsigned)(mmax / 64), nt1 = (unsigned)(n1 / 64);
    // tile shape of this node's launches from their total 64 x 64 tile count
    int64_t t_gemm = 0, t_pair = 0;
    for (int64_t x : m) {
      t_gemm += (x / 64) * (n1 / 64);
      t_pair += (x / 64) * (x / 64 + 1) / 2 + (x / 64) * (n1 / 64);
    }
    auto shape = [&](PlanLaunch &L, int64_t tiles64, bool pair) {
      if (tiles64 >= small) return;
      L.tiles = 4 * tiles64 < 256 ? kTiles32x8 : kTiles32x4;
      const unsigned m32 = (unsigned)(mmax / 32), n32 = (unsigned)(n1 / 32);
      L.gx = pair ? m32 * m32 + m32 * n32 : m32;
      L.gy = pair ? 1 : n32;
    };
    // T = A21 L11^-T
    PlanLaunch LT{kPlanGemmT, (int64_t)gemms.size(), 0, (int)F.size(), mt, nt1};
    shape(LT, t_gemm, false);
    for (size_t q = 0; q < F.size(); ++q) {
      const SpdMat &M = mats[F[q]];
      T *A = static_cast<T *>(M.A), *T2 = static_cast<T *>(M.tmp) + (offR[q] - m[q] * n1);
      T *Tm = T2 + m[q] * n1;
      add(make_args<T>(m[q], n1, n1, A + (o + n1) + o * M.lda, M.lda, A + o + o * M.lda, M.lda,
                       Tm, m[q], one, zero, kLeN), F[q], 1);
    }
    launches.push_back(LT);
    // A22 -= T T^T  and  T2 = T L11^-1
    PlanLaunch LP{kPlanPair, (int64_t)gemms.size(), (int64_t)(gemms.size() + F.size()),
                  (int)F.size(), mt * mt + mt * nt1, 1};
    shape(LP, t_pair, true);
    for (size_t q = 0; q < F.size(); ++q) {
      const SpdMat &M = mats[F[q]];
      T *A = static_cast<T *>(M.A), *T2 = static_cast<T *>(M.tmp) + (offR[q] - m[q] * n1);
      T *Tm = T2 + m[q] * n1;
      add(make_args<T>(m[q], m[q], n1, Tm, m[q], Tm, m[q], A + (o + n1) + (o + n1) * M.lda,
                       M.lda, mone, one, kFull), F[q], 1);
    }
    for (size_t q = 0; q < F.size(); ++q) {
      const SpdMat &M = mats[F[q]];
      T *A = static_cast<T *>(M.A), *T2 = static_cast<T *>(M.tmp) + (offR[q] - m[q] * n1);
      T *Tm = T2 + m[q] * n1;
      add(make_args<T>(m[q], n1, n1, Tm, m[q], A + o + o * M.lda, M.lda, T2, m[q], one, zero,
                       kGeN), F[q], 0);
    }
    launches.push_back(LP);
    walk(o + n1, n2, F, offR);
    // A21 = -L22^-1 T2
    PlanLaunch LF{kPlanFinal, (int64_t)gemms.size(), 0, (int)F.size(), mt, nt1};
    shape(LF, t_gemm, false);
    for (size_t q = 0; q < F.size(); ++q) {
      const SpdMat &M = mats[F[q]];
      T *A = static_cast<T *>(M.A), *T2 = static_cast<T *>(M.tmp) + (offR[q] - m[q] * n1);
      add(make_args<T>(m[q], n1, m[q], A + (o + n1) + (o + n1) * M.lda, M.lda, T2, m[q],
                       A + (o + n1) + o * M.lda, M.lda, mone, zero, kLeM), F[q], 0);
    }
    launches.push_back(LF);
  }
};

// Every product and leaf of a plan must stay inside its own matrix (lda x np
// elements from A) or its own scratch (need elements from tmp); the kernels
// assume it, so a plan that breaks it is refused.
template <typename T>
bool plan_in_bounds(const PlanBuilder<T> &b, const SpdMat *mats, std::string *why) {
  auto inside = [&](const T *p, int64_t span, int s) {
    const T *A = static_cast<const T *>(mats[s].A), *tmp = static_cast<const T *>(mats[s].tmp);
    if (p >= A && p + span <= A + mats[s].lda * mats[s].np) return true;
    return tmp && p >= tmp && p + span <= tmp + b.need[s];
  };
  for (size_t e = 0; e < b.gemms.size(); ++e) {
    const GemmArgs<T> &g = b.gemms[e];
    const int s = b.gemm_owner[e];
    const bool bt = b.gemm_bt[e] != 0;
    const bool ok = g.M > 0 && g.N > 0 && g.K > 0 && g.M % 64 == 0 && g.N % 64 == 0 &&
                    g.K % 64 == 0 && g.lda >= g.M && g.ldc >= g.M &&
                    g.ldb >= (bt ? g.N : g.K) &&
                    inside(g.A, (g.K - 1) * g.lda + g.M, s) &&
                    inside(g.B, bt ? (g.K - 1) * g.ldb + g.N : (g.N - 1) * g.ldb + g.K, s) &&
                    inside(g.C, (g.N - 1) * g.ldc + g.M, s);
    if (!ok) {
      if (why) *why = "product " + std::to_string(e) + " of matrix " + std::to_string(s);
      return false;
    }
  }
  for (size_t e = 0; e < b.leaves.size(); ++e) {
    const LeafArg<T> &l = b.leaves[e];
    const int s = b.leaf_owner[e], nb = b.leaf_nb[e];
    if (l.o < 0 || l.o + nb > mats[s].np || !inside(l.A + l.o + l.o * l.lda, (nb - 1) * l.lda + nb, s)) {
      if (why) *why = "leaf " + std::to_string(e) + " of matrix " + std::to_string(s);
      return false;
    }
  }
  return true;
}

template <typename T>
PlanBuilder<T> make_plan(const SpdMat *mats, int count, int64_t small = 0) {
  int64_t P = 0;
  for (int s = 0; s < count; ++s) P = std::max(P, mats[s].np);
  PlanBuilder<T> b;
  b.mats = mats;
  b.small = small;
  b.need.assign(count, 0);
  std::vector<int> act(count);
  for (int s = 0; s < count; ++s) act[s] = s;
  b.walk(0, P, act, std::vector<int64_t>(count, 0));
  return b;
}

}  // namespace

int spd_plan_check_host(const int64_t *np, int count, std::string *why, int64_t *n_launches) {
  // disjoint fake address ranges: matrix s at slot 2s, its scratch at 2s + 1
  std::vector<int64_t> need(count);
  spd_batch_scratch(np, count, need.data());
  std::vector<SpdMat> mats(count);
  uintptr_t base = 1 << 20;
  for (int s = 0; s < count; ++s) {
    const uintptr_t a = base;
    base += (uintptr_t)(np[s] * np[s] + 64) * 8;
    const uintptr_t t = base;
    base += (uintptr_t)(need[s] + 64) * 8;
    mats[s] = SpdMat{reinterpret_cast<void *>(a), np[s], np[s], reinterpret_cast<void *>(t), nullptr};
  }
  PlanBuilder<double> b = make_plan<double>(mats.data(), count);
  if (n_launches) *n_launches = (int64_t)b.launches.size();
  // every column block of every matrix must be factored by exactly one leaf
  std::vector<std::vector<int>> covered(count);
  for (int s = 0; s < count; ++s) covered[s].assign(np[s] / 64, 0);
  for (size_t e = 0; e < b.leaves.size(); ++e) {
    const int s = b.leaf_owner[e];
    for (int k = 0; k < b.leaf_nb[e] / 64; ++k) covered[s][b.leaves[e].o / 64 + k]++;
  }
  for (int s = 0; s < count; ++s)
    for (int c : covered[s])
      if (c != 1) {
        if (why) *why = "matrix " + std::to_string(s) + " column blocks not covered exactly once";
        return -1;
      }
  return plan_in_bounds(b, mats.data(), why) ? 0 : -1;
}

namespace {
}  // namespace

struct SpdPlan {
  std::vector<SpdMat> key;
  int64_t key_small = -1;
  std::vector<GemmArgs<double>> gemms;
  std::vector<LeafArg<double>> leaves;
  std::vector<PlanLaunch> launches;
  void *dev = nullptr;
  size_t dev_cap = 0;
};

void spd_batch_scratch(const int64_t *np, int count, int64_t *out) {
  std::vector<SpdMat> mats(count);
  int64_t P = 0;
  for (int s = 0; s < count; ++s) {
    mats[s] = SpdMat{nullptr, np[s], np[s], nullptr, nullptr};
    P = std::max(P, np[s]);
  }
  (void)P;
  PlanBuilder<double> b = make_plan<double>(mats.data(), count);
  for (int s = 0; s < count; ++s) out[s] = b.need[s];
}

SpdPlan *spd_plan_create() { return new SpdPlan(); }

void spd_plan_destroy(SpdPlan *p) {
  if (!p) return;
  if (p->dev) hipFree(p->dev);
  delete p;
}

static bool same_mats(const std::vector<SpdMat> &a, const SpdMat *b, int count) {
  if ((int)a.size() != count) return false;
  for (int s = 0; s < count; ++s)
    if (a[s].A != b[s].A || a[s].lda != b[s].lda || a[s].np != b[s].np || a[s].tmp != b[s].tmp ||
        a[s].ds != b[s].ds)
      return false;
  return true;
}

int spd_plan_build(SpdPlan *p, const SpdMat *mats, int count, hipStream_t st, int64_t small) {
  if (same_mats(p->key, mats, count) && p->key_small == small) return 0;
  PlanBuilder<double> b = make_plan<double>(mats, count, small);
  if (!plan_in_bounds(b, mats, nullptr)) return -2;
  const size_t bytes = sizeof(GemmArgs<double>) * b.gemms.size() +
                       sizeof(LeafArg<double>) * b.leaves.size() + 64;
  if (p->dev_cap < bytes) {
    if (p->dev) hipFree(p->dev);
    p->dev = nullptr;
    p->dev_cap = 0;
    if (hipMalloc(&p->dev, bytes) != hipSuccess) return -1;
    p->dev_cap = bytes;
  }
  p->gemms.swap(b.gemms);
  p->leaves.swap(b.leaves);
  p->launches.swap(b.launches);
  char *d = static_cast<char *>(p->dev);
  const size_t gb = sizeof(GemmArgs<double>) * p->gemms.size();
  if (gb && hipMemcpyAsync(d, p->gemms.data(), gb, hipMemcpyHostToDevice, st) != hipSuccess)
    return -1;
  if (!p->leaves.empty() &&
      hipMemcpyAsync(d + gb, p->leaves.data(), sizeof(LeafArg<double>) * p->leaves.size(),
                     hipMemcpyHostToDevice, st) != hipSuccess)
    return -1;
  if (hipStreamSynchronize(st) != hipSuccess) return -1;
  p->key.assign(mats, mats + count);
  p->key_small = small;
  return 0;
}

int64_t spd_plan_launches(const SpdPlan *p) { return (int64_t)p->launches.size(); }

void spd_plan_run(const SpdPlan *p, hipStream_t st) {
  const GemmArgs<double> *g = static_cast<const GemmArgs<double> *>(p->dev);
  const LeafArg<double> *lv =
      reinterpret_cast<const LeafArg<double> *>(static_cast<const char *>(p->dev) +
                                                sizeof(GemmArgs<double>) * p->gemms.size());
  for (const PlanLaunch &L : p->launches) {
    switch (L.kind) {
      case kPlanLeaf64:
        hipLaunchKernelGGL((k_leaf_mfma_b<double, 64>), dim3(L.gx), dim3(LeafThreads<64>::value), 0,
                           st, lv + L.first);
        break;
      case kPlanLeaf128:
        hipLaunchKernelGGL((k_leaf_mfma_b<double, 128>), dim3(L.gx), dim3(LeafThreads<128>::value), 0, st,
                           lv + L.first);
        break;
      case kPlanGemmT:
        if (L.tiles == kTiles32x8)
          hipLaunchKernelGGL((k_gemm32s_b<double, false, true, false, 8>),
                             dim3(L.gx, L.gy, L.count), dim3(512), 0, st, g + L.first);
        else if (L.tiles == kTiles32x4)
          hipLaunchKernelGGL((k_gemm32s_b<double, false, true, false, 4>),
                             dim3(L.gx, L.gy, L.count), dim3(256), 0, st, g + L.first);
        else
          hipLaunchKernelGGL((k_gemm64_b<double, false, true, false>), dim3(L.gx, L.gy, L.count),
                             dim3(256), 0, st, g + L.first);
        break;
      case kPlanPair:
        if (L.tiles == kTiles32x8)
          hipLaunchKernelGGL((k_gemm32s_pair_b<double, 8>), dim3(L.gx, 1, L.count), dim3(512), 0,
                             st, g + L.first, g + L.second);
        else if (L.tiles == kTiles32x4)
          hipLaunchKernelGGL((k_gemm32s_pair_b<double, 4>), dim3(L.gx, 1, L.count), dim3(256), 0,
                             st, g + L.first, g + L.second);
        else
          hipLaunchKernelGGL((k_gemm64_pair_b<double>), dim3(L.gx, 1, L.count), dim3(256), 0, st,
                             g + L.first, g + L.second);
        break;
      case kPlanFinal:
        if (L.tiles == kTiles32x8)
          hipLaunchKernelGGL((k_gemm32s_b<double, false, false, false, 8>),
                             dim3(L.gx, L.gy, L.count), dim3(512), 0, st, g + L.first);
        else if (L.tiles == kTiles32x4)
          hipLaunchKernelGGL((k_gemm32s_b<double, false, false, false, 4>),
                             dim3(L.gx, L.gy, L.count), dim3(256), 0, st, g + L.first);
        else  // A21 = -L22^-1 T2 (kLeM): grid transposed, see k_gemm64_b
          hipLaunchKernelGGL((k_gemm64_b<double, false, false, false>), dim3(L.gy, L.gx, L.count),
                             dim3(256), 0, st, g + L.first);
        break;
    }
  }
}

namespace {

inline dim3 grid2(int64_t n) { return dim3((unsigned)((n + 255) / 256), (unsigned)n); }

}  // namespace

void launch_scale_dense(int64_t N, const double *z, int64_t ldz, const double *q,
                        const double *s, const double *alpha, double *a, int64_t lda,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_scale_dense, grid2(N), dim3(256), 0, st, N, z, ldz, q, s, alpha, a, lda);
}

void launch_tuning_matrix(int64_t n, double *a, int64_t lda, hipStream_t st) {
  hipLaunchKernelGGL(k_tuning_matrix, grid2(n), dim3(256), 0, st, n, a, lda);
}

void launch_pad_identity(int64_t N, int64_t Np, double *a, int64_t lda, hipStream_t st) {
  if (Np == N) return;
  hipLaunchKernelGGL(k_pad_identity, dim3((unsigned)Np), dim3(64), 0, st, N, Np, a, lda);
}

int64_t spd_lower_inverse_scratch(int64_t Np) { return recurse_scratch(Np); }

void spd_lower_inverse_fp64(double *a, int64_t lda, int64_t Np, double *tmp, DevStatus *ds,
                            hipStream_t st, int64_t small) {
  recurse<double>(a, lda, 0, Np, tmp, ds, st, small);
}

static_assert((int)kFull == (int)kGemmFull && (int)kLeN == (int)kGemmLeN &&
                  (int)kGeN == (int)kGemmGeN && (int)kLeM == (int)kGemmLeM &&
                  (int)kGeMN == (int)kGemmGeMN,
              "public K-range modes follow the tile kernels'");

void gemm_f64(bool at, bool bt, bool lower, int64_t M, int64_t N, int64_t K, const double *A,
              int64_t lda, const double *B, int64_t ldb, double *C, int64_t ldc, double alpha,
              double beta, int kmode, hipStream_t st) {
  if (!at && !bt && !lower)
    gemm<double, false, false, false>(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, kmode, st);
  else if (!at && bt && !lower)
    gemm<double, false, true, false>(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, kmode, st);
  else if (at && !bt && !lower)
    gemm<double, true, false, false>(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, kmode, st);
  else if (at && !bt && lower)
    gemm<double, true, false, true>(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, kmode, st);
}

void spd_inverse_from_factor(const double *linv, int64_t ld, int64_t Np, double *x, int64_t ldx,
                             hipStream_t st) {
  // X = L^-T L^-1 on the tiles on or below the diagonal (diagonal tiles whole),
  // then the strict upper triangle from the lower one
  gemm<double, true, false, true>(Np, Np, Np, linv, ld, linv, ld, x, ldx, 1.0, 0.0, kGeMN, st);
  hipLaunchKernelGGL(k_mirror_lower, dim3((unsigned)(Np / 32), (unsigned)(Np / 32)), dim3(256), 0,
                     st, x, ldx);
}

void launch_pad_identity_scenes(int n_scenes, int64_t max_np, const int32_t *cam_off,
                                const int64_t *a_off, const int64_t *a_ld, double *amat,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_pad_identity_scenes, dim3((unsigned)max_np, (unsigned)n_scenes), dim3(64),
                     0, st, cam_off, a_off, a_ld, amat);
}

void launch_extract_scenes(int64_t n_cams, const int32_t *cam_scene, const int32_t *cam_off,
                           const int64_t *a_off, const int64_t *a_ld, const double *amat,
                           const double *s, const double *q, const double *alpha, double *cov,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_extract_scenes, dim3((unsigned)n_cams), dim3(256), 0, st, cam_scene,
                     cam_off, a_off, a_ld, amat, 9 * n_cams, s, q, alpha, cov);
}

void launch_extract(int64_t N, const double *linv, int64_t ld, const double *s,
                    const double *q, int64_t ldq, const double *alpha, bool subtract, double *cov,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_extract, dim3((unsigned)(N / 9)), dim3(256), 0, st, N, linv, ld, s, q,
                     ldq, alpha, (int)subtract, cov);
}

void launch_extract_full(int64_t N, const double *x, int64_t ld, const double *s,
                         const double *q, int64_t ldq, const double *alpha, bool subtract,
                         double *cov, hipStream_t st) {
  hipLaunchKernelGGL(k_extract_full, dim3((unsigned)(N / 9)), dim3(128), 0, st, N, x, ld, s, q,
                     ldq, alpha, (int)subtract, cov);
}

void mixed_initial_inverse(int64_t Np, const double *a, int64_t lda, float *a32, float *x32,
                           float *tmp32, DevStatus *ds, hipStream_t st) {
  // FP32 copy of the lower triangle, its inverse Cholesky factor, then
  // X0 = L^-T L^-1 (full, both triangles) on FP32 MFMA
  hipLaunchKernelGGL(k_lower_to_f32, grid2(Np), dim3(256), 0, st, Np, a, lda, a32, Np);
  recurse<float>(a32, Np, 0, Np, tmp32, ds, st);
  gemm<float, true, false, false>(Np, Np, Np, a32, Np, a32, Np, x32, Np, 1.0f, 0.0f, kGeMN, st);
}

void mixed_prepare(int64_t Np, double *a, int64_t lda, const float *x32, double *x,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_symmetrize, grid2(Np), dim3(256), 0, st, Np, a, lda);
  hipLaunchKernelGGL(k_f32_to_f64, grid2(Np), dim3(256), 0, st, Np, x32, Np, x, Np);
}

void mixed_residual(int64_t Np, const double *a, int64_t lda, const double *x, double *r,
                    double *sumsq, hipStream_t st) {
  // R = I - A X in FP64, and sumsq[0] = |R|_F^2 (sumsq: Np + 1 doubles, the
  // column sums after the total)
  hipLaunchKernelGGL(k_identity, grid2(Np), dim3(256), 0, st, Np, r, Np);
  gemm<double, false, false, false>(Np, Np, Np, a, lda, x, Np, r, Np, -1.0, 1.0, kFull, st);
  hipLaunchKernelGGL(k_sumsq, dim3((unsigned)Np), dim3(256), 0, st, Np, r, Np, sumsq + 1);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, st, Np, sumsq + 1, sumsq);
}

void mixed_update(int64_t Np, double *x, const double *r, float *x32, float *r32, float *d32,
                  hipStream_t st) {
  // X <- X + X R with the correction X R on FP32 MFMA
  hipLaunchKernelGGL(k_f64_to_f32, grid2(Np), dim3(256), 0, st, Np, x, Np, x32, Np);
  hipLaunchKernelGGL(k_f64_to_f32, grid2(Np), dim3(256), 0, st, Np, r, Np, r32, Np);
  gemm<float, false, false, false>(Np, Np, Np, x32, Np, r32, Np, d32, Np, 1.0f, 0.0f, kFull, st);
  hipLaunchKernelGGL(k_add_f32, grid2(Np), dim3(256), 0, st, Np, d32, Np, x, Np);
}

}  // namespace ucov

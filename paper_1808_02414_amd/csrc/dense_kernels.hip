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
// The leaves are 64x64 or 128x128 blocks factored and inverted by one workgroup;
// the products run on FP64 MFMA (v_mfma_f64_16x16x4f64) in 64x64 output tiles.
#include <algorithm>

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
// (Measured on MI355X: single-buffered LDS with a register prefetch and
// occupancy 4 beats double buffering, larger tiles and die-aware tile orders
// for every product shape of the recursion.)
// ---------------------------------------------------------------------------
constexpr int kKc = 16;     // K chunk staged in LDS
constexpr int kLdsPad = 4;  // row padding of the LDS tiles (doubles)

struct GemmArgs {
  int64_t M, N, K;
  const double *A;
  int64_t lda;
  const double *B;
  int64_t ldb;
  double *C;
  int64_t ldc;
  double alpha, beta;
  int kmode;
};

template <bool BT, bool LOWER>
__device__ inline void gemm_tile(const GemmArgs &g, int tm, int tn) {
  if (LOWER && tn > tm) return;
  const int64_t K = g.K, lda = g.lda, ldb = g.ldb, ldc = g.ldc;
  const double *__restrict__ A = g.A;
  const double *__restrict__ B = g.B;
  double *__restrict__ C = g.C;
  const double alpha = g.alpha, beta = g.beta;
  const int kmode = g.kmode;
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

// One product; grid (M/64, N/64), tile rows fastest.
template <bool BT, bool LOWER>
__global__ __launch_bounds__(256) void k_gemm64(GemmArgs g) {
  gemm_tile<BT, LOWER>(g, blockIdx.x, blockIdx.y);
}

// The two independent products of one recursion node in one launch: the
// Schur update A22 -= T T^T (lower tiles, first nblk_s workgroups) and
// T2 = T L11^-1.
__global__ __launch_bounds__(256) void k_gemm64_pair(GemmArgs s, GemmArgs t, int nblk_s) {
  const int b = blockIdx.x;
  if (b < nblk_s) {
    const int mt = (int)(s.M / 64);
    gemm_tile<true, true>(s, b % mt, b / mt);
  } else {
    const int mt = (int)(t.M / 64), bb = b - nblk_s;
    gemm_tile<false, false>(t, bb % mt, bb / mt);
  }
}

// ---------------------------------------------------------------------------
// Leaf of NB x NB (64 or 128): Cholesky factor L of the lower triangle and its
// inverse L^-1, by 4-column block steps.  The lower triangle is cut into 4x4
// micro-tiles (R, C), one per thread, held in registers.
//
// Factorisation, block step J:
//   1. the owners of block column J publish their (updated) tiles in LDS;
//   2. they factor the 4x4 diagonal block D = L_JJ L_JJ^T (each one locally)
//      and publish L(R,J) = A(R,J) L_JJ^-T;
//   3. every tile right of J applies A(R,C) -= L(R,J) L(C,J)^T.
// Inversion, block step J (right-looking forward elimination of L Y = I):
//   Y(J,C) = L_JJ^-1 W(J,C), then W(R,C) -= L(R,J) Y(J,C) for R > J, C <= J.
// Writes L^-1 (lower) into the tile and zeros above its diagonal.
// ---------------------------------------------------------------------------
// 4x4 Cholesky of the symmetric block d (only d[a][b], a >= b, is read):
// writes the lower factor into l and its inverse into li; returns false if a
// pivot is not positive.
__device__ inline bool chol4(const double (&d)[4][4], double (&l)[4][4], double (&li)[4][4]) {
  bool ok = true;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) l[a][b] = 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double p = d[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) p -= l[j][k] * l[j][k];
    ok = ok && (p > 0.0);
    const double ljj = sqrt(p);
    const double il = 1.0 / ljj;
    l[j][j] = ljj;
#pragma unroll
    for (int r = j + 1; r < 4; ++r) {
      double x = d[r][j];
#pragma unroll
      for (int k = 0; k < j; ++k) x -= l[r][k] * l[j][k];
      l[r][j] = x * il;
    }
    li[j][j] = il;
  }
  // li = l^-1 (lower), column by column
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (r < c) li[r][c] = 0.0;
      if (r > c) {
        double x = 0.0;
#pragma unroll
        for (int k = c; k < r; ++k) x -= l[r][k] * li[k][c];
        li[r][c] = x * li[r][r];
      }
    }
  }
  return ok;
}

template <int NB, int NT>
__global__ __launch_bounds__(NT) void k_leaf(double *A, int64_t lda, int64_t o, DevStatus *ds) {
  constexpr int MB = NB / 4;                // micro-tiles per edge
  constexpr int NMT = MB * (MB + 1) / 2;    // lower-triangle micro-tiles
  static_assert(NMT <= NT, "one micro-tile per thread");
  // panels indexed [column b][row a within the tile][tile row R] so that lanes
  // (consecutive tile rows) touch consecutive words
  __shared__ double P[4][4][MB];            // raw block column J
  __shared__ double Q[2][4][4][MB];         // L(., J)
  __shared__ double Yb[2][4][NB];           // block row J of W
  __shared__ double Dinv[MB][4][4];         // L_JJ^-1
  const int tid = threadIdx.x;
  const bool own = tid < NMT;
  double *T = A + o + o * lda;
  int R = MB, C = MB;  // idle threads own no tile
  if (own) {
    const double b = 2.0 * MB + 1.0;
    int cg = (int)((b - sqrt(b * b - 8.0 * tid)) * 0.5);
    cg = cg < 0 ? 0 : (cg > MB - 1 ? MB - 1 : cg);
    while (cg > 0 && cg * MB - cg * (cg - 1) / 2 > tid) --cg;
    while (cg < MB - 1 && (cg + 1) * MB - (cg + 1) * cg / 2 <= tid) ++cg;
    C = cg;
    R = C + (tid - (C * MB - C * (C - 1) / 2));
  }
  const int r0 = 4 * R, c0 = 4 * C;
  const int rr = own ? r0 : 0, cr = own ? c0 : 0;  // clamped LDS indices
  double v[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      // diagonal tiles are loaded symmetric so they stay symmetric under updates
      const int r = r0 + a, c = c0 + b;
      const int hi = r > c ? r : c, lo = r > c ? c : r;
      v[a][b] = own ? T[hi + (int64_t)lo * lda] : 0.0;
    }

  for (int J = 0; J < MB; ++J) {
    if (C == J) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) P[b][a][R] = v[a][b];
    }
    __syncthreads();
    if (C == J) {
      double d[4][4], l[4][4], li[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) d[a][b] = P[b][a][J];
      const bool ok = chol4(d, l, li);
      if (R == J) {
        if (!ok) report_error(ds, UCOV_EGAUGE, (int)((o + 4 * J) / 9));
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            v[a][b] = l[a][b];
            Dinv[J][a][b] = li[a][b];
          }
      } else {
        // L(R,J) = A(R,J) L_JJ^-T: row a times li^T
        double x[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m <= k; ++m) acc += v[a][m] * li[k][m];
            x[a][k] = acc;
          }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            v[a][b] = x[a][b];
            Q[0][b][a][R] = x[a][b];
          }
      }
    }
    __syncthreads();
    if (C > J && C < MB) {
      double lr[4][4], lc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          lr[a][b] = Q[0][b][a][rr >> 2];
          lc[a][b] = Q[0][b][a][cr >> 2];
        }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          v[a][b] -= lr[a][0] * lc[b][0] + lr[a][1] * lc[b][1] + lr[a][2] * lc[b][2] +
                     lr[a][3] * lc[b][3];
    }
  }
  // v now holds L (lower; the upper part of diagonal tiles is zero)
  double y[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) y[a][b] = (R == C && a == b) ? 1.0 : 0.0;
  for (int J = 0; J < MB; ++J) {
    const int buf = J & 1;
    if (C == J && R > J) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) Q[buf][b][a][R] = v[a][b];
    }
    if (R == J) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) Yb[buf][a][c0 + b] = y[a][b];
    }
    __syncthreads();
    if (C <= J && R >= J && R < MB) {
      double di[4][4], w[4][4], x[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          di[a][b] = Dinv[J][a][b];
          w[a][b] = Yb[buf][a][cr + b];
        }
      // X = Y(J,C) = L_JJ^-1 W(J,C)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          double acc = 0.0;
#pragma unroll
          for (int m = 0; m <= a; ++m) acc += di[a][m] * w[m][b];
          x[a][b] = acc;
        }
      if (R == J) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) y[a][b] = x[a][b];
      } else {
        double lr[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) lr[a][b] = Q[buf][b][a][rr >> 2];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b)
            y[a][b] -= lr[a][0] * x[0][b] + lr[a][1] * x[1][b] + lr[a][2] * x[2][b] +
                       lr[a][3] * x[3][b];
      }
    }
  }
  if (own) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int r = r0 + a, c = c0 + b;
        T[r + (int64_t)c * lda] = r >= c ? y[a][b] : 0.0;
      }
  }
  for (int e = tid; e < NB * NB; e += NT) {
    const int r = e % NB, c = e / NB;
    if ((r >> 2) < (c >> 2)) T[r + (int64_t)c * lda] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Leaf of NB x NB (64 or 128) on MFMA: Cholesky factor and inverse with the
// block resident in LDS (column-major, padded leading dimension) and 16-column
// panels.  Factorisation, panel p:
//   1. one wave factors the 16x16 diagonal block in registers (cross-lane
//      shuffles, reciprocal square roots refined by Newton steps) and inverts
//      it: L_pp and L_pp^-1;
//   2. the panel below: L_ip = A_ip L_pp^-T            (FP64 MFMA, 4 waves)
//   3. the trailing lower blocks: A_ij -= L_ip L_jp^T   (FP64 MFMA, 4 waves)
// Inversion (forward elimination of L Y = I by block rows), panel p:
//   a. L(., p) is staged in the unused upper blocks of block row p, and
//      Y(p, c) = L_pp^-1 W(p, c) for c < p, Y(p, p) = L_pp^-1;
//   b. W(i, c) -= L_ip Y(p, c) for i > p, c <= p.
// Writes L^-1 (lower) into the tile and zeros above its diagonal.
// ---------------------------------------------------------------------------
constexpr int kLP = 4;  // LDS leading-dimension padding (doubles)

// Broadcast lane l's value of x to the whole wave (scalar lane reads).
__device__ inline double readlane_d(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double rsqrt_nr(double x) {
  // hardware reciprocal square root, then two Newton-Raphson steps
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}

template <int NB>
__global__ __launch_bounds__(256) void k_leaf_mfma(double *A, int64_t lda, int64_t o,
                                                  DevStatus *ds) {
  constexpr int LD = NB + kLP;
  constexpr int NPAN = NB / 16;
  __shared__ double S[NB * LD];
  __shared__ double Dinv[NPAN][16 * 16];  // L_pp^-1, column-major 16x16
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  double *T = A + o + o * lda;
  // whole columns with 16-byte loads (the upper part is read and discarded)
  constexpr int NL = NB * NB / 2 / 256;
  double2 ld2[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int e = 2 * (tid + 256 * k);
    const int r = e % NB, c = e / NB;
    ld2[k] = *reinterpret_cast<const double2 *>(T + r + (int64_t)c * lda);
  }
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int e = 2 * (tid + 256 * k);
    const int r = e % NB, c = e / NB;
    S[c * LD + r] = r >= c ? ld2[k].x : 0.0;
    S[c * LD + r + 1] = r + 1 >= c ? ld2[k].y : 0.0;
  }
  __syncthreads();
  const int lr = lane & 15, lg = lane >> 4;  // row in block, column group

  for (int p = 0; p < NPAN; ++p) {
    const int c0 = 16 * p;
    // ---- 1. diagonal block on wave 0: lane r < 16 holds row r in registers;
    //         column values are broadcast with scalar lane reads ----
    if (wid == 0) {
      double v[16], y[16], rsv[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        v[c] = S[(c0 + c) * LD + c0 + lr];
        y[c] = (lr == c) ? 1.0 : 0.0;
      }
      bool ok = true;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const double piv = readlane_d(v[j], j);
        ok = ok && (piv > 0.0);
        const double rs = rsqrt_nr(piv);
        rsv[j] = rs;
        const double lj = v[j] * rs;  // L[lr][j]
#pragma unroll
        for (int c = j + 1; c < 16; ++c) v[c] -= lj * (readlane_d(v[j], c) * rs);
        v[j] = lr > j ? lj : (lr == j ? piv * rs : 0.0);
      }
      // y = L^-1: with row y_j final, y_r -= (L[r][j] / L[j][j]) y_j for r > j
#pragma unroll
      for (int j = 0; j < 15; ++j) {
        const double f = v[j] * rsv[j];
#pragma unroll
        for (int c = 0; c <= j; ++c) {
          const double yjc = readlane_d(y[c], j);
          if (lr > j) y[c] -= f * yjc;
        }
      }
      double my_rs = 0.0;
#pragma unroll
      for (int j = 0; j < 16; ++j) my_rs = (lr == j) ? rsv[j] : my_rs;
      if (lane < 16) {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          S[(c0 + c) * LD + c0 + lr] = v[c];
          Dinv[p][c * 16 + lr] = y[c] * my_rs;
        }
      }
      if (!ok && lane == 0) report_error(ds, UCOV_EGAUGE, (int)((o + c0) / 9));
    }
    __syncthreads();
    // ---- 2. panel: L_ip = A_ip L_pp^-T ----
    for (int i = p + 1 + wid; i < NPAN; i += 4) {
      d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int k = 4 * kk + lg;
        const double a = S[(c0 + k) * LD + 16 * i + lr];
        const double b = Dinv[p][k * 16 + lr];  // (L_pp^-1)[lr][k] = B^T[k][lr]
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) S[(c0 + lr) * LD + 16 * i + 4 * v + lg] = acc[v];
    }
    __syncthreads();
    // ---- 3. trailing: A_ij -= L_ip L_jp^T, p < j <= i ----
    {
      const int m = NPAN - 1 - p;  // trailing block rows
      const int nblk = m * (m + 1) / 2;
      for (int b = wid; b < nblk; b += 4) {
        // b -> (ii, jj) in the lower triangle of the m x m trailing blocks
        int jj = 0, rem = b;
        while (rem >= m - jj) {
          rem -= m - jj;
          ++jj;
        }
        const int i = p + 1 + jj + rem, j = p + 1 + jj;
        d4 acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = S[(16 * j + lr) * LD + 16 * i + 4 * v + lg];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int k = 4 * kk + lg;
          const double a = -S[(c0 + k) * LD + 16 * i + lr];
          const double bb = S[(c0 + k) * LD + 16 * j + lr];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) S[(16 * j + lr) * LD + 16 * i + 4 * v + lg] = acc[v];
      }
    }
    __syncthreads();
  }

  // ---- inversion by block rows ----
  for (int p = 0; p < NPAN; ++p) {
    const int c0 = 16 * p;
    // a. stage L(i, p), i > p, in block (p, i) (upper, unused) as a 16x16
    //    column-major copy; Y(p, c) = L_pp^-1 W(p, c) for c < p; Y(p, p).
    for (int i = p + 1 + wid; i < NPAN; i += 4) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 4 * v + lg;  // (row r, col lr) of L_ip
        S[(16 * i + lr) * LD + c0 + r] = S[(c0 + lr) * LD + 16 * i + r];
      }
    }
    for (int c = wid; c <= p; c += 4) {
      if (c == p) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int col = lg + 4 * v;
          S[(c0 + col) * LD + c0 + lr] = Dinv[p][col * 16 + lr];
        }
      } else {
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int k = 4 * kk + lg;
          const double a = Dinv[p][k * 16 + lr];                  // (L_pp^-1)[lr][k]
          const double b = S[(16 * c + lr) * LD + c0 + k];         // W(p, c)[k][lr]
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) S[(16 * c + lr) * LD + c0 + 4 * v + lg] = acc[v];
      }
    }
    __syncthreads();
    // b. W(i, c) -= L_ip Y(p, c), i > p, c <= p (W(i, p) starts at zero)
    {
      const int m = NPAN - 1 - p;
      const int nblk = m * (p + 1);
      for (int b = wid; b < nblk; b += 4) {
        const int i = p + 1 + b % m, c = b / m;
        d4 acc;
#pragma unroll
        for (int v = 0; v < 4; ++v)
          acc[v] = (c == p) ? 0.0 : S[(16 * c + lr) * LD + 16 * i + 4 * v + lg];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int k = 4 * kk + lg;
          const double a = -S[(16 * i + k) * LD + c0 + lr];        // L_ip[lr][k] from the stage
          const double bb = S[(16 * c + lr) * LD + c0 + k];       // Y(p, c)[k][lr]
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) S[(16 * c + lr) * LD + 16 * i + 4 * v + lg] = acc[v];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int e = 2 * (tid + 256 * k);
    const int r = e % NB, c = e / NB;
    double2 x;
    x.x = r >= c ? S[c * LD + r] : 0.0;
    x.y = r + 1 >= c ? S[c * LD + r + 1] : 0.0;
    *reinterpret_cast<double2 *>(T + r + (int64_t)c * lda) = x;
  }
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

GemmArgs make_args(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
                   const double *B, int64_t ldb, double *C, int64_t ldc, double alpha,
                   double beta, int kmode) {
  GemmArgs g;
  g.M = M; g.N = N; g.K = K; g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.alpha = alpha; g.beta = beta; g.kmode = kmode;
  return g;
}

template <bool BT, bool LOWER>
void gemm(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda, const double *B,
          int64_t ldb, double *C, int64_t ldc, double alpha, double beta, int kmode,
          hipStream_t st) {
  GemmArgs g = make_args(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, kmode);
  hipLaunchKernelGGL((k_gemm64<BT, LOWER>), dim3((unsigned)(M / 64), (unsigned)(N / 64)),
                     dim3(256), 0, st, g);
}

void gemm_pair(const GemmArgs &s, const GemmArgs &t, hipStream_t st) {
  const unsigned a = (unsigned)((s.M / 64) * (s.N / 64)), b = (unsigned)((t.M / 64) * (t.N / 64));
  hipLaunchKernelGGL(k_gemm64_pair, dim3(a + b), dim3(256), 0, st, s, t, (int)a);
}

// Scratch needed by recurse() for an n x n block (doubles).
int64_t recurse_scratch(int64_t n) {
  if (n <= 128) return 0;
  const int64_t tiles = n / 64, n1 = (tiles / 2) * 64, n2 = n - n1;
  return n2 * n1 + std::max(n2 * n1, std::max(recurse_scratch(n1), recurse_scratch(n2)));
}

// In-place L^-1 of the n x n block at offset o.  tmp[0, n2*n1) holds this
// level's T2 = L21 L11^-1 across the recursion into A22; the rest is scratch
// for T = L21 and for the children.
void recurse(double *A, int64_t lda, int64_t o, int64_t n, double *tmp, DevStatus *ds,
             hipStream_t st) {
  if (n == 64) {
    hipLaunchKernelGGL((k_leaf_mfma<64>), dim3(1), dim3(256), 0, st, A, lda, o, ds);
    return;
  }
  if (n == 128) {
    hipLaunchKernelGGL((k_leaf_mfma<128>), dim3(1), dim3(256), 0, st, A, lda, o, ds);
    return;
  }
  const int64_t tiles = n / 64;
  const int64_t n1 = (tiles / 2) * 64, n2 = n - n1;
  double *T2 = tmp;
  double *T = tmp + n2 * n1;
  double *child = T;
  recurse(A, lda, o, n1, child, ds, st);
  double *A11 = A + o + o * lda;
  double *A21 = A + (o + n1) + o * lda;
  double *A22 = A + (o + n1) + (o + n1) * lda;
  gemm<true, false>(n2, n1, n1, A21, lda, A11, lda, T, n2, 1.0, 0.0, kLeN, st);   // L21
  gemm_pair(make_args(n2, n2, n1, T, n2, T, n2, A22, lda, -1.0, 1.0, kFull),      // Schur
            make_args(n2, n1, n1, T, n2, A11, lda, T2, n2, 1.0, 0.0, kGeN), st);  // L21 L11^-1
  recurse(A, lda, o + n1, n2, child, ds, st);
  gemm<false, false>(n2, n1, n2, A22, lda, T2, n2, A21, lda, -1.0, 0.0, kLeM, st); // (L^-1)21
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

int64_t spd_lower_inverse_scratch(int64_t Np) { return recurse_scratch(Np); }

void spd_lower_inverse_fp64(double *a, int64_t lda, int64_t Np, double *tmp, DevStatus *ds,
                            hipStream_t st) {
  recurse(a, lda, 0, Np, tmp, ds, st);
}

void launch_extract(int64_t N, const double *linv, int64_t ld, const double *s,
                    const double *q, const double *alpha, double *cov, hipStream_t st) {
  hipLaunchKernelGGL(k_extract, dim3((unsigned)(N / 9)), dim3(256), 0, st, N, linv, ld, s, q,
                     alpha, cov);
}

}  // namespace ucov

// Whole camera covariance and point covariances (Sec. 5.2).
//
// The points are eliminated by block inversion: M = L diag(Z, V) L^T with
// L = [[I, W V^-1], [0, I]], so the camera covariance X (in either gauge)
// extends to the whole parameter vector, and the 3 x 3 block of point j is
// recovered from X and the point's own observations:
//
//   camera gauge (X = Z^+):  V_j^-1 + A_j^T Z^+ A_j,                A_j = W_j V_j^-1
//   paper gauge  (X = (M^+)_cc):
//     V_j^-1 - u_j^T u_j + E_j^T X E_j,  E_j = A_j + q u_j,  u_j = L_F^-1 H_p,j^T V_j^-1
//
// W_j holds the 9 x 3 blocks W_o = J_P,o^T J_X,o of the point's observations
// (whitened), so A_j's block of camera cam(o) is J_P,o^T Y_o with
// Y_o = J_X,o V_j^-1 from the slot record.  q = G L_F^-T is the paper gauge's
// rank-7 factor (G F^-1 G^T = q q^T) and L_F the Cholesky factor of
// F = H_p^T V^-1 H_p.  Expanding E_j^T X E_j gives the pair sum over the
// point's observations, P u_j + u_j^T P^T with P = A_j^T (X q), and
// u_j^T (q^T X q) u_j.
//
// X is held as the scaled inverse Xs = (S A S)^-1 of the dense stage, with
// X = S Xs S - Q Q^T / alpha (camera gauge) or X = S Xs S (paper gauge).
#include "ucov_internal.h"

namespace ucov {
namespace {

__device__ inline double wsum(double v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// The whole N x N camera covariance, column-major with leading dimension
// ldc, from Xs (both triangles, leading dimension ldx).  Grid: x over rows in
// 256s, y over columns (strided when N exceeds the grid).
__global__ __launch_bounds__(256) void k_full_camera(int64_t N, const double *x, int64_t ldx,
                                                     const double *s, const double *q,
                                                     const double *alpha, int subtract,
                                                     double *cov, int64_t ldc) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= N) return;
  double qr[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) qr[k] = subtract ? q[k * N + r] : 0.0;
  const double sr = s[r];
  const double ia = subtract ? 1.0 / alpha[0] : 0.0;
  for (int64_t c = blockIdx.y; c < N; c += gridDim.y) {
    double g = 0.0;
    if (subtract) {
#pragma unroll
      for (int k = 0; k < 7; ++k) g += qr[k] * q[k * N + c];
    }
    cov[r + c * ldc] = (sr * s[c]) * x[r + c * ldx] - g * ia;  // exactly symmetric
  }
}

// Partial sums of Xs (S q): part[(split * 7 + k) * N + r] over the columns of
// split blockIdx.y.
__global__ __launch_bounds__(256) void k_xq_partial(int64_t N, const double *x, int64_t ldx,
                                                    const double *s, const double *q,
                                                    int64_t chunk, double *part) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= N) return;
  const int64_t c0 = (int64_t)blockIdx.y * chunk;
  const int64_t c1 = c0 + chunk < N ? c0 + chunk : N;
  double acc[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) acc[k] = 0.0;
  for (int64_t c = c0; c < c1; ++c) {
    const double xv = x[r + c * ldx] * s[c];
#pragma unroll
    for (int k = 0; k < 7; ++k) acc[k] += xv * q[k * N + c];
  }
#pragma unroll
  for (int k = 0; k < 7; ++k) part[((int64_t)blockIdx.y * 7 + k) * N + r] = acc[k];
}

// X q = S (sum of the partial sums), N x 7 column-major (ld N).
__global__ __launch_bounds__(256) void k_xq_finish(int64_t N, int nsplit, const double *part,
                                                   const double *s, double *xq) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= N) return;
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    double v = 0.0;
    for (int p = 0; p < nsplit; ++p) v += part[((int64_t)p * 7 + k) * N + r];
    xq[k * N + r] = s[r] * v;
  }
}

// K = q^T (X q), 7 x 7 row-major, one workgroup.
__global__ __launch_bounds__(256) void k_gram7(int64_t N, const double *q, const double *xq,
                                               double *kmat) {
  double acc[28];
#pragma unroll
  for (int k = 0; k < 28; ++k) acc[k] = 0.0;
  for (int64_t r = threadIdx.x; r < N; r += 256) {
    double a[7], b[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      a[k] = q[k * N + r];
      b[k] = xq[k * N + r];
    }
    int idx = 0;
#pragma unroll
    for (int i = 0; i < 7; ++i)
#pragma unroll
      for (int j = i; j < 7; ++j) acc[idx++] += 0.5 * (a[i] * b[j] + a[j] * b[i]);
  }
  __shared__ double part[4][28];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 28; ++k) {
    const double v = wsum(acc[k]);
    if (lane == 0) part[wid][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 28) {
    int i = 0, rem = threadIdx.x;
    while (rem >= 7 - i) {
      rem -= 7 - i;
      ++i;
    }
    const int j = i + rem;
    const double v = part[0][threadIdx.x] + part[1][threadIdx.x] + part[2][threadIdx.x] +
                     part[3][threadIdx.x];
    kmat[7 * i + j] = v;
    kmat[7 * j + i] = v;
  }
}

// Wave-wide sum of a symmetric 3 x 3 held as (00 01 02 11 12 22).
__device__ inline void wsum6(double *v) {
#pragma unroll
  for (int k = 0; k < 6; ++k) v[k] = wsum(v[k]);
}

// One wave per point (4 points per workgroup).  See the file comment for
// the formula; b is Q (camera gauge) or X q (paper gauge), N x 7 with ld N;
// lf (L_F, 7 x 7 row-major) and kmat (q^T X q) are read in the paper gauge
// only.  Output: 9 values per point, the row-major 3 x 3 block.
__global__ __launch_bounds__(256) void k_point_cov(int m, const int64_t *ptr_p,
                                                   const int32_t *slot_cam, const double *rec,
                                                   const double *pts, const double *x,
                                                   int64_t ldx, const double *s, const double *b,
                                                   int64_t N, const double *alpha,
                                                   const double *lf, const double *kmat,
                                                   int paper, double *out) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= m) return;  // whole waves leave; no workgroup barrier follows
  const int64_t p0 = ptr_p[j], p1 = ptr_p[j + 1];
  const int64_t t = p1 - p0;
  if (t < 2) {  // rejected by the scene stage; never reached in a successful call
    if (lane < 9) out[9 * j + lane] = __builtin_nan("");
    return;
  }
  // V_j = sum of J_X^T J_X over the slots, and its inverse
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t sl = p0 + lane; sl < p1; sl += 64) {
    const double *jx = rec + sl * kRec + kRecJX;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const double a0 = jx[3 * p], a1 = jx[3 * p + 1], a2 = jx[3 * p + 2];
      v[0] += a0 * a0;
      v[1] += a0 * a1;
      v[2] += a0 * a2;
      v[3] += a1 * a1;
      v[4] += a1 * a2;
      v[5] += a2 * a2;
    }
  }
  wsum6(v);
  double w[3][3];
  spd3_inverse(v, w);
  // sum over ordered slot pairs: the unordered pairs (ia >= ib), the
  // off-diagonal ones counted with their transposes
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const int64_t npairs = t * (t + 1) / 2;
  for (int64_t e = lane; e < npairs; e += 64) {
    int64_t ia = (int64_t)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
    while (ia * (ia + 1) / 2 > e) --ia;
    while ((ia + 1) * (ia + 2) / 2 <= e) ++ia;
    const int64_t ib = e - ia * (ia + 1) / 2;
    const int64_t sa = p0 + ia, sb = p0 + ib;
    const int64_t ca = slot_cam[sa], cb = slot_cam[sb];
    const double *ra = rec + sa * kRec, *rb = rec + sb * kRec;
    double ja[2][9], jb[2][9];
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      const double sa_r = s[9 * ca + r], sb_r = s[9 * cb + r];
      ja[0][r] = ra[kRecJP + r] * sa_r;
      ja[1][r] = ra[kRecJP + 9 + r] * sa_r;
      jb[0][r] = rb[kRecJP + r] * sb_r;
      jb[1][r] = rb[kRecJP + 9 + r] * sb_r;
    }
    // n = Ja Xs_ab Jb^T (2 x 2)
    double n00 = 0, n01 = 0, n10 = 0, n11 = 0;
#pragma unroll
    for (int cc = 0; cc < 9; ++cc) {
      const double *col = x + (9 * cb + cc) * ldx + 9 * ca;
      double t0 = 0, t1 = 0;
#pragma unroll
      for (int r = 0; r < 9; ++r) {
        const double xv = col[r];
        t0 += ja[0][r] * xv;
        t1 += ja[1][r] * xv;
      }
      n00 += t0 * jb[0][cc];
      n01 += t0 * jb[1][cc];
      n10 += t1 * jb[0][cc];
      n11 += t1 * jb[1][cc];
    }
    // M = Ya^T n Yb (3 x 3)
    double ya[2][3], yb[2][3];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        ya[p][l] = ra[kRecY + 3 * p + l];
        yb[p][l] = rb[kRecY + 3 * p + l];
      }
    double ny[2][3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      ny[0][l] = n00 * yb[0][l] + n01 * yb[1][l];
      ny[1][l] = n10 * yb[0][l] + n11 * yb[1][l];
    }
    double M[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l) M[k][l] = ya[0][k] * ny[0][l] + ya[1][k] * ny[1][l];
    const double f = ia == ib ? 1.0 : 2.0;  // M + M^T on the symmetric part
    acc[0] += f * M[0][0];
    acc[1] += (ia == ib) ? 0.5 * (M[0][1] + M[1][0]) : M[0][1] + M[1][0];
    acc[2] += (ia == ib) ? 0.5 * (M[0][2] + M[2][0]) : M[0][2] + M[2][0];
    acc[3] += f * M[1][1];
    acc[4] += (ia == ib) ? 0.5 * (M[1][2] + M[2][1]) : M[1][2] + M[2][1];
    acc[5] += f * M[2][2];
  }
  wsum6(acc);
  // P = A_j^T B (3 x 7): per slot Y^T (J_P B_cam)
  double P[3][7];
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int k = 0; k < 7; ++k) P[l][k] = 0.0;
  for (int64_t sl = p0 + lane; sl < p1; sl += 64) {
    const int64_t ca = slot_cam[sl];
    const double *r = rec + sl * kRec;
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      const double *bk = b + k * N + 9 * ca;
      double g0 = 0, g1 = 0;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        g0 += r[kRecJP + i] * bk[i];
        g1 += r[kRecJP + 9 + i] * bk[i];
      }
#pragma unroll
      for (int l = 0; l < 3; ++l) P[l][k] += r[kRecY + l] * g0 + r[kRecY + 3 + l] * g1;
    }
  }
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int k = 0; k < 7; ++k) P[l][k] = wsum(P[l][k]);
  if (lane != 0) return;
  double C[3][3] = {{acc[0], acc[1], acc[2]}, {acc[1], acc[3], acc[4]}, {acc[2], acc[4], acc[5]}};
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) C[k][l] += w[k][l];
  if (!paper) {
    const double ia = 1.0 / alpha[0];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        double g = 0.0;
#pragma unroll
        for (int i = 0; i < 7; ++i) g += P[k][i] * P[l][i];
        C[k][l] -= g * ia;
      }
  } else {
    const double X0 = pts[3 * j], X1 = pts[3 * j + 1], X2 = pts[3 * j + 2];
    // H_p,j = [I, [X]x, X] (3 x 7); h = H_p,j^T V^-1 (7 x 3)
    const double H[3][7] = {{1, 0, 0, 0, -X2, X1, X0},
                            {0, 1, 0, X2, 0, -X0, X1},
                            {0, 0, 1, -X1, X0, 0, X2}};
    double u[7][3];
#pragma unroll
    for (int i = 0; i < 7; ++i)
#pragma unroll
      for (int l = 0; l < 3; ++l) u[i][l] = H[0][i] * w[0][l] + H[1][i] * w[1][l] + H[2][i] * w[2][l];
    // u = L_F^-1 h (forward substitution, column by column)
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int i = 0; i < 7; ++i) {
        double sum = u[i][l];
#pragma unroll
        for (int c = 0; c < i; ++c) sum -= lf[7 * i + c] * u[c][l];
        u[i][l] = sum / lf[7 * i + i];
      }
    // C += -u^T u + P u + (P u)^T + u^T K u
    double Ku[7][3];
#pragma unroll
    for (int i = 0; i < 7; ++i)
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        double sum = 0.0;
#pragma unroll
        for (int c = 0; c < 7; ++c) sum += kmat[7 * i + c] * u[c][l];
        Ku[i][l] = sum;
      }
    double Pu[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        double sum = 0.0;
#pragma unroll
        for (int i = 0; i < 7; ++i) sum += P[k][i] * u[i][l];
        Pu[k][l] = sum;
      }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        double uu = 0.0, uku = 0.0;
#pragma unroll
        for (int i = 0; i < 7; ++i) {
          uu += u[i][k] * u[i][l];
          uku += u[i][k] * Ku[i][l];
        }
        C[k][l] += -uu + Pu[k][l] + Pu[l][k] + uku;
      }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) out[9 * j + 3 * k + l] = 0.5 * (C[k][l] + C[l][k]);
}

}  // namespace

void launch_full_camera(int64_t N, const double *x, int64_t ldx, const double *s,
                        const double *q, const double *alpha, bool subtract, double *cov,
                        int64_t ldc, hipStream_t st) {
  const unsigned gy = (unsigned)(N < 65535 ? N : 65535);
  hipLaunchKernelGGL(k_full_camera, dim3((unsigned)((N + 255) / 256), gy), dim3(256), 0, st, N,
                     x, ldx, s, q, alpha, (int)subtract, cov, ldc);
}

int64_t xq_splits(int64_t N) {
  const int64_t rows = (N + 255) / 256;
  int64_t sp = (1024 + rows - 1) / rows;
  if (sp > N) sp = N;
  return sp < 1 ? 1 : sp;
}

void launch_xq(int64_t N, const double *x, int64_t ldx, const double *s, const double *q,
               double *part, double *xq, double *kmat, hipStream_t st) {
  const int64_t sp = xq_splits(N);
  const int64_t chunk = (N + sp - 1) / sp;
  const unsigned rows = (unsigned)((N + 255) / 256);
  hipLaunchKernelGGL(k_xq_partial, dim3(rows, (unsigned)sp), dim3(256), 0, st, N, x, ldx, s, q,
                     chunk, part);
  hipLaunchKernelGGL(k_xq_finish, dim3(rows), dim3(256), 0, st, N, (int)sp, part, s, xq);
  hipLaunchKernelGGL(k_gram7, dim3(1), dim3(256), 0, st, N, q, xq, kmat);
}

void launch_point_cov(const SceneDev &sc, const SceneWork &w, const double *x, int64_t ldx,
                      const double *b, const double *lf, const double *kmat, bool paper,
                      double *out, hipStream_t st) {
  if (sc.m == 0) return;
  hipLaunchKernelGGL(k_point_cov, dim3((unsigned)((sc.m + 3) / 4)), dim3(256), 0, st, sc.m,
                     w.ptr_p, w.slot_cam, w.rec, sc.pts, x, ldx, w.s, b, 9 * (int64_t)sc.n,
                     w.alpha, lf, kmat, (int)paper, out);
}

}  // namespace ucov

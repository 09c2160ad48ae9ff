// Incremental update of the camera covariance on adding observations or a
// camera (Sec. 6: the information of added observations adds to the Schur
// complement, and the Woodbury identity gives the new covariance).
//
// A new observation o of an existing point j acts on the cameras, once j is
// eliminated from the old system, as the rows
//     Jt_o = J_c,o - J_x,o V_j^-1 W_j^T
// (J_c,o on o's camera when that camera is an old one; the second term on the
// point's old cameras, block -(J_x,o V_j^-1 J_X,s^T) J_P,s for each old slot
// s) with error covariance I + J_x,o V_j^-1 J_x,o'^T between the new
// observations o, o' of one point (all rows whitened by their information).
// With JtT = Jt^T (N x 2k), B = Z^+ JtT and S = Omega^-1 + JtT^T B = L L^T,
//     Z^+  <-  Z^+ - T T^T,   T = B L^-T,
// and for a new camera (its own rows J_n, eliminated with a flat prior),
// U = L^-1 J_n, C_n = (U^T U)^-1, V = T U:
//     Z^+  <-  Z^+ - T T^T + V C_n V^T,  cross-covariance -V C_n.
// The products run on the FP64 MFMA tile kernels of the dense stage.
#include "camera_model.h"
#include "ucov_internal.h"
#include "../../include/ucov.h"

namespace ucov {
namespace {

__device__ inline double wsum(double v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// One thread per new observation (point-grouped position a, caller's index
// ord[a]): whitened J_P (2 x 9) and J_X (2 x 3) into nj[24 a ..], and for
// an observation by the new camera its J_P into rows 2a, 2a + 1 of jn
// (Kp x 64, leading dimension kp).
__global__ void k_new_jacobians(SceneDev sc, int64_t k, const int32_t *ord, const int32_t *ncam,
                                const int32_t *npt, const double *ninfo, const double *cam_new,
                                double *nj, double *jn, int64_t kp, DevStatus *ds) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= k) return;
  const int32_t o = ord[a];
  const int i = ncam[o], j = npt[o];
  const double *cp = i < sc.n ? sc.cams + 9 * (int64_t)i : cam_new;
  double cam[9], X[3];
#pragma unroll
  for (int q = 0; q < 9; ++q) cam[q] = cp[q];
#pragma unroll
  for (int q = 0; q < 3; ++q) X[q] = sc.pts[3 * (int64_t)j + q];
  if (!finite9(cam, 9) || !finite9(X, 3)) {
    report_error(ds, UCOV_EINVAL, o);
    return;
  }
  double l00 = 1.0, l01 = 0.0, l11 = 1.0;
  if (ninfo) {
    const double ia = ninfo[3 * (int64_t)o], ib = ninfo[3 * (int64_t)o + 1],
                 ic = ninfo[3 * (int64_t)o + 2];
    if (!(ia > 0.0) || !(ia * ic - ib * ib > 0.0) || !isfinite(ia + ib + ic)) {
      report_error(ds, UCOV_EINVAL, o);
      return;
    }
    l00 = sqrt(ia);
    l01 = ib / l00;
    l11 = sqrt(ic - l01 * l01);
  }
  Jac J;
  projection_jacobian(cam, X, J);
  if (!(J.x[2] > 0.0)) {
    report_error(ds, UCOV_EINVAL, o);
    return;
  }
  double *out = nj + 24 * a;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    out[q] = l00 * J.jp[0][q] + l01 * J.jp[1][q];
    out[9 + q] = l11 * J.jp[1][q];
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    out[18 + q] = l00 * J.jx[0][q] + l01 * J.jx[1][q];
    out[21 + q] = l11 * J.jx[1][q];
  }
  if (i >= sc.n) {
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      jn[2 * a + q * kp] = out[q];
      jn[2 * a + 1 + q * kp] = out[9 + q];
    }
  }
}

// One wave per new observation a: columns 2a, 2a + 1 of JtT (np x kp,
// zeroed beforehand) and rows 2a, 2a + 1 of S in the columns of the same
// point's new observations up to a (lower triangle).  grp0[a] is the first
// position of a's point.  An old camera of the point equal to o's camera is a
// duplicate observation (UCOV_EINVAL).
__global__ __launch_bounds__(64) void k_new_rows(SceneDev sc, const int32_t *ord,
                                                 const int32_t *ncam, const int32_t *npt,
                                                 const int32_t *grp0, const int64_t *ptr_p,
                                                 const int32_t *slot_cam, const double *rec,
                                                 const double *nj, double *jt, int64_t np,
                                                 double *S, int64_t kp, DevStatus *ds) {
  const int64_t a = blockIdx.x;
  const int lane = threadIdx.x;
  const int32_t o = ord[a];
  const int i = ncam[o], j = npt[o];
  const int64_t p0 = ptr_p[j], p1 = ptr_p[j + 1];
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t s = p0 + lane; s < p1; s += 64) {
    const double *x = rec + s * kRec + kRecJX;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const double a0 = x[3 * p], a1 = x[3 * p + 1], a2 = x[3 * p + 2];
      v[0] += a0 * a0;
      v[1] += a0 * a1;
      v[2] += a0 * a2;
      v[3] += a1 * a1;
      v[4] += a1 * a2;
      v[5] += a2 * a2;
    }
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) v[q] = wsum(v[q]);
  double w[3][3];
  spd3_inverse(v, w);
  const double *na = nj + 24 * a;
  double g[2][3];  // J_x,o V_j^-1
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int l = 0; l < 3; ++l)
      g[p][l] = na[18 + 3 * p] * w[0][l] + na[19 + 3 * p] * w[1][l] + na[20 + 3 * p] * w[2][l];
  if (i < sc.n && lane < 18) {
    const int p = lane / 9, r = lane % 9;
    jt[(9 * (int64_t)i + r) + (2 * a + p) * np] = na[9 * p + r];
  }
  for (int64_t s = p0 + lane; s < p1; s += 64) {
    const int cs = slot_cam[s];
    if (cs == i) report_error(ds, UCOV_EINVAL, o);
    const double *r = rec + s * kRec;
    double c[2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q)
        c[p][q] = g[p][0] * r[kRecJX + 3 * q] + g[p][1] * r[kRecJX + 3 * q + 1] +
                  g[p][2] * r[kRecJX + 3 * q + 2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int rr = 0; rr < 9; ++rr)
        jt[(9 * (int64_t)cs + rr) + (2 * a + p) * np] =
            -(c[p][0] * r[kRecJP + rr] + c[p][1] * r[kRecJP + 9 + rr]);
  }
  for (int64_t b = grp0[a] + lane; b <= a; b += 64) {
    const double *xb = nj + 24 * b + 18;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const double val = g[p][0] * xb[3 * q] + g[p][1] * xb[3 * q + 1] + g[p][2] * xb[3 * q + 2];
        S[(2 * a + p) + (2 * b + q) * kp] = val + ((b == a && p == q) ? 1.0 : 0.0);
      }
  }
}

// Zp (np x np) = the caller's N x N matrix (leading dimension ldc), zero padded.
__global__ __launch_bounds__(256) void k_copy_in(int64_t N, int64_t np, const double *src,
                                                 int64_t ldc, double *zp) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= np) return;
  for (int64_t c = blockIdx.y; c < np; c += gridDim.y)
    zp[r + c * np] = (r < N && c < N) ? src[r + c * ldc] : 0.0;
}

// The caller's matrix = the symmetric part of Zp's leading N x N block.
__global__ __launch_bounds__(256) void k_copy_out(int64_t N, int64_t np, const double *zp,
                                                  double *dst, int64_t ldc) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= N) return;
  for (int64_t c = blockIdx.y; c < N; c += gridDim.y)
    dst[r + c * ldc] = 0.5 * (zp[r + c * np] + zp[c + r * np]);
}

// One thread: C_n = (U^T U)^-1 from the leading 9 x 9 of g (64 x 64), its
// Cholesky factor L_C (C_n = L_C L_C^T); both 9 x 9 row-major into cn and lc.
// A Gram matrix that is not positive definite means the new camera is not
// determined by its observations (UCOV_EGAUGE).
__global__ void k_new_camera(const double *g, double *cn, double *lc, DevStatus *ds) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double A[9][9], L[9][9], Li[9][9];
  double tr = 0.0;
  for (int r = 0; r < 9; ++r)
    for (int c = 0; c < 9; ++c) A[r][c] = 0.5 * (g[r + 64 * c] + g[c + 64 * r]);
  for (int r = 0; r < 9; ++r) tr += A[r][r];
  for (int r = 0; r < 9; ++r) {
    for (int c = 0; c <= r; ++c) {
      double s = A[r][c];
      for (int q = 0; q < c; ++q) s -= L[r][q] * L[c][q];
      if (r == c) {
        if (!(s > 1e-15 * tr)) {
          report_error(ds, UCOV_EGAUGE, -1);
          s = 1.0;
        }
        L[r][r] = sqrt(s);
      } else {
        L[r][c] = s / L[c][c];
      }
    }
    for (int c = r + 1; c < 9; ++c) L[r][c] = 0.0;
  }
  // Li = L^-1 (lower)
  for (int c = 0; c < 9; ++c)
    for (int r = 0; r < 9; ++r) {
      if (r < c) {
        Li[r][c] = 0.0;
        continue;
      }
      double s = (r == c) ? 1.0 : 0.0;
      for (int q = c; q < r; ++q) s -= L[r][q] * Li[q][c];
      Li[r][c] = s / L[r][r];
    }
  // C = Li^T Li; its Cholesky factor (lower)
  double C[9][9];
  for (int r = 0; r < 9; ++r)
    for (int c = 0; c < 9; ++c) {
      double s = 0.0;
      for (int q = 0; q < 9; ++q) s += Li[q][r] * Li[q][c];
      C[r][c] = s;
    }
  for (int r = 0; r < 9; ++r)
    for (int c = 0; c < 9; ++c) cn[9 * r + c] = 0.5 * (C[r][c] + C[c][r]);
  for (int r = 0; r < 9; ++r) {
    for (int c = 0; c <= r; ++c) {
      double s = cn[9 * r + c];
      for (int q = 0; q < c; ++q) s -= lc[9 * r + q] * lc[9 * c + q];
      lc[9 * r + c] = (r == c) ? sqrt(s > 0.0 ? s : 0.0) : s / lc[9 * c + c];
    }
    for (int c = r + 1; c < 9; ++c) lc[9 * r + c] = 0.0;
  }
}

// W = V L_C (np x 64, columns 9.. zero) and, for rows r < N when cross is
// not null, cross[9 r + k] = -(V C_n)[r][k].  V: np x 64 (ld np).
__global__ __launch_bounds__(256) void k_new_camera_rows(int64_t N, int64_t np, const double *V,
                                                         const double *cn, const double *lc,
                                                         double *W, double *cross) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= np) return;
  double v[9];
#pragma unroll
  for (int l = 0; l < 9; ++l) v[l] = V[r + l * np];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    double s = 0.0, x = 0.0;
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      s += v[l] * lc[9 * l + q];
      x += v[l] * cn[9 * l + q];
    }
    W[r + q * np] = s;
    if (cross && r < N) cross[9 * r + q] = -x;
  }
  for (int q = 9; q < 64; ++q) W[r + q * np] = 0.0;
}

}  // namespace

void launch_new_jacobians(const SceneDev &sc, int64_t k, const int32_t *ord,
                          const int32_t *ncam, const int32_t *npt, const double *ninfo,
                          const double *cam_new, double *nj, double *jn, int64_t kp,
                          DevStatus *ds, hipStream_t st) {
  hipLaunchKernelGGL(k_new_jacobians, dim3((unsigned)((k + 127) / 128)), dim3(128), 0, st, sc, k,
                     ord, ncam, npt, ninfo, cam_new, nj, jn, kp, ds);
}

void launch_new_rows(const SceneDev &sc, const SceneWork &w, int64_t k, const int32_t *ord,
                     const int32_t *ncam, const int32_t *npt, const int32_t *grp0,
                     const double *nj, double *jt, int64_t np, double *S, int64_t kp,
                     DevStatus *ds, hipStream_t st) {
  hipLaunchKernelGGL(k_new_rows, dim3((unsigned)k), dim3(64), 0, st, sc, ord, ncam, npt, grp0,
                     w.ptr_p, w.slot_cam, w.rec, nj, jt, np, S, kp, ds);
}

void launch_copy_in(int64_t N, int64_t np, const double *src, int64_t ldc, double *zp,
                    hipStream_t st) {
  const unsigned gy = (unsigned)(np < 65535 ? np : 65535);
  hipLaunchKernelGGL(k_copy_in, dim3((unsigned)((np + 255) / 256), gy), dim3(256), 0, st, N, np,
                     src, ldc, zp);
}

void launch_copy_out(int64_t N, int64_t np, const double *zp, double *dst, int64_t ldc,
                     hipStream_t st) {
  const unsigned gy = (unsigned)(N < 65535 ? N : 65535);
  hipLaunchKernelGGL(k_copy_out, dim3((unsigned)((N + 255) / 256), gy), dim3(256), 0, st, N, np,
                     zp, dst, ldc);
}

void launch_new_camera(const double *g, double *cn, double *lc, int64_t N, int64_t np,
                       const double *V, double *W, double *cross, DevStatus *ds, hipStream_t st) {
  hipLaunchKernelGGL(k_new_camera, dim3(1), dim3(64), 0, st, g, cn, lc, ds);
  hipLaunchKernelGGL(k_new_camera_rows, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, N,
                     np, V, cn, lc, W, cross);
}

}  // namespace ucov

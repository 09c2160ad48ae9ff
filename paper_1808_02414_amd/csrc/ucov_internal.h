// Internal declarations shared by the ucov HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include <cstdint>

namespace ucov {

// First device-detected error of a call.  Kernels record it with
// report_error(); the host reads it back after the stream has drained.
struct DevStatus {
  int code;   // 0 or a negative UCOV_E* code
  int index;  // offending observation / point / camera
};

__device__ inline void report_error(DevStatus *st, int code, int index) {
  if (atomicCAS(&st->code, 0, code) == 0) atomicExch(&st->index, index);
}

// Inverse of a symmetric positive definite 3 x 3 held as (00 01 02 11 12 22),
// through its Cholesky factor (full 3 x 3 result).
__device__ inline void spd3_inverse(const double *v, double w[3][3]) {
  const double L00 = sqrt(v[0]), L10 = v[1] / L00, L20 = v[2] / L00;
  const double L11 = sqrt(v[3] - L10 * L10), L21 = (v[4] - L20 * L10) / L11;
  const double L22 = sqrt(v[5] - L20 * L20 - L21 * L21);
  const double M00 = 1.0 / L00, M11 = 1.0 / L11, M22 = 1.0 / L22;
  const double M10 = -L10 * M00 * M11, M21 = -L21 * M11 * M22;
  const double M20 = -(L20 * M00 + L21 * M10) * M22;
  w[0][0] = M00 * M00 + M10 * M10 + M20 * M20;
  w[0][1] = w[1][0] = M10 * M11 + M20 * M21;
  w[0][2] = w[2][0] = M20 * M22;
  w[1][1] = M11 * M11 + M21 * M21;
  w[1][2] = w[2][1] = M21 * M22;
  w[2][2] = M22 * M22;
}

// Tile edge of the dense factorisation; every dense dimension is padded to it.
constexpr int kTile = 64;

// Per-slot record (observations grouped by point, cameras ascending within
// a point), 32 doubles = 256 bytes:
//   [0..17]  whitened J_P (2x9 row-major)
//   [18..23] whitened J_X (2x3 row-major)
//   [24..29] Y = J_X V^-1 (2x3 row-major), the point-eliminated coupling
constexpr int kRec = 32;
constexpr int kRecJP = 0;
constexpr int kRecJX = 18;
constexpr int kRecY = 24;

// ---- scene stage (scene_kernels.hip) ---------------------------------------
struct SceneDev {
  int n = 0, m = 0;
  int64_t t = 0;
  const double *cams = nullptr, *pts = nullptr, *info = nullptr;
  const int32_t *oc = nullptr, *op = nullptr;
  // Several independent scenes concatenated (cameras, points and observations
  // of scene s follow those of scene s-1); all null for a single scene.
  int n_scenes = 1;
  const int32_t *cam_scene = nullptr;  // n: scene of each camera
  const int32_t *cam_off = nullptr;    // n_scenes + 1: first camera of each scene
  const int64_t *bin_off = nullptr;    // n_scenes + 1: first camera-pair bin of each scene
  const int64_t *a_off = nullptr;      // n_scenes + 1: offset of each scene's dense matrix
  const int64_t *a_ld = nullptr;       // n_scenes: leading dimension of each scene's matrix
};

// One scene of a batch as the caller passed it (local indices) and where it
// goes in the concatenation.
struct BatchEntry {
  const double *cams, *pts, *info;
  const int32_t *oc, *op;
  int32_t n, m;
  int64_t t;
  int32_t cam0, pt0;
  int64_t obs0;
};

struct SceneWork {
  // observations grouped by point
  int32_t *cnt_p;     // m
  int64_t *ptr_p;     // m + 1
  int32_t *cur_p;     // m
  int64_t *slot_key;  // t: (camera << 32 | observation) of each slot before the sort
  int32_t *slot_obs;  // t: observation id of each slot
  int32_t *slot_cam;  // t
  int32_t *slot_pt;   // t
  double *rec;        // t x kRec
  // camera-pair bins (lower triangle, bin(i,k) = i(i+1)/2 + k, i >= k)
  int32_t *bin_cnt;   // nbins
  int64_t *bin_ptr;   // nbins + 1
  int32_t *bin_cur;   // nbins
  int2 *pairs;        // n_pairs (slot a of camera i, slot b of camera k)
  // slots grouped by camera (camera-major bin construction)
  int32_t *cam_keys;  // t: camera of each slot, sorted
  int32_t *cam_slots; // t: slots in camera order, ascending within a camera
  int64_t *cam_ptr;   // n + 1
  int2 *nzlist;       // (i, k) of every non-empty bin, in bin order
  int64_t *nzcount;   // [0]: number of non-empty bins
  int64_t *nzpos;     // nbins + 1: exclusive scan of the non-empty flags
  // per camera
  double *zdiag;      // n x 81, diagonal blocks of Z (row-major)
  double *hc;         // N x 7 column-major (ld N)
  double *q;          // N x 7 column-major (ld N)
  double *s;          // N, Jacobi scaling of Z + a QQ^T
  double *alpha;      // 1
  int64_t *scan_tmp;  // scan block sums
};

void exclusive_scan(const int32_t *in, int64_t *out, int64_t len, int64_t *tmp,
                    hipStream_t st);
void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st);
void fill_f64(double *p, double v, int64_t n, hipStream_t st);

// Gathers the scenes of a batch into one concatenation (cams, pts, oc, op and,
// when info is not null, the information blocks; identity for a scene without
// them).  Local indices outside their own scene are reported as UCOV_EINVAL
// (index: observation in the concatenation) and replaced by index 0 of the
// scene, so that no later kernel leaves the scene.  Also fills cam_scene.
void launch_concat_scenes(int n_scenes, const BatchEntry *tab, int64_t max_elems, double *cams,
                          double *pts, double *info, int32_t *oc, int32_t *op,
                          int32_t *cam_scene, DevStatus *ds, hipStream_t st);
void launch_count_points(const SceneDev &sc, SceneWork &w, DevStatus *ds, hipStream_t st);
void launch_group_points(const SceneDev &sc, SceneWork &w, DevStatus *ds, hipStream_t st);
void launch_jacobians(const SceneDev &sc, SceneWork &w, double *jp_out, double *jx_out,
                      DevStatus *ds, hipStream_t st);
void launch_point_blocks(const SceneDev &sc, SceneWork &w, DevStatus *ds, hipStream_t st);
void launch_pair_count(const SceneDev &sc, SceneWork &w, hipStream_t st);
// nzlist / nzcount from bin_cnt (needs bin_cur as scratch; leaves it zero)
void launch_nonzero_bins(const SceneDev &sc, SceneWork &w, int64_t nbins, hipStream_t st);
// Pairs into the list (capacity cap entries; nothing is written when the pair
// count bin_ptr[nbins] exceeds it or *skip, when skip is given, is set).
void launch_pair_fill(const SceneDev &sc, SceneWork &w, int64_t nbins, int64_t cap,
                      const int32_t *skip, hipStream_t st);
// A recorded launch sequence replayed on a scene whose camera-pair structure
// grew: when the pair count (bin_ptr[nbins]) exceeds pairs_cap, every bin is
// emptied (flag: one device int32) and UCOV_EINVAL reported; more non-empty
// bins than nz_cap are reported as well.
void launch_guard_pairs(SceneWork &w, int64_t nbins, int64_t pairs_cap, int32_t *flag,
                        DevStatus *ds, hipStream_t st);
void launch_check_nonzero(const SceneWork &w, int64_t nz_cap, DevStatus *ds, hipStream_t st);
// Camera-major bins for scenes of at most kCamHistMax cameras (LDS counters
// per camera): the camera lists, then every bin count (no prior zero fill),
// then the pairs (fewer than 2^31 in all; else launch_pair_fill).
// camera_lists_scratch: bytes of sort scratch for t slots;
// launch_camera_lists returns nonzero when the sort cannot be launched.
constexpr int kCamHistMax = 16384;
size_t camera_lists_scratch(int64_t t);
int launch_camera_lists(const SceneDev &sc, SceneWork &w, void *tmp, size_t tmp_bytes,
                        hipStream_t st);
void launch_pair_count_cam(const SceneDev &sc, SceneWork &w, int max_scene_cams,
                           hipStream_t st);
void launch_pair_fill_cam(const SceneDev &sc, SceneWork &w, int max_scene_cams, int64_t nbins,
                          int64_t cap, const int32_t *skip, hipStream_t st);
void launch_camera_diag(const SceneDev &sc, SceneWork &w, DevStatus *ds, hipStream_t st);
// Orthonormal Q (Cholesky-QR2 of hc; skipped when hc is null and q is given),
// the gauge weight alpha and the Jacobi scaling s.  diag(Z) comes from the
// per-camera blocks zdiag (n x 81) or, when that is null, from a dense z.
void launch_gauge(int64_t N, const double *hc, double *q, const double *zdiag,
                  const double *zdense, int64_t ldz, double user_alpha, double *s,
                  double *alpha, DevStatus *ds, hipStream_t st);
// The same for every scene of a concatenation (one workgroup per scene; hc, q
// are N_total x 7 with leading dimension N_total; alpha has one entry per scene).
void launch_gauge_scenes(const SceneDev &sc, const double *hc, double *q, const double *zdiag,
                         double user_alpha, double *s, double *alpha, DevStatus *ds,
                         hipStream_t st);
// The paper's gauge (M^+)_cc: q <- G L_F^-T (N x 7) with G = H_c - W V^-1 H_p
// and F = H_p^T V^-1 H_p = L_F L_F^T (f: paper_gauge_doubles(m) doubles, F's
// upper triangle, then L_F row-major, then scratch), alpha <- 1, so that (Z + q q^T)^-1 is the covariance.
// Needs hc from the scene stage.
constexpr int kPaperF = 28 + 49;
// Doubles of f for a scene of m points (kPaperF, then per-workgroup sums).
int64_t paper_gauge_doubles(int64_t m);
void launch_paper_gauge(const SceneDev &sc, SceneWork &w, double *f, DevStatus *ds,
                        hipStream_t st);
// mode 0: write Z (both triangles) into out; mode 1: write the lower triangle of
// S (Z + a QQ^T) S into out (per scene at out + a_off[s] with leading dimension
// a_ld[s] for a concatenation).  n_nonzero is the number of non-empty bins;
// max_scene_cams: cameras of the largest scene (n for one scene).
void launch_assemble(const SceneDev &sc, SceneWork &w, int mode, double *out, int64_t ld,
                     int64_t n_nonzero, hipStream_t st, int64_t max_scene_cams = -1);

// Sub-reconstructions: sub-scene arrays gathered from a parent scene through
// index maps (camera, point and, when pinfo is set, observation of the parent
// for every row of the concatenation), and the minimum-trace choice per parent
// camera among n_decomp candidate blocks (pos: n_decomp x n rows of cand).
void launch_gather_subscenes(int64_t n, int64_t m, int64_t t, const int32_t *cam_src,
                             const int32_t *pt_src, const int32_t *obs_src, const double *pcams,
                             const double *ppts, const double *pinfo, double *cams, double *pts,
                             double *info, hipStream_t st);
void launch_min_trace(int64_t n, int n_decomp, const int32_t *pos, const double *cand,
                      double *cov, int32_t *chosen, hipStream_t st);
// The sub-scenes' points and observations, chosen on the device from the
// parent's observations (oc, op: t each) and the cameras' groups: gsub
// (n_decomp x n) the sub-scene of camera c in decomposition d, numbered so
// that sub-scene ids grow with d; cslot (n_decomp x n) its camera slot in that
// sub-scene.  A point belongs to a sub-scene when at least two of its
// observations fall in it.  Outputs per sub-scene s <= S: obs_off, pt_off
// (first row in the concatenation, [S] the totals); per kept observation
// (sub-scene order, points ascending): obs_src (parent observation), loc_c,
// loc_p (camera and point in the sub-scene); per kept point its parent index
// pt_src.  Observation indices out of range are reported in ds (index: the
// observation).  n_decomp * t must be below 2^31; tmp holds
// subscene_select_scratch(n_decomp * t) bytes.
size_t subscene_select_scratch(int64_t T);
void launch_subscene_select(int64_t t, int n_decomp, int32_t n, int32_t m, int32_t S,
                            const int32_t *oc, const int32_t *op, const int32_t *gsub,
                            const int32_t *cslot, void *tmp, int64_t *obs_off, int64_t *pt_off,
                            int32_t *obs_src, int32_t *loc_c, int32_t *loc_p, int32_t *pt_src,
                            DevStatus *ds, hipStream_t st);

// ---- learned screener (screener_kernels.hip) -------------------------------
// Per-camera features (n x 55 FP32) from the scene stage's data; hist (8 n),
// ang (n) and covis (n) are scratch.
void launch_screener_features(const SceneDev &sc, const SceneWork &w, int32_t *hist,
                              double *ang, int32_t *covis, float *feat, hipStream_t st);
int64_t mlp_param_count();
size_t mlp_workspace_bytes(int64_t batch);
// y = MLP((x - mean) / std); mean, std may be null
void mlp_forward(const float *params, int64_t batch, const float *x, const float *mean,
                 const float *stdv, float *y, void *ws, hipStream_t st);
// gradient of the mean squared error against target (batch x 45); loss (device
// scalar) may be null
void mlp_gradient(const float *params, int64_t batch, const float *x, const float *mean,
                  const float *stdv, const float *target, float *grad, float *loss, void *ws,
                  hipStream_t st);
void mlp_adam(int64_t n, float *params, const float *grad, float *m, float *v, float lr,
              int64_t step, hipStream_t st);
// Per column of x (n x cols FP32): mean and standard deviation (n - 1, at
// least 1e-6).  Per camera: b (n x 9) = sqrt(diag((Z_ii)^-1)) from its Z_ii
// features.  Per diagonal entry of n 9 x 9 blocks: s = sqrt(lower median of
// cov_aa / b_a^2).  Label transforms with the per-camera scale D = s b.
void launch_col_stats(int64_t n, int cols, const float *x, float *mean, float *stdv,
                      hipStream_t st);
// Per column: the lower median and 1.4826 x the lower median absolute
// deviation (at least 1e-6).
void launch_col_robust(int64_t n, int cols, const float *x, float *center, float *spread,
                       hipStream_t st);
void launch_block_scale(int64_t n, const float *feat, double *b, DevStatus *ds, hipStream_t st);
void launch_diag_median(int64_t n, const double *cov, const double *b, double *s_glob,
                        hipStream_t st);
void launch_labels(int64_t n, const double *cov, const double *b, const double *s_glob,
                   const float *mean, const float *stdv, bool clip, float *lab, DevStatus *ds,
                   hipStream_t st);
void launch_predicted_cov(int64_t n, const float *y, const double *b, const double *s_glob,
                          const float *mean, const float *stdv, double *cov, double *spread,
                          hipStream_t st);

// ---- dense stage (dense_kernels.hip) ---------------------------------------
// Scaled positive-definite matrix a = S (Z + alpha QQ^T) S from a caller's Z.
void launch_scale_dense(int64_t N, const double *z, int64_t ldz, const double *q,
                        const double *s, const double *alpha, double *a, int64_t lda,
                        hipStream_t st);
// Identity on the padding rows/columns [N, Np) of the lower triangle.
void launch_pad_identity(int64_t N, int64_t Np, double *a, int64_t lda, hipStream_t st);
// In-place L^-1 of the Cholesky factor of the lower triangle of a (Np x Np),
// using tmp (spd_lower_inverse_scratch(Np) doubles) as workspace.
int64_t spd_lower_inverse_scratch(int64_t Np);
// Batched form for many matrices of different padded sizes np (multiples of
// 64): each matrix's lower triangle is replaced by its inverse Cholesky
// factor; tmp is the matrix's own scratch of spd_batch_scratch() elements.
struct SpdMat {
  void *A;
  int64_t lda, np;
  void *tmp;
  DevStatus *ds;
};
void spd_batch_scratch(const int64_t *np, int count, int64_t *out);
struct SpdPlan;  // launch plan with its argument tables in device memory
SpdPlan *spd_plan_create();
void spd_plan_destroy(SpdPlan *p);
// Builds the plan for these matrices (kept when they are the same as in the
// last build); returns 0 or -1 on a HIP failure.
// Products of a launch with fewer 64 x 64 tiles (summed over the scenes) than
// `small` run on split 32 x 32 tiles.
int spd_plan_build(SpdPlan *p, const SpdMat *mats, int count, hipStream_t st, int64_t small = 0);
int64_t spd_plan_launches(const SpdPlan *p);
void spd_plan_run(const SpdPlan *p, hipStream_t st);
// Host-only check of the plan for matrices of sizes np: every access inside
// its matrix or scratch, every column block factored once.  0 when it holds.
int spd_plan_check_host(const int64_t *np, int count, std::string *why, int64_t *n_launches);
// Products of the recursion with fewer 64 x 64 tiles than `small` run on
// 32 x 32 tiles; the default comes from a sweep on the 4500 x 4500 case,
// ucov_tune_dense picks it per size.
constexpr int64_t kSmallTilesDefault = 4096;
void spd_lower_inverse_fp64(double *a, int64_t lda, int64_t Np, double *tmp, DevStatus *ds,
                            hipStream_t st, int64_t small = kSmallTilesDefault);
// n x n symmetric positive definite matrix for timing (no padding).
void launch_tuning_matrix(int64_t n, double *a, int64_t lda, hipStream_t st);
// C = alpha op(A) op(B) + beta C in FP64 on the MFMA tile kernels (column-
// major; M, N, K multiples of 64).  at: A stored K x M; bt: B stored N x K;
// lower: only tiles on or below the diagonal (with at and no bt only).
// kmode limits K to the nonzero part of a triangular operand:
enum GemmK {
  kGemmFull = 0,
  kGemmLeN = 1,   // k < (tile_n + 1) 64: B lower triangular, used transposed
  kGemmGeN = 2,   // k >= tile_n 64: B lower triangular
  kGemmLeM = 3,   // k < (tile_m + 1) 64: A lower triangular
  kGemmGeMN = 4,  // k >= max(tile_m, tile_n) 64: A^T B, both lower triangular
};
void gemm_f64(bool at, bool bt, bool lower, int64_t M, int64_t N, int64_t K, const double *A,
              int64_t lda, const double *B, int64_t ldb, double *C, int64_t ldc, double alpha,
              double beta, int kmode, hipStream_t st);
// x = L^-T L^-1 (Np x Np, both triangles) from the in-place inverse factor
// of spd_lower_inverse_fp64 (lower triangle, zero upper part of its diagonal
// tiles).
void spd_inverse_from_factor(const double *linv, int64_t ld, int64_t Np, double *x, int64_t ldx,
                             hipStream_t st);
// Concatenated scenes: identity padding of every scene's matrix, and the
// blocks of every camera (cov: n_cams x 81 in concatenation order).
void launch_pad_identity_scenes(int n_scenes, int64_t max_np, const int32_t *cam_off,
                                const int64_t *a_off, const int64_t *a_ld, double *amat,
                                hipStream_t st);
void launch_extract_scenes(int64_t n_cams, const int32_t *cam_scene, const int32_t *cam_off,
                           const int64_t *a_off, const int64_t *a_ld, const double *amat,
                           const double *s, const double *q, const double *alpha, double *cov,
                           hipStream_t st);
// cov[i] = S_i (Linv^T Linv)_ii S_i - Q_i Q_i^T / alpha (q: N x 7, leading
// dimension ldq; the last term only when subtract is set)
void launch_extract(int64_t N, const double *linv, int64_t ld, const double *s,
                    const double *q, int64_t ldq, const double *alpha, bool subtract, double *cov,
                    hipStream_t st);
// cov[i] = S_i X_ii S_i - Q_i Q_i^T / alpha from a full inverse X
void launch_extract_full(int64_t N, const double *x, int64_t ld, const double *s,
                         const double *q, int64_t ldq, const double *alpha, bool subtract,
                         double *cov, hipStream_t st);

// Mixed precision (all matrices Np x Np, leading dimension Np):
// X0 = L^-T L^-1 of the FP32 Cholesky factor of the lower triangle of a;
void mixed_initial_inverse(int64_t Np, const double *a, int64_t lda, float *a32, float *x32,
                           float *tmp32, DevStatus *ds, hipStream_t st);
// a made symmetric from its lower triangle, x = (double) x32;
void mixed_prepare(int64_t Np, double *a, int64_t lda, const float *x32, double *x,
                   hipStream_t st);
// r = I - a x (FP64), sumsq[0] = |r|_F^2 (sumsq: Np + 1 doubles);
void mixed_residual(int64_t Np, const double *a, int64_t lda, const double *x, double *r,
                    double *sumsq, hipStream_t st);
// x += x r with the correction on FP32 MFMA.
void mixed_update(int64_t Np, double *x, const double *r, float *x32, float *r32, float *d32,
                  hipStream_t st);

// Split-BF16 correction (split_bf16_kernels.hip): x (n x n, leading
// dimension n, n a multiple of 64) += x r with the product formed from
// split_bf16_slices(n) 8-bit slices of x (per row) and r (per column) on BF16
// MFMA, exact FP32 chunk sums accumulated in FP64: 3 slices up to
// kSplitSmallN, 4 beyond (the product's error grows like sqrt(n) times the
// slice truncation); scratch: split_bf16_scratch(n) bytes.
constexpr int64_t kSplitSmallN = 8192;
int split_bf16_slices(int64_t n);
size_t split_bf16_scratch(int64_t n);
void split_bf16_update(int64_t n, double *x, const double *r, void *scratch, hipStream_t st);

// ---- whole covariance (point_kernels.hip) -----------------------------------
// cov (N x N, ld ldc) = S X S - [subtract] Q Q^T / alpha from the scaled
// inverse x (both triangles, ld ldx).
void launch_full_camera(int64_t N, const double *x, int64_t ldx, const double *s,
                        const double *q, const double *alpha, bool subtract, double *cov,
                        int64_t ldc, hipStream_t st);
// Number of column splits of launch_xq; its part buffer holds 7 N splits values.
int64_t xq_splits(int64_t N);
// xq = S x S q (N x 7, ld N) and kmat = q^T xq (7 x 7 row-major).
void launch_xq(int64_t N, const double *x, int64_t ldx, const double *s, const double *q,
               double *part, double *xq, double *kmat, hipStream_t st);
// 3 x 3 covariance of every point (out: m x 9 row-major); b is Q (camera
// gauge) or X q (paper gauge, with lf = L_F and kmat = q^T X q).
void launch_point_cov(const SceneDev &sc, const SceneWork &w, const double *x, int64_t ldx,
                      const double *b, const double *lf, const double *kmat, bool paper,
                      double *out, hipStream_t st);


// ---- incremental update (update_kernels.hip) --------------------------------
// New observations in point-grouped order (position a -> caller's index
// ord[a]): whitened Jacobians nj (k x 24) and the new camera's rows jn
// (kp x 64, zeroed beforehand).
void launch_new_jacobians(const SceneDev &sc, int64_t k, const int32_t *ord,
                          const int32_t *ncam, const int32_t *npt, const double *ninfo,
                          const double *cam_new, double *nj, double *jn, int64_t kp,
                          DevStatus *ds, hipStream_t st);
// Effective rows JtT (np x kp, zeroed) and the lower triangle of their error
// covariance S (kp x kp, zeroed); grp0[a]: first position of a's point.
void launch_new_rows(const SceneDev &sc, const SceneWork &w, int64_t k, const int32_t *ord,
                     const int32_t *ncam, const int32_t *npt, const int32_t *grp0,
                     const double *nj, double *jt, int64_t np, double *S, int64_t kp,
                     DevStatus *ds, hipStream_t st);
void launch_copy_in(int64_t N, int64_t np, const double *src, int64_t ldc, double *zp,
                    hipStream_t st);
void launch_copy_out(int64_t N, int64_t np, const double *zp, double *dst, int64_t ldc,
                     hipStream_t st);
// C_n = (U^T U)^-1 from g = U^T U (64 x 64) and its factor lc; W = V L_C
// (np x 64) and cross = -V C_n (N x 9, when not null).
void launch_new_camera(const double *g, double *cn, double *lc, int64_t N, int64_t np,
                       const double *V, double *W, double *cross, DevStatus *ds, hipStream_t st);

}  // namespace ucov

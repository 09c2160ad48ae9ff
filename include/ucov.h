/*
 * ucov: exact per-camera covariance of a bundle-adjusted reconstruction on
 * AMD Instinct MI355X (gfx950).
 *
 * The library computes, for every camera i of a reconstruction, the 9x9
 * diagonal block of Z^+, the Moore-Penrose inverse of the reduced camera
 * matrix Z = U - W V^-1 W^T (Polic, Forstner, Pajdla, "Fast and Accurate
 * Camera Covariance Computation for Large 3D Reconstruction", ECCV 2018:
 * Sec. 4 for the normal equations and the gauge, Sec. 5.1 for the similarity
 * nullspace, Sec. 5.2 for the block inversion and the Schur complement).
 * Z^+ is evaluated as (Z + a Q Q^T)^-1 - Q Q^T / a with Q an orthonormal basis
 * of the camera rows H_c of the nullspace and a > 0.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every pointer argument is a DEVICE pointer (memory of the context's GPU)
 *   unless its comment says "host".  The caller owns all inputs and outputs;
 *   the context owns its workspace, grows it on demand and frees it in
 *   ucov_destroy.
 * - Work is enqueued on the context's stream (ucov_set_stream; default: the
 *   null stream of the device).  Every entry point returns only after its
 *   work has completed, because it reports device-detected errors.
 * - Return value: UCOV_OK (0) or a negative UCOV_E* code.  On error the
 *   outputs are unspecified; ucov_last_error() describes the failure and
 *   ucov_report.bad_index names the offending observation, point or camera
 *   where there is one.
 * - A context may be used by one host thread at a time.
 * - Matrices are column-major with an explicit leading dimension.
 *
 * Scene layout (all float64 unless stated)
 * ----------------------------------------
 *   cams[9*i + 0..2]   r_i, angle-axis of the world-to-camera rotation R(r_i)
 *   cams[9*i + 3..5]   C_i, camera centre
 *   cams[9*i + 6]      f_i, focal length (pixels)
 *   cams[9*i + 7..8]   k1_i, k2_i, radial distortion
 *   pts[3*j + 0..2]    X_j
 *   obs_cam[o], obs_pt[o]  (int32) camera and point of observation o, any order
 *   obs_info[3*o+0..2] (a, b, c) of the 2x2 information Sigma_u^-1 =
 *                      [[a, b], [b, c]]; NULL means identity
 * The projection is u = f d(rho2) pi + (cx, cy) with pi = x[0:2] / x[2],
 * x = R(r)(X - C), rho2 = |pi|^2 and d = 1 + k1 rho2 + k2 rho2^2 (Sec. 5.1,
 * focal length applied after the division); the principal point is a
 * constant and does not enter the covariance.
 *
 * Input rules (violations return UCOV_EINVAL unless noted): n_cams >= 2,
 * n_pts >= 1, n_obs >= 1; indices in range; finite parameters; positive
 * definite information blocks; no camera observes a point twice; every
 * observed point lies in front of its camera (x[2] > 0); every point has at
 * least two observations (else UCOV_EPOINT).
 */
#ifndef UCOV_H
#define UCOV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define UCOV_OK       0
#define UCOV_EINVAL  (-1) /* malformed input */
#define UCOV_EPOINT  (-2) /* a point block V_j cannot be inverted (bad_index = point) */
#define UCOV_EGAUGE  (-3) /* Z + aQQ^T is not positive definite: the null space of Z is
                             not exactly the 7-dimensional similarity gauge (e.g. a
                             disconnected scene or an unconstrained camera) */
#define UCOV_ENOCONV (-4) /* refinement did not reach the requested tolerance */
#define UCOV_EDEVICE (-5) /* HIP runtime failure */
#define UCOV_ENOMEM  (-6) /* device allocation failed */

/* Precision of the dense inverse (step a4). */
#define UCOV_FP64     0   /* FP64 Cholesky inverse on FP64 MFMA */
#define UCOV_FP32_NS  1   /* FP32 MFMA Cholesky inverse X0 of A_s, then Newton-Schulz steps
                             X <- X + X (I - A_s X): residual in FP64, correction on FP32
                             MFMA; UCOV_ENOCONV if the FP32 factorisation fails or the
                             tolerance is not reached */
#define UCOV_BF16X_NS 2   /* as UCOV_FP32_NS, with each correction X R formed from 8-bit
                             slices of X (per row) and R (per column) on BF16 MFMA: the
                             slice products sum exactly in FP32 over K chunks and the
                             chunks in FP64, so the correction's error (~2^-24 relative to
                             the row and column bounds) does not grow with N */

typedef struct ucov_ctx ucov_ctx;

typedef struct {
  int32_t n_cams;
  int32_t n_pts;
  int64_t n_obs;
  const double *cams;      /* n_cams x 9 */
  const double *pts;       /* n_pts x 3 */
  const int32_t *obs_cam;  /* n_obs */
  const int32_t *obs_pt;   /* n_obs */
  const double *obs_info;  /* n_obs x 3 or NULL */
} ucov_scene;

/* Gauge of the covariance.
 * UCOV_GAUGE_CAMERA: Z^+, the Moore-Penrose inverse of the reduced camera
 *   matrix (camera parameters orthogonal to the similarity nullspace).
 * UCOV_GAUGE_PAPER: (M^+)_cc, the camera block of the Moore-Penrose inverse
 *   of the full information matrix (Sec. 4: the whole parameter vector,
 *   points included, orthogonal to the nullspace; Sec. 5.2: the points
 *   eliminated by block inversion).  Evaluated as (Z + G F^-1 G^T)^-1 with
 *   G = H_c - W V^-1 H_p and F = H_p^T V^-1 H_p, H_p the point rows of the
 *   nullspace.  The two agree after projection: Z^+ = P_c (M^+)_cc P_c with
 *   P_c the projector onto the complement of range(H_c); their intrinsics
 *   blocks coincide. */
#define UCOV_GAUGE_CAMERA 0
#define UCOV_GAUGE_PAPER  1

typedef struct {
  int32_t precision;  /* UCOV_FP64, UCOV_FP32_NS or UCOV_BF16X_NS */
  int32_t max_iter;   /* Newton-Schulz iterations allowed (mixed precision); 0 = default 6 */
  double tol;         /* Newton-Schulz stop: |I - A X|_F / sqrt(N) <= tol; 0 = default 1e-10 */
  double alpha;       /* gauge weight a; 0 = balanced automatic choice (UCOV_GAUGE_CAMERA only) */
  int32_t gauge;      /* UCOV_GAUGE_CAMERA (default) or UCOV_GAUGE_PAPER */
  uint32_t flags;     /* UCOV_HOST_PTRS or 0 */
} ucov_options;

/* Options flag: the scene's arrays and the output of ucov_camera_covariance
 * (and of its allocation-free variant) are HOST memory.  The library stages
 * them through device buffers of its workspace (copies on the context's
 * stream; the call returns with the output on the host).  The other entry
 * points take device pointers only (UCOV_EINVAL with this flag). */
#define UCOV_HOST_PTRS 1u

typedef struct {
  double alpha;        /* gauge weight used */
  int32_t bad_index;   /* offending observation / point / camera, -1 if none */
  int32_t ns_iters;    /* Newton-Schulz iterations performed */
  double ns_residual;  /* final |I - A X|_F / sqrt(N) (mixed precision only) */
  int64_t n_pairs;     /* (observation, observation) pairs in the Schur scatter */
  /* stage times in milliseconds, measured with HIP events on the stream
   * (host round trips inside a stage count towards it) */
  float ms_structure;  /* grouping the observations by point, camera-pair binning */
  float ms_schur;      /* Jacobians, point blocks, diagonal camera blocks with the
                          rotation rows of the nullspace, assembly of the scaled
                          Z + aQQ^T (steps a1, a2) */
  float ms_gauge;      /* orthonormal gauge basis, weight and scaling (step a3) */
  float ms_inverse;    /* dense factorisation and inversion (step a4) */
  float ms_extract;    /* covariance block extraction (step a4) */
  int32_t bad_scene;   /* batched calls: scene of the failure, -1 if none */
  float ms_total;      /* the whole call on the stream, HIP events */
} ucov_report;

/* Create a context on HIP device `device`.  Returns UCOV_EDEVICE if the
 * device cannot be selected. */
int ucov_create(ucov_ctx **ctx, int device);

/* Use `stream` (a hipStream_t; NULL = null stream) for subsequent calls. */
int ucov_set_stream(ucov_ctx *ctx, void *stream);

/* Release the context and its workspace. */
void ucov_destroy(ucov_ctx *ctx);

/* Per-camera covariance blocks, the whole hot path (steps a1-a4).
 * cov_out: n_cams x 81 float64, block i row-major at cov_out + 81*i; it is
 * the diagonal block of Z^+ (or of (M^+)_cc with UCOV_GAUGE_PAPER) for the
 * parameters (r, C, f, k1, k2) of camera i.
 * opt may be NULL (defaults); rep may be NULL. */
int ucov_camera_covariance(ucov_ctx *ctx, const ucov_scene *scene,
                           const ucov_options *opt, double *cov_out,
                           ucov_report *rep);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * computation as ucov_camera_covariance in UCOV_FP64 (either gauge), with
 * every work buffer carved from one static device array of
 * UCOV_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends, instead of the context's workspace.  The call makes
 * no hipMalloc, hipFree or other allocating call; the context (made by
 * ucov_create, which does allocate) supplies its status word, pinned
 * readback scalars and events.  The caller passes inputs and outputs as for
 * ucov_camera_covariance.
 * Limits and errors: UCOV_ENOMEM (nothing is launched past the failing stage,
 * cov_out unspecified) when the scene's work buffers exceed the scratch --
 * roughly 8 Np^2 * 1.5 bytes for the dense stage (Np = 9 n_cams rounded up to
 * 64) plus about 300 bytes per observation and 8 bytes per observation pair,
 * e.g. scenes up to ~1500 cameras with a few hundred thousand observations;
 * UCOV_EINVAL for any precision other than UCOV_FP64.
 * Every call on one GPU shares that GPU's array (whatever context it comes
 * from) and leaves its contents behind; each call clears what it needs.
 * Calls that overlap on one GPU (two host threads, or two streams in flight)
 * race on the array: serialise them. */
#define UCOV_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int ucov_camera_covariance_noalloc(ucov_ctx *ctx, const ucov_scene *scene,
                                   const ucov_options *opt, double *cov_out,
                                   ucov_report *rep);

/* The whole camera covariance and the covariance of every point (Sec. 5.2:
 * the points are eliminated by block inversion, M = L diag(Z, V) L^T with
 * L = [[I, W V^-1], [0, I]], and their blocks recovered from the camera
 * covariance X; the sum runs over the point's observations only).
 *   UCOV_GAUGE_CAMERA: X = Z^+ and the block of point j is
 *     V_j^-1 + V_j^-1 W_j^T Z^+ W_j V_j^-1
 *     (the generalised inverse of M whose null space holds the similarity
 *     directions of the cameras alone);
 *   UCOV_GAUGE_PAPER: X = (M^+)_cc and the block is the point block of M^+.
 * cam_cov: N x N float64 column-major with leading dimension ldc >= N
 * (N = 9 n_cams), both triangles, or NULL; its diagonal blocks are those of
 * ucov_camera_covariance.  pt_cov: n_pts x 9 float64 (row-major 3 x 3 per
 * point), or NULL; not both NULL (UCOV_EINVAL).  Device arrays.
 * opt->precision must be UCOV_FP64.  Device workspace: two Np x Np float64
 * matrices (Np = N rounded up to 64) besides the scene's.
 * rep: ms_inverse covers the factorisation and the product L^-T L^-1,
 * ms_extract the output kernels. */
int ucov_full_covariance(ucov_ctx *ctx, const ucov_scene *scene, const ucov_options *opt,
                         double *cam_cov, int64_t ldc, double *pt_cov, ucov_report *rep);

/* Incremental update (Sec. 6): the whole camera covariance after adding
 * observations to the scene, from the covariance before, by the Woodbury
 * identity (in its corrected form
 * (Z + J^T W J)^-1 = Z^-1 - Z^-1 J^T (W^-1 + J Z^-1 J^T)^-1 J Z^-1).  A new
 * observation of an existing point acts on the cameras, once the point is
 * eliminated, as the rows J_c - J_x V_j^-1 W_j^T with error covariance
 * Lambda^-1 + J_x V_j^-1 J_x^T (shared between new observations of one
 * point).  Observations may come from existing cameras or from one new
 * camera, which is then eliminated as well (flat prior): the old cameras keep
 * their gauge (the similarity of the old cameras held fixed).
 * scene: the reconstruction before the addition (its rules as for
 * ucov_camera_covariance).  n_new >= 1 observations, device arrays:
 * new_cam[k] in [0, n_cams] (n_cams = the new camera, only with cam_new),
 * new_pt[k] in [0, n_pts), new_info (n_new x 3 as obs_info, or NULL for
 * identity).  No camera may observe a point twice (UCOV_EINVAL, rep->bad_index
 * the new observation).  cam_new: 9 parameters of the new camera (device), or
 * NULL; if given, some new observation must use it.
 * cam_cov: in, the scene's whole camera covariance in the camera gauge
 * (N x N column-major, leading dimension ldc >= N, N = 9 n_cams, as
 * ucov_full_covariance writes it); out, the covariance of the same cameras
 * after the addition.  new_cov (9 x 9 row-major) and new_cross (N x 9
 * row-major: old parameter, new-camera parameter) receive the new camera's
 * covariance and its cross-covariance with the old cameras, or are NULL;
 * UCOV_EGAUGE when the new camera's observations do not determine it.  On
 * any error cam_cov is left as it was.
 * Device workspace: an Np x Np matrix and three Np x Kp ones (Np = N, Kp =
 * 2 n_new, each rounded up to 64).
 * rep: ms_schur covers the new rows, ms_inverse the Woodbury products,
 * ms_extract the copy back. */
int ucov_update_covariance(ucov_ctx *ctx, const ucov_scene *scene, int64_t n_new,
                           const int32_t *new_cam, const int32_t *new_pt, const double *new_info,
                           const double *cam_new, double *cam_cov, int64_t ldc, double *new_cov,
                           double *new_cross, ucov_report *rep);

/* Tune the dense stage's tile schedule for matrices of size n (N = 9 n_cams
 * of a scene): the recursion's products run on 128 x 128, 64 x 64 or 32 x 32
 * MFMA tiles depending on their size (a product with at least 512 tiles of
 * 128 x 128, a recursion node's paired launch with 1024, always on those; the
 * threshold below decides between the other two); every candidate threshold
 * is timed on a synthetic positive definite matrix of the padded size and the
 * fastest is kept in this context for that size (used by
 * ucov_camera_covariance and ucov_full_covariance in UCOV_FP64).  Results are unchanged by the choice up
 * to rounding order.  threshold (HOST, or NULL): the chosen number of 64 x 64
 * tiles below which products use 32 x 32 tiles; ms (HOST, or NULL): its dense
 * stage time.  Allocates the dense workspace for that size. */
int ucov_tune_dense(ucov_ctx *ctx, int64_t n, int64_t *threshold, float *ms);

/* Tune the batched dense stage (ucov_camera_covariance_batched) for scenes
 * whose matrices have sizes n[0..count) (N = 9 n_cams per scene, in the
 * batch's scene order): each launch of the batched recursion serves one node
 * for all scenes that reach it, and launches with fewer 64 x 64 tiles in all
 * than the threshold run on split 32 x 32 tiles.  Every candidate is timed on
 * synthetic positive definite matrices of those sizes (best of three) and the
 * fastest is kept in this context for batches of exactly these sizes (an
 * untuned batch runs every product on 64 x 64 tiles).  threshold, ms: HOST,
 * or NULL.  Results are unchanged by the choice up to rounding order. */
int ucov_tune_batched(ucov_ctx *ctx, int32_t count, const int64_t *n, int64_t *threshold,
                      float *ms);

/* Set the tile-schedule threshold of ucov_tune_dense for matrices of size n
 * without timing (e.g. one a previous tuning chose), in this context. */
int ucov_set_dense_threshold(ucov_ctx *ctx, int64_t n, int64_t threshold);

/* Covariance blocks of several independent scenes in one call: the
 * sub-reconstructions of Sec. 6, each evaluated exactly on its own gauge (a
 * camera's covariance from a sub-reconstruction around it bounds the one from
 * the whole reconstruction from above).
 * scenes: HOST array of n_scenes descriptors (n_scenes >= 1); the arrays each
 * descriptor points to are device arrays whose indices are local to that
 * scene.  The input rules of ucov_camera_covariance hold per scene.
 * cov_out: (sum of n_cams) x 81 float64; the blocks of scene s follow those of
 * scene s - 1, each as in ucov_camera_covariance.
 * alphas: HOST array receiving the gauge weight of every scene, or NULL.
 * opt->precision must be UCOV_FP64 and opt->gauge UCOV_GAUGE_CAMERA (else
 * UCOV_EINVAL).
 * rep: ms_inverse covers the dense stage of all scenes (identity padding,
 * the batched factorisation and inversion), ms_extract the block extraction,
 * alpha is scene 0's; on failure bad_scene names the scene and bad_index the
 * observation, point or camera within it.
 * Limits: at most 2^27 cameras and 2^31 - 1 points and observations in total. */
int ucov_camera_covariance_batched(ucov_ctx *ctx, int32_t n_scenes, const ucov_scene *scenes,
                                   const ucov_options *opt, double *cov_out, double *alphas,
                                   ucov_report *rep);

/* A batch of independent scenes (as for ucov_camera_covariance_batched)
 * recorded once and replayed: ucov_batch_create solves the batch eagerly in
 * a private workspace (validating every scene, sizing every buffer, building
 * the dense plan; cov_out then holds the blocks), then records the same
 * launches, with no host round trip, into a HIP graph.  ucov_batch_run
 * replays the graph on the context's current stream and checks the status;
 * cov_out is rewritten.  Between runs the scenes' parameter values
 * (cams, pts, obs_info) may change, their sizes and index arrays may not: a
 * run whose camera-pair structure grew beyond the recorded one returns
 * UCOV_EINVAL without writing out of its buffers.  The scenes' device arrays
 * and cov_out must outlive the batch.  rep of a run: alpha, n_pairs,
 * bad_scene / bad_index on failure, ms_total (the graph's time); the stage
 * times are 0.  The batch holds its own device workspace (as much as the
 * batched call) until ucov_batch_destroy; runs of one batch must not overlap. */
typedef struct ucov_batch ucov_batch;
int ucov_batch_create(ucov_ctx *ctx, int32_t n_scenes, const ucov_scene *scenes,
                      const ucov_options *opt, double *cov_out, ucov_batch **batch);
int ucov_batch_run(ucov_batch *batch, ucov_report *rep);
void ucov_batch_destroy(ucov_batch *batch);

/* Sub-reconstructions (Sec. 6): each camera's covariance evaluated from
 * sub-reconstructions around it instead of the whole scene.  A sub-
 * reconstruction is a group of cameras with the points that at least two of
 * its cameras observe and those observations; each is solved exactly on its
 * own gauge (one batched call for all of them).  The scene is decomposed
 * n_decomp times and every camera keeps the block with the smallest trace
 * among the sub-reconstructions that contain it.
 * groups: HOST array n_decomp x n_cams; groups[d * n_cams + i] is camera i's
 * group in decomposition d (any ids in [0, n_cams)); every group needs at
 * least two cameras and a connected, non-degenerate sub-scene, else the
 * batched call's error is returned with rep->bad_scene naming the
 * sub-reconstruction (in the order decomposition, then group by its first
 * camera).
 * cov_out: n_cams x 81 as in ucov_camera_covariance.  chosen: HOST array of
 * n_cams receiving the decomposition whose block was kept, or NULL.  n_sub:
 * HOST, receives the number of sub-reconstructions, or NULL.  opt as for
 * ucov_camera_covariance_batched. */
int ucov_subrecon_covariance(ucov_ctx *ctx, const ucov_scene *scene, int32_t n_decomp,
                             const int32_t *groups, const ucov_options *opt, double *cov_out,
                             int32_t *chosen, int32_t *n_sub, ucov_report *rep);

/* Step a1 alone: per-observation Jacobian blocks of the projection (Sec. 5.1),
 * in the caller's observation order, unweighted by obs_info.
 * jp: n_obs x 18 (2x9 row-major per observation, columns r, C, f, k1, k2);
 * jx: n_obs x 6 (2x3 row-major per observation). */
int ucov_jacobians(ucov_ctx *ctx, const ucov_scene *scene, double *jp, double *jx);

/* Steps a1-a2: the reduced camera matrix Z = U - W V^-1 W^T (Sec. 5.2,
 * Schur complement of the point block), written densely (both triangles)
 * into z, an N x N column-major matrix with leading dimension ldz >= N,
 * N = 9 n_cams. */
int ucov_reduced_camera_matrix(ucov_ctx *ctx, const ucov_scene *scene,
                               double *z, int64_t ldz, ucov_report *rep);

/* Step a3: the camera rows H_c of the similarity nullspace (Sec. 5.1,
 * column order translation, rotation, scale; rotation block from
 * J_r H_r = B) and an orthonormal basis Q of their span.
 * hc, q: N x 7 column-major with leading dimension N (either may be NULL). */
int ucov_gauge_basis(ucov_ctx *ctx, const ucov_scene *scene, double *hc, double *q);

/* Step a4 alone: diagonal 9x9 blocks of Z^+ = (Z + a QQ^T)^-1 - QQ^T/a for a
 * caller-supplied symmetric positive semi-definite z (N x N, column-major,
 * leading dimension ldz, only the lower triangle is read) whose null space is
 * spanned by the orthonormal columns of q (N x 7, leading dimension N).
 * N must be a multiple of 9.  alpha <= 0 selects the balanced weight.
 * cov_out: (N/9) x 81 as in ucov_camera_covariance. */
int ucov_pinv_blocks(ucov_ctx *ctx, int64_t n, const double *z, int64_t ldz,
                     const double *q, const ucov_options *opt, double *cov_out,
                     ucov_report *rep);

/* Step a4's split-BF16 product alone (the correction of UCOV_BF16X_NS):
 * x += x r for n x n column-major float64 x and r (leading dimension n, n a
 * positive multiple of 64).  Entry (m, c) of the product carries at most
 * about 2^(e_m + f_c - 24) n error, 2^e_m and 2^f_c the powers of two that
 * bound row m of x and column c of r. */
int ucov_split_bf16_update(ucov_ctx *ctx, int64_t n, double *x, const double *r);

/* ---- learned screener -----------------------------------------------------
 * A small network that predicts a camera's 9x9 covariance from 55 cheap
 * features, for screening cameras by their uncertainty (the paper's Sec. 1
 * names filtering weakly constrained cameras as a use of the covariance).  It
 * is not part of the paper's method: its labels come from
 * ucov_camera_covariance, which stays the reference for its error.
 *
 * Network: 55 -> 256 -> 256 -> 256 -> 45, ReLU between layers, linear
 * output.  Parameters are one float32 vector of ucov_mlp_param_count()
 * values: for each layer W (out x in, row-major) then b (out).  Products
 * round their operands to bfloat16 and accumulate in float32; hidden
 * activations are stored in bfloat16.  Inputs are standardised as
 * (x - in_mean) / in_std per feature when both are given.  All arrays are
 * device arrays, row-major per sample. */
#define UCOV_SCREENER_FEATURES 55
#define UCOV_SCREENER_OUTPUTS  45

int64_t ucov_mlp_param_count(void);

/* Per-camera features (n_cams x 55 float32): 45 from the diagonal block Z_ii
 * of the reduced camera matrix (Sec. 5.2; log10 of its 9 diagonal entries,
 * then its 36 correlations, row-major upper triangle), log(1 + count) of the
 * camera's observations in the track-length bins 2, 3, 4, 5, 6-7, 8-10, 11-15,
 * >= 16, the mean over its observations of the largest angle (rad) between
 * its ray and another track camera's ray to the point, and log(1 + number of
 * cameras sharing a point with it).  Input rules as ucov_camera_covariance. */
int ucov_screener_features(ucov_ctx *ctx, const ucov_scene *scene, float *feat);

/* y (batch x 45) = network(x (batch x 55)).  in_mean / in_std: 55 values each,
 * or both NULL. */
int ucov_mlp_forward(ucov_ctx *ctx, const float *params, int64_t batch, const float *x,
                     const float *in_mean, const float *in_std, float *y);

/* Gradient (ucov_mlp_param_count() values) of the mean squared error
 * mean((network(x) - target)^2) over batch x 45 outputs; loss: device scalar
 * or NULL. */
int ucov_mlp_gradient(ucov_ctx *ctx, const float *params, int64_t batch, const float *x,
                      const float *in_mean, const float *in_std, const float *target,
                      float *grad, float *loss);

/* n_batches Adam steps (beta1 0.9, beta2 0.999, eps 1e-8; step counts start
 * at step0 >= 1 for the bias correction) on consecutive batches of x and
 * target (n_batches * batch rows each), updating params and the moment
 * vectors adam_m, adam_v (zero before the first step) in place.  losses:
 * n_batches device floats (the loss of each batch before its step) or NULL. */
int ucov_mlp_train(ucov_ctx *ctx, float *params, float *adam_m, float *adam_v, int64_t step0,
                   float lr, int64_t batch, int64_t n_batches, const float *x,
                   const float *in_mean, const float *in_std, const float *target,
                   float *losses);

/* The label scale.  Each camera's covariance is measured against its
 * block-diagonal estimate (Z_ii)^-1, which its own features determine: b_a =
 * sqrt(((Z_ii)^-1)_aa) (a = 0..8), with Z_ii rebuilt from the camera's first
 * 45 features (the correlation matrix must be positive definite), and the
 * per-camera scale is D_a = scale_a b_a, scale (9 float64) a training-set
 * statistic (ucov_screener_stats).  The normalised covariance is
 * D^-1 Sigma D^-1. */

/* Training labels: for each of n covariance blocks (n x 81 float64,
 * row-major) with the features of the same cameras (n x 55 float32), the 45
 * log-Cholesky parameters of the normalised covariance D^-1 Sigma D^-1 =
 * L L^T (log L_aa on the diagonal, L_ab below it, row-major lower triangle),
 * standardised as (p - out_mean) / out_std and clipped to [-6, 6] (a camera
 * that the other cameras barely constrain has parameters far outside the
 * rest, which would otherwise dominate the training loss).  UCOV_EINVAL if a
 * block or a camera's Z_ii correlation matrix is not positive definite
 * (bad_index: the camera). */
int ucov_screener_labels(ucov_ctx *ctx, int64_t n, const double *cov, const float *feat,
                         const double *scale, const float *out_mean, const float *out_std,
                         float *labels);

/* The inverse map: network outputs y (n x 45) and the cameras' features
 * (n x 55) -> covariance blocks D L L^T D (n x 81, may be NULL) and the
 * spread trace(L L^T) of the normalised covariance (n, may be NULL).
 * UCOV_EINVAL if a camera's Z_ii correlation matrix is not positive
 * definite. */
int ucov_screener_covariance(ucov_ctx *ctx, int64_t n, const float *y, const float *feat,
                             const double *scale, const float *out_mean, const float *out_std,
                             double *cov, double *spread);

/* Standardisation statistics of a training set of n >= 2 cameras: feat
 * (n x 55) and their exact covariance blocks cov (n x 81).  in_mean, in_std
 * (55 each): per feature the mean and the standard deviation (n - 1 in the
 * denominator, at least 1e-6); scale (9): per parameter a the square root of
 * the lower median (rank (n - 1) / 2 ascending) over the blocks of the
 * variance ratio Sigma_aa / b_a^2; out_mean, out_std (45 each): per
 * log-Cholesky parameter p of the normalised covariances (as FP32) its lower
 * median m and 1.4826 times the lower median of |p - m| (the median absolute
 * deviation, scaled to a normal distribution's standard deviation; at least
 * 1e-6).  Every sum runs in a fixed order and the medians are exact order
 * statistics (the same bits on every call).  UCOV_EINVAL if a block is not
 * positive definite. */
int ucov_screener_stats(ucov_ctx *ctx, int64_t n, const float *feat, const double *cov,
                        float *in_mean, float *in_std, double *scale, float *out_mean,
                        float *out_std);

/* A trained screener: its parameters, statistics and (optionally) the Adam
 * state to resume training.  All arrays are device arrays of the sizes given. */
typedef struct {
  float *params;    /* ucov_mlp_param_count() */
  float *in_mean;   /* 55 */
  float *in_std;    /* 55 */
  double *scale;    /* 9 */
  float *out_mean;  /* 45 */
  float *out_std;   /* 45 */
  float *adam_m;    /* ucov_mlp_param_count(), or NULL (then adam_v NULL too) */
  float *adam_v;    /* ucov_mlp_param_count(), or NULL */
  int64_t step;     /* Adam steps taken so far (host value) */
} ucov_screener;

/* Write the screener to a file (host path): a 64-byte header (magic
 * "UCOVSCR1", version 1, the network's sizes, whether the Adam moments are
 * stored, the parameter count and step), then params, in_mean, in_std,
 * out_mean, out_std (float32), scale (float64), adam_m, adam_v (float32, when
 * given), then a 64-bit FNV-1a hash of that payload; little-endian.  The
 * context's stream is synchronised first.  UCOV_EINVAL on a bad argument or
 * an I/O failure. */
int ucov_screener_save(ucov_ctx *ctx, const char *path, const ucov_screener *s);

/* Read a file written by ucov_screener_save into the caller's device arrays
 * (s->adam_m and s->adam_v may be NULL to skip the Adam moments; asking for
 * them from a file without them is UCOV_EINVAL) and set s->step.  UCOV_EINVAL
 * when the file is missing, of another network, truncated or its hash does
 * not match. */
int ucov_screener_load(ucov_ctx *ctx, const char *path, ucov_screener *s);

/* Diagnostic, host only (no device needed): builds the launch plan that the
 * batched entry point uses for matrices of padded sizes np[0..count)
 * (multiples of 64) and checks that every product and leaf stays inside its
 * matrix or scratch and that every 64-column block is factored exactly once.
 * UCOV_OK when it holds, UCOV_EDEVICE when not, UCOV_EINVAL for bad sizes.
 * n_launches (may be NULL) receives the number of kernel launches. */
int ucov_plan_check(const int64_t *np, int32_t count, int64_t *n_launches);

/* Text for an error code; description of the last failure on this context. */
const char *ucov_strerror(int code);
const char *ucov_last_error(const ucov_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* UCOV_H */

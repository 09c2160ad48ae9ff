// C-ABI of the ucov library: context, workspace and the sequence of stages.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "ucov_internal.h"
#include "../../include/ucov.h"

using namespace ucov;

namespace {

struct Buf {
  void *p = nullptr;
  size_t cap = 0;
};

const char *code_name(int code) {
  switch (code) {
    case UCOV_OK: return "ok";
    case UCOV_EINVAL: return "invalid input";
    case UCOV_EPOINT: return "point block cannot be inverted";
    case UCOV_EGAUGE: return "regularised camera matrix is not positive definite";
    case UCOV_ENOCONV: return "refinement did not converge";
    case UCOV_EDEVICE: return "HIP runtime failure";
    case UCOV_ENOMEM: return "device allocation failed";
    default: return "unknown error";
  }
}

}  // namespace

struct ucov_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  DevStatus *ds = nullptr;       // device
  DevStatus *ds_host = nullptr;  // pinned host mirror
  int64_t *i64_host = nullptr;   // pinned host scalars [0] pairs, [1] non-empty bins
  int64_t n_nonzero = 0;         // non-empty bins of the last scene stage
  hipEvent_t ev[8] = {};
  // workspace
  Buf cnt_p, ptr_p, cur_p, slot_obs, slot_cam, slot_pt, rec;
  Buf bin_cnt, bin_ptr, bin_cur, pairs, scan_tmp, nzlist, nzcount;
  Buf zdiag, hc, q, s, alpha, amat, tmat;
  Buf m_a32, m_x32, m_r32, m_d32, m_tmp32, m_x64, m_r64, m_sum;  // mixed precision

  int fail(int code, const std::string &msg) {
    last_error = std::string(code_name(code)) + ": " + msg;
    return code;
  }
};

namespace {

int ensure(ucov_ctx *c, Buf &b, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (b.cap >= bytes) return UCOV_OK;
  if (b.p) hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
  if (hipMalloc(&b.p, bytes) != hipSuccess) {
    hipGetLastError();
    return c->fail(UCOV_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  b.cap = bytes;
  return UCOV_OK;
}

template <class T>
T *as(Buf &b) {
  return reinterpret_cast<T *>(b.p);
}

#define UCOV_TRY(expr)          \
  do {                          \
    int _rc = (expr);           \
    if (_rc != UCOV_OK) return _rc; \
  } while (0)

int check_hip(ucov_ctx *c, const char *where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return c->fail(UCOV_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
  return UCOV_OK;
}

// Wait for the stream and translate the device status into a return code.
int sync_status(ucov_ctx *c, ucov_report *rep, const char *where) {
  if (hipMemcpyAsync(c->ds_host, c->ds, sizeof(DevStatus), hipMemcpyDeviceToHost, c->stream) !=
          hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    hipError_t e = hipGetLastError();
    return c->fail(UCOV_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
  }
  if (rep) rep->bad_index = c->ds_host->index;
  if (c->ds_host->code != 0) {
    char buf[160];
    snprintf(buf, sizeof buf, "%s (index %d)", where, c->ds_host->index);
    return c->fail(c->ds_host->code, buf);
  }
  return UCOV_OK;
}

int check_scene(ucov_ctx *c, const ucov_scene *s) {
  if (!s) return c->fail(UCOV_EINVAL, "scene is NULL");
  if (s->n_cams < 2 || s->n_pts < 1 || s->n_obs < 1)
    return c->fail(UCOV_EINVAL, "need n_cams >= 2, n_pts >= 1, n_obs >= 1");
  if (s->n_obs >= (int64_t)1 << 31)
    return c->fail(UCOV_EINVAL, "n_obs must be below 2^31");
  if (!s->cams || !s->pts || !s->obs_cam || !s->obs_pt)
    return c->fail(UCOV_EINVAL, "NULL scene array");
  return UCOV_OK;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Steps a1-a2 up to the per-camera diagonal blocks and the nullspace rows.
// On return the slot records, pair bins, zdiag and hc are valid.
int run_scene_stage(ucov_ctx *c, const ucov_scene *scene, double *jp_out, double *jx_out,
                    bool jac_only, ucov_report *rep) {
  SceneDev sc;
  sc.n = scene->n_cams;
  sc.m = scene->n_pts;
  sc.t = scene->n_obs;
  sc.cams = scene->cams;
  sc.pts = scene->pts;
  sc.info = scene->obs_info;
  sc.oc = scene->obs_cam;
  sc.op = scene->obs_pt;
  const int64_t n = sc.n, m = sc.m, t = sc.t;
  const int64_t N = 9 * n;
  const int64_t nbins = n * (n + 1) / 2;
  const int64_t scan_tiles = (std::max(nbins, m) + 4095) / 4096 + 2;
  UCOV_TRY(ensure(c, c->cnt_p, 4 * m));
  UCOV_TRY(ensure(c, c->ptr_p, 8 * (m + 1)));
  UCOV_TRY(ensure(c, c->cur_p, 4 * m));
  UCOV_TRY(ensure(c, c->slot_obs, 4 * t));
  UCOV_TRY(ensure(c, c->slot_cam, 4 * t));
  UCOV_TRY(ensure(c, c->slot_pt, 4 * t));
  UCOV_TRY(ensure(c, c->rec, 8 * kRec * t));
  UCOV_TRY(ensure(c, c->scan_tmp, 8 * scan_tiles));
  SceneWork w{};
  w.cnt_p = as<int32_t>(c->cnt_p);
  w.ptr_p = as<int64_t>(c->ptr_p);
  w.cur_p = as<int32_t>(c->cur_p);
  w.slot_obs = as<int32_t>(c->slot_obs);
  w.slot_cam = as<int32_t>(c->slot_cam);
  w.slot_pt = as<int32_t>(c->slot_pt);
  w.rec = as<double>(c->rec);
  w.scan_tmp = as<int64_t>(c->scan_tmp);
  hipStream_t st = c->stream;

  hipEventRecord(c->ev[0], st);
  fill_i32(reinterpret_cast<int32_t *>(c->ds), 0, 2, st);
  fill_i32(w.cnt_p, 0, m, st);
  fill_i32(w.cur_p, 0, m, st);
  launch_count_points(sc, w, c->ds, st);
  exclusive_scan(w.cnt_p, w.ptr_p, m, w.scan_tmp, st);
  launch_group_points(sc, w, c->ds, st);
  launch_jacobians(sc, w, jp_out, jx_out, c->ds, st);
  UCOV_TRY(check_hip(c, "jacobian kernels"));
  if (jac_only) return sync_status(c, rep, "jacobians");

  UCOV_TRY(ensure(c, c->bin_cnt, 4 * nbins));
  UCOV_TRY(ensure(c, c->bin_ptr, 8 * (nbins + 1)));
  UCOV_TRY(ensure(c, c->bin_cur, 4 * nbins));
  UCOV_TRY(ensure(c, c->nzlist, sizeof(int2) * nbins));  // at most one entry per bin
  UCOV_TRY(ensure(c, c->nzcount, 8));
  w.bin_cnt = as<int32_t>(c->bin_cnt);
  w.bin_ptr = as<int64_t>(c->bin_ptr);
  w.bin_cur = as<int32_t>(c->bin_cur);
  w.nzlist = as<int2>(c->nzlist);
  w.nzcount = as<int64_t>(c->nzcount);
  launch_point_blocks(sc, w, c->ds, st);
  fill_i32(w.bin_cnt, 0, nbins, st);
  fill_i32(w.bin_cur, 0, nbins, st);
  fill_i32(reinterpret_cast<int32_t *>(w.nzcount), 0, 2, st);
  launch_pair_count(sc, w, st);
  exclusive_scan(w.bin_cnt, w.bin_ptr, nbins, w.scan_tmp, st);
  UCOV_TRY(check_hip(c, "point kernels"));
  // the pair count sizes the next buffer: one host round trip
  hipMemcpyAsync(c->i64_host, w.bin_ptr + nbins, sizeof(int64_t), hipMemcpyDeviceToHost, st);
  hipMemcpyAsync(c->i64_host + 1, w.nzcount, sizeof(int64_t), hipMemcpyDeviceToHost, st);
  UCOV_TRY(sync_status(c, rep, "point blocks"));
  const int64_t npairs = c->i64_host[0];
  c->n_nonzero = c->i64_host[1];
  if (rep) rep->n_pairs = npairs;
  UCOV_TRY(ensure(c, c->pairs, sizeof(int2) * npairs));
  UCOV_TRY(ensure(c, c->zdiag, 8 * 81 * n));
  UCOV_TRY(ensure(c, c->hc, 8 * 7 * N));
  w.pairs = as<int2>(c->pairs);
  w.zdiag = as<double>(c->zdiag);
  w.hc = as<double>(c->hc);
  launch_pair_fill(sc, w, st);
  hipEventRecord(c->ev[1], st);
  launch_camera_diag(sc, w, c->ds, st);
  UCOV_TRY(check_hip(c, "schur kernels"));
  return UCOV_OK;
}

SceneWork scene_work(ucov_ctx *c) {
  SceneWork w{};
  w.cnt_p = as<int32_t>(c->cnt_p);
  w.ptr_p = as<int64_t>(c->ptr_p);
  w.cur_p = as<int32_t>(c->cur_p);
  w.slot_obs = as<int32_t>(c->slot_obs);
  w.slot_cam = as<int32_t>(c->slot_cam);
  w.slot_pt = as<int32_t>(c->slot_pt);
  w.rec = as<double>(c->rec);
  w.bin_cnt = as<int32_t>(c->bin_cnt);
  w.bin_ptr = as<int64_t>(c->bin_ptr);
  w.bin_cur = as<int32_t>(c->bin_cur);
  w.pairs = as<int2>(c->pairs);
  w.nzlist = as<int2>(c->nzlist);
  w.nzcount = as<int64_t>(c->nzcount);
  w.zdiag = as<double>(c->zdiag);
  w.hc = as<double>(c->hc);
  w.q = as<double>(c->q);
  w.s = as<double>(c->s);
  w.alpha = as<double>(c->alpha);
  w.scan_tmp = as<int64_t>(c->scan_tmp);
  return w;
}

SceneDev scene_dev(const ucov_scene *scene) {
  SceneDev sc;
  sc.n = scene->n_cams;
  sc.m = scene->n_pts;
  sc.t = scene->n_obs;
  sc.cams = scene->cams;
  sc.pts = scene->pts;
  sc.info = scene->obs_info;
  sc.oc = scene->obs_cam;
  sc.op = scene->obs_pt;
  return sc;
}

void fill_defaults(const ucov_options *opt, ucov_options &o) {
  o.precision = UCOV_FP64;
  o.max_iter = 6;
  o.tol = 1e-10;
  o.alpha = 0.0;
  if (opt) {
    o.precision = opt->precision;
    if (opt->max_iter > 0) o.max_iter = opt->max_iter;
    if (opt->tol > 0) o.tol = opt->tol;
    o.alpha = opt->alpha;
  }
}

// Mixed-precision inverse of A_s (Np x Np in c->amat): FP32 MFMA Cholesky
// inverse X0, then Newton-Schulz steps X <- X + X (I - A X) with the residual
// in FP64 and the correction on FP32 MFMA, until |I - A X|_F / sqrt(N) <= tol.
int run_mixed(ucov_ctx *c, int64_t N, int64_t Np, const ucov_options &o, double *cov_out,
              ucov_report *rep) {
  hipStream_t st = c->stream;
  const size_t f32 = 4 * (size_t)Np * Np, f64 = 8 * (size_t)Np * Np;
  UCOV_TRY(ensure(c, c->m_a32, f32));
  UCOV_TRY(ensure(c, c->m_x32, f32));
  UCOV_TRY(ensure(c, c->m_r32, f32));
  UCOV_TRY(ensure(c, c->m_d32, f32));
  UCOV_TRY(ensure(c, c->m_tmp32, 4 * std::max<int64_t>(1, spd_lower_inverse_scratch(Np))));
  UCOV_TRY(ensure(c, c->m_x64, f64));
  UCOV_TRY(ensure(c, c->m_r64, f64));
  UCOV_TRY(ensure(c, c->m_sum, 8));
  double *A = as<double>(c->amat);
  mixed_initial_inverse(Np, A, Np, as<float>(c->m_a32), as<float>(c->m_x32),
                        as<float>(c->m_tmp32), c->ds, st);
  UCOV_TRY(check_hip(c, "mixed initial inverse"));
  {
    const int rc = sync_status(c, rep, "FP32 factorisation");
    if (rc == UCOV_EGAUGE)
      return c->fail(UCOV_ENOCONV, "FP32 Cholesky factorisation failed: the scaled matrix is "
                                   "too ill-conditioned for the mixed path (use UCOV_FP64)");
    if (rc != UCOV_OK) return rc;
  }
  mixed_prepare(Np, A, Np, as<float>(c->m_x32), as<double>(c->m_x64), st);
  double res = 0.0;
  int it = 0;
  for (;; ++it) {
    fill_f64(as<double>(c->m_sum), 0.0, 1, st);
    mixed_residual(Np, A, Np, as<double>(c->m_x64), as<double>(c->m_r64), as<double>(c->m_sum),
                   st);
    double h = 0.0;
    if (hipMemcpyAsync(&h, c->m_sum.p, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return c->fail(UCOV_EDEVICE, "residual readback");
    res = std::sqrt(h / (double)N);
    if (res <= o.tol || it >= o.max_iter) break;
    mixed_update(Np, as<double>(c->m_x64), as<double>(c->m_r64), as<float>(c->m_x32),
                 as<float>(c->m_r32), as<float>(c->m_d32), st);
  }
  if (rep) {
    rep->ns_iters = it;
    rep->ns_residual = res;
  }
  if (!(res <= o.tol)) {
    char buf[160];
    snprintf(buf, sizeof buf, "Newton-Schulz residual %.3e above tol %.3e after %d steps", res,
             o.tol, it);
    return c->fail(UCOV_ENOCONV, buf);
  }
  hipEventRecord(c->ev[4], st);
  launch_extract_full(N, as<double>(c->m_x64), Np, as<double>(c->s), as<double>(c->q),
                      as<double>(c->alpha), cov_out, st);
  return UCOV_OK;
}

// Dense stage on the already assembled lower triangle of A_s in c->amat.
int run_dense_stage(ucov_ctx *c, int64_t N, const ucov_options &o, double *cov_out,
                    ucov_report *rep) {
  const int64_t Np = round_up(N, kTile);
  hipStream_t st = c->stream;
  double *A = as<double>(c->amat);
  launch_pad_identity(N, Np, A, Np, st);
  hipEventRecord(c->ev[3], st);
  if (o.precision == UCOV_FP64) {
    UCOV_TRY(ensure(c, c->tmat, 8 * std::max<int64_t>(1, spd_lower_inverse_scratch(Np))));
    spd_lower_inverse_fp64(A, Np, Np, as<double>(c->tmat), c->ds, st);
    hipEventRecord(c->ev[4], st);
    launch_extract(N, A, Np, as<double>(c->s), as<double>(c->q), as<double>(c->alpha), cov_out,
                   st);
  } else {
    UCOV_TRY(run_mixed(c, N, Np, o, cov_out, rep));
  }
  hipEventRecord(c->ev[5], st);
  UCOV_TRY(check_hip(c, "dense kernels"));
  UCOV_TRY(sync_status(c, rep, "dense inverse"));
  if (rep) {
    hipMemcpy(&rep->alpha, c->alpha.p, sizeof(double), hipMemcpyDeviceToHost);
    hipEventElapsedTime(&rep->ms_inverse, c->ev[3], c->ev[4]);
    hipEventElapsedTime(&rep->ms_extract, c->ev[4], c->ev[5]);
  }
  return UCOV_OK;
}

}  // namespace

extern "C" {

int ucov_create(ucov_ctx **ctx, int device) {
  if (!ctx) return UCOV_EINVAL;
  *ctx = nullptr;
  if (hipSetDevice(device) != hipSuccess) {
    hipGetLastError();
    return UCOV_EDEVICE;
  }
  ucov_ctx *c = new ucov_ctx();
  c->device = device;
  if (hipMalloc(&c->ds, sizeof(DevStatus)) != hipSuccess ||
      hipHostMalloc(&c->ds_host, sizeof(DevStatus)) != hipSuccess ||
      hipHostMalloc(&c->i64_host, 2 * sizeof(int64_t)) != hipSuccess) {
    hipGetLastError();
    delete c;
    return UCOV_ENOMEM;
  }
  for (auto &e : c->ev) hipEventCreate(&e);
  if (ensure(c, c->alpha, 8) != UCOV_OK) {
    ucov_destroy(c);
    return UCOV_ENOMEM;
  }
  *ctx = c;
  return UCOV_OK;
}

int ucov_set_stream(ucov_ctx *ctx, void *stream) {
  if (!ctx) return UCOV_EINVAL;
  ctx->stream = reinterpret_cast<hipStream_t>(stream);
  return UCOV_OK;
}

void ucov_destroy(ucov_ctx *c) {
  if (!c) return;
  hipSetDevice(c->device);
  if (c->stream) hipStreamSynchronize(c->stream);
  else hipDeviceSynchronize();
  Buf *bufs[] = {&c->cnt_p, &c->ptr_p, &c->cur_p, &c->slot_obs, &c->slot_cam, &c->slot_pt,
                 &c->rec, &c->bin_cnt, &c->bin_ptr, &c->bin_cur, &c->pairs, &c->scan_tmp, &c->nzlist, &c->nzcount,
                 &c->zdiag, &c->hc, &c->q, &c->s, &c->alpha, &c->amat, &c->tmat,
                 &c->m_a32, &c->m_x32, &c->m_r32, &c->m_d32, &c->m_tmp32, &c->m_x64, &c->m_r64,
                 &c->m_sum};
  for (Buf *b : bufs)
    if (b->p) hipFree(b->p);
  if (c->ds) hipFree(c->ds);
  if (c->ds_host) hipHostFree(c->ds_host);
  if (c->i64_host) hipHostFree(c->i64_host);
  for (auto &e : c->ev)
    if (e) hipEventDestroy(e);
  delete c;
}

int ucov_jacobians(ucov_ctx *c, const ucov_scene *scene, double *jp, double *jx) {
  if (!c) return UCOV_EINVAL;
  UCOV_TRY(check_scene(c, scene));
  if (!jp || !jx) return c->fail(UCOV_EINVAL, "NULL output");
  hipSetDevice(c->device);
  return run_scene_stage(c, scene, jp, jx, true, nullptr);
}

int ucov_reduced_camera_matrix(ucov_ctx *c, const ucov_scene *scene, double *z, int64_t ldz,
                               ucov_report *rep) {
  if (!c) return UCOV_EINVAL;
  UCOV_TRY(check_scene(c, scene));
  const int64_t N = 9 * (int64_t)scene->n_cams;
  if (!z || ldz < N) return c->fail(UCOV_EINVAL, "bad output matrix");
  hipSetDevice(c->device);
  if (rep) memset(rep, 0, sizeof *rep);
  UCOV_TRY(run_scene_stage(c, scene, nullptr, nullptr, false, rep));
  SceneDev sc = scene_dev(scene);
  SceneWork w = scene_work(c);
  launch_assemble(sc, w, 0, z, ldz, c->n_nonzero, c->stream);
  UCOV_TRY(check_hip(c, "assemble"));
  return sync_status(c, rep, "reduced camera matrix");
}

int ucov_gauge_basis(ucov_ctx *c, const ucov_scene *scene, double *hc, double *q) {
  if (!c) return UCOV_EINVAL;
  UCOV_TRY(check_scene(c, scene));
  hipSetDevice(c->device);
  UCOV_TRY(run_scene_stage(c, scene, nullptr, nullptr, false, nullptr));
  const int64_t N = 9 * (int64_t)scene->n_cams;
  UCOV_TRY(ensure(c, c->q, 8 * 7 * N));
  UCOV_TRY(ensure(c, c->s, 8 * N));
  launch_gauge(N, as<double>(c->hc), as<double>(c->q), as<double>(c->zdiag), nullptr, 0, 0.0,
               as<double>(c->s), as<double>(c->alpha), c->ds, c->stream);
  if (hc) hipMemcpyAsync(hc, c->hc.p, 8 * 7 * N, hipMemcpyDeviceToDevice, c->stream);
  if (q) hipMemcpyAsync(q, c->q.p, 8 * 7 * N, hipMemcpyDeviceToDevice, c->stream);
  UCOV_TRY(check_hip(c, "gauge"));
  return sync_status(c, nullptr, "gauge basis");
}

int ucov_camera_covariance(ucov_ctx *c, const ucov_scene *scene, const ucov_options *opt,
                           double *cov_out, ucov_report *rep) {
  if (!c) return UCOV_EINVAL;
  UCOV_TRY(check_scene(c, scene));
  if (!cov_out) return c->fail(UCOV_EINVAL, "NULL output");
  ucov_options o;
  fill_defaults(opt, o);
  if (o.precision != UCOV_FP64 && o.precision != UCOV_FP32_NS)
    return c->fail(UCOV_EINVAL, "unknown precision");
  hipSetDevice(c->device);
  if (rep) memset(rep, 0, sizeof *rep);
  UCOV_TRY(run_scene_stage(c, scene, nullptr, nullptr, false, rep));
  const int64_t N = 9 * (int64_t)scene->n_cams;
  const int64_t Np = round_up(N, kTile);
  UCOV_TRY(ensure(c, c->q, 8 * 7 * N));
  UCOV_TRY(ensure(c, c->s, 8 * N));
  UCOV_TRY(ensure(c, c->amat, 8 * Np * Np));
  SceneDev sc = scene_dev(scene);
  SceneWork w = scene_work(c);
  hipEventRecord(c->ev[2], c->stream);
  launch_gauge(N, w.hc, w.q, w.zdiag, nullptr, 0, o.alpha, w.s, w.alpha, c->ds, c->stream);
  launch_assemble(sc, w, 1, as<double>(c->amat), Np, c->n_nonzero, c->stream);
  UCOV_TRY(check_hip(c, "assemble"));
  UCOV_TRY(run_dense_stage(c, N, o, cov_out, rep));
  if (rep) {
    hipEventElapsedTime(&rep->ms_structure, c->ev[0], c->ev[1]);
    hipEventElapsedTime(&rep->ms_schur, c->ev[1], c->ev[2]);
    hipEventElapsedTime(&rep->ms_gauge, c->ev[2], c->ev[3]);
  }
  return UCOV_OK;
}

int ucov_pinv_blocks(ucov_ctx *c, int64_t n, const double *z, int64_t ldz, const double *q,
                     const ucov_options *opt, double *cov_out, ucov_report *rep) {
  if (!c) return UCOV_EINVAL;
  if (n < 9 || n % 9 != 0 || !z || ldz < n || !q || !cov_out)
    return c->fail(UCOV_EINVAL, "bad dense arguments");
  ucov_options o;
  fill_defaults(opt, o);
  if (o.precision != UCOV_FP64 && o.precision != UCOV_FP32_NS)
    return c->fail(UCOV_EINVAL, "unknown precision");
  hipSetDevice(c->device);
  if (rep) memset(rep, 0, sizeof *rep);
  const int64_t N = n, Np = round_up(N, kTile);
  UCOV_TRY(ensure(c, c->q, 8 * 7 * N));
  UCOV_TRY(ensure(c, c->s, 8 * N));
  UCOV_TRY(ensure(c, c->amat, 8 * Np * Np));
  hipStream_t st = c->stream;
  fill_i32(reinterpret_cast<int32_t *>(c->ds), 0, 2, st);
  hipMemcpyAsync(c->q.p, q, 8 * 7 * N, hipMemcpyDeviceToDevice, st);
  hipEventRecord(c->ev[2], st);
  launch_gauge(N, nullptr, as<double>(c->q), nullptr, z, ldz, o.alpha, as<double>(c->s),
               as<double>(c->alpha), c->ds, st);
  launch_scale_dense(N, z, ldz, as<double>(c->q), as<double>(c->s), as<double>(c->alpha),
                     as<double>(c->amat), Np, st);
  UCOV_TRY(check_hip(c, "scale"));
  UCOV_TRY(run_dense_stage(c, N, o, cov_out, rep));
  if (rep) hipEventElapsedTime(&rep->ms_gauge, c->ev[2], c->ev[3]);
  return UCOV_OK;
}

const char *ucov_strerror(int code) { return code_name(code); }

const char *ucov_last_error(const ucov_ctx *c) { return c ? c->last_error.c_str() : "no context"; }

}  // extern "C"

// C-ABI of the ucov library: context, workspace and the sequence of stages.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_map>
#include <map>
#include <mutex>
#include <vector>

#include "ucov_internal.h"
#include "../../include/ucov.h"

using namespace ucov;

namespace {

struct Buf {
  void *p = nullptr;
  size_t cap = 0;
};

}  // namespace

// Static scratch of the allocation-free entry point (one array on every GPU
// the library runs on, held until the process ends).  Host code never uses
// its name as an address: each device's address comes from
// hipGetSymbolAddress, taken once per device when a context is created.
static __device__ __align__(256) unsigned char scratch[UCOV_NOALLOC_SCRATCH_BYTES];

namespace {

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

// Stage marks of a call: HIP events recorded on the context's stream between
// the launches of the stages the report times.
enum EvMark {
  kEvStart,      // before the first kernel
  kEvGrouped,    // observations grouped and sorted by point
  kEvPoints,     // Jacobians and point blocks done
  kEvBins,       // camera-pair bins built and filled
  kEvDiag,       // diagonal camera blocks and rotation nullspace rows done
  kEvGauge,      // gauge basis, weight and scaling done
  kEvAssembled,  // scaled regularised matrix assembled and padded
  kEvInverse,    // dense factorisation and inversion done
  kEvEnd,        // outputs written
  kEvBatch,      // batched calls: before the concatenation of the scenes
  kEvTune0,
  kEvTune1,
  kEvCount
};

constexpr int kMaxDevices = 64;
void *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// This device's address of the static scratch; the device must be current.
int scratch_address(int device, void **out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return UCOV_EDEVICE;
  if (!g_scratch[device]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      hipGetLastError();
      return UCOV_EDEVICE;
    }
    g_scratch[device] = p;
  }
  *out = g_scratch[device];
  return UCOV_OK;
}

constexpr int kArenaSlots = 64;

}  // namespace

struct ucov_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  DevStatus *ds = nullptr;       // device
  DevStatus *ds_host = nullptr;  // pinned host mirror
  int64_t *i64_host = nullptr;   // pinned host scalars [0] pairs, [1] non-empty bins
  int64_t n_nonzero = 0;         // non-empty bins of the last scene stage
  int64_t pairs_cap = 0;         // entries of the pair list of the last scene stage
  // Recording a launch sequence (a batch's graph): no host round trip, no
  // event, no upload; the counts of the eager call that sized the buffers hold.
  bool replay = false;
  hipEvent_t ev[kEvCount] = {};
  // workspace
  Buf cnt_p, ptr_p, cur_p, slot_key, slot_obs, slot_cam, slot_pt, rec;
  Buf bin_cnt, bin_ptr, bin_cur, pairs, scan_tmp, nzlist, nzcount, nzpos, flag;
  Buf cam_keys, cam_slots, cam_ptr, cam_tmp;  // slots grouped by camera
  Buf zdiag, hc, q, s, alpha, amat, tmat;
  Buf m_a32, m_x32, m_r32, m_d32, m_tmp32, m_x64, m_r64, m_sum;  // mixed precision
  Buf m_split;  // split-BF16 slices and exponents
  Buf hp_cams, hp_pts, hp_oc, hp_op, hp_info, hp_out;  // staging of UCOV_HOST_PTRS calls
  // batched calls: the concatenated scenes, their tables and per-scene status
  Buf b_cams, b_pts, b_info, b_oc, b_op, b_cam_scene, b_tab, b_ds, b_scratch;
  SpdPlan *plan = nullptr;  // batched inverse plan, kept while the batch is unchanged
  void *h_stage = nullptr;  // pinned host staging of the scene tables
  size_t h_stage_cap = 0;
  DevStatus *h_ds = nullptr;  // pinned host copy of the per-scene status
  size_t h_ds_cap = 0;
  // learned screener
  Buf f_hist, f_ang, f_covis, mlp_ws, mlp_grad, f_lab, f_zero, f_bscale;
  Buf sr_off, sr_tmp;  // sub-scene sizes and selection scratch
  Buf pg_f;  // the paper gauge's F (28 upper values), L_F (7 x 7 row-major), partial sums
  // dense stage: the tuned 32 x 32-tile threshold per padded size
  std::map<int64_t, int64_t> small_tiles;
  int64_t small_for(int64_t np) const {
    const auto it = small_tiles.find(np);
    return it == small_tiles.end() ? kSmallTilesDefault : it->second;
  }
  // batched dense stage: the tuned threshold per list of padded sizes (scene
  // order); untuned batches run every product on 64 x 64 tiles
  std::map<std::vector<int64_t>, int64_t> batch_small;
  int64_t batch_small_for(const std::vector<int64_t> &np) const {
    const auto it = batch_small.find(np);
    return it == batch_small.end() ? 0 : it->second;
  }
  Buf fc_x, fc_part, fc_xq, fc_k;  // whole covariance: X, X q partial sums, X q, q^T X q
  // incremental update: indices, padded Z^+, JtT, B, T, S, scratch, Jacobians, J_n, U, small, V, W
  Buf up_idx, up_z, up_jt, up_b, up_t, up_s, up_tmp, up_nj, up_jn, up_u, up_g, up_v, up_w;
  // sub-reconstructions: index maps, the gathered sub-scenes and their blocks
  Buf sr_idx, sr_cams, sr_pts, sr_info, sr_cand, sr_chosen;

  // Allocation-free calls: while `on`, ensure() carves every buffer from
  // this device's static scratch (base, cap) and remembers the context's own
  // buffer, which is put back when the call ends.
  struct Arena {
    char *base = nullptr;
    size_t cap = 0, off = 0;
    bool on = false;
    int n_saved = 0;
    Buf *who[kArenaSlots] = {};
    Buf was[kArenaSlots] = {};
  } arena;

  int fail(int code, const std::string &msg) {
    last_error = std::string(code_name(code)) + ": " + msg;
    return code;
  }
};

namespace {

int ensure(ucov_ctx *c, Buf &b, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (c->arena.on) {
    auto &a = c->arena;
    int k = 0;
    while (k < a.n_saved && a.who[k] != &b) ++k;
    if (k < a.n_saved && b.cap >= bytes) return UCOV_OK;  // carved earlier in this call
    const size_t off = (a.off + 255) & ~(size_t)255;
    if (off > a.cap || bytes > a.cap - off)
      return c->fail(UCOV_ENOMEM, "the scene needs more than the " +
                                      std::to_string((size_t)UCOV_NOALLOC_SCRATCH_BYTES) +
                                      " bytes of static scratch of the allocation-free call");
    if (k == a.n_saved) {
      if (a.n_saved == kArenaSlots) return c->fail(UCOV_EDEVICE, "internal: scratch table full");
      a.who[k] = &b;
      a.was[k] = b;
      ++a.n_saved;
    }
    b.p = a.base + off;
    b.cap = bytes;
    a.off = off + bytes;
    return UCOV_OK;
  }
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

// Carves the buffers of one call from the static scratch; the context's own
// buffers are put back when the scope ends.
struct ArenaScope {
  ucov_ctx *c;
  explicit ArenaScope(ucov_ctx *ctx) : c(ctx) {
    c->arena.on = true;
    c->arena.off = 0;
    c->arena.n_saved = 0;
  }
  ~ArenaScope() {
    for (int k = c->arena.n_saved - 1; k >= 0; --k) *c->arena.who[k] = c->arena.was[k];
    c->arena.n_saved = 0;
    c->arena.on = false;
  }
};

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
  if (c->ds_host->code != 0) {
    if (rep) rep->bad_index = c->ds_host->index;
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

// UCOV_ENOMEM before any launch when a scene's work buffers alone exceed the
// device's memory: the dense matrix and its recursion scratch, the camera-pair
// bins and the per-observation records (a lower bound of what the call needs).
int check_fits(ucov_ctx *c, const ucov_scene *s) {
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    hipGetLastError();
    return UCOV_OK;  // unknown: the allocations will tell
  }
  const double n = s->n_cams, Np = (double)round_up(9 * (int64_t)s->n_cams, kTile);
  const double need = 8.0 * Np * Np * 1.5 + 32.0 * n * (n + 1) / 2 + 300.0 * (double)s->n_obs;
  if (need <= (double)total_b) return UCOV_OK;
  char buf[200];
  snprintf(buf, sizeof buf, "the scene needs at least %.3g bytes of device memory, the device has %.3g",
           need, (double)total_b);
  return c->fail(UCOV_ENOMEM, buf);
}

void mark(ucov_ctx *c, int k, hipStream_t st) {
  if (!c->replay) hipEventRecord(c->ev[k], st);
}

float ev_ms(ucov_ctx *c, int a, int b) {
  float t = 0.0f;
  if (hipEventElapsedTime(&t, c->ev[a], c->ev[b]) != hipSuccess) {
    hipGetLastError();
    t = 0.0f;
  }
  return t;
}

// Stage times of a call that ran the whole scene stage: index grouping and
// pair binning are "structure"; Jacobians, point blocks, the diagonal camera
// blocks and the assembly of the Schur complement are "schur"; the gauge
// basis, weight and scaling are "gauge".
void report_stages(ucov_ctx *c, ucov_report *rep) {
  if (!rep) return;
  rep->ms_structure = ev_ms(c, kEvStart, kEvGrouped) + ev_ms(c, kEvPoints, kEvBins);
  rep->ms_schur = ev_ms(c, kEvGrouped, kEvPoints) + ev_ms(c, kEvBins, kEvDiag) +
                  ev_ms(c, kEvGauge, kEvAssembled);
  rep->ms_gauge = ev_ms(c, kEvDiag, kEvGauge);
  rep->ms_inverse = ev_ms(c, kEvAssembled, kEvInverse);
  rep->ms_extract = ev_ms(c, kEvInverse, kEvEnd);
  rep->ms_total = ev_ms(c, kEvStart, kEvEnd);
}

// Steps a1-a2 up to the per-camera diagonal blocks and the nullspace rows.
// On return the slot records, pair bins, zdiag and hc are valid.
// nbins: camera-pair bins, n(n+1)/2 for one scene, the sum over the scenes of
// a concatenation; max_scene_cams: cameras of the largest scene (n for one
// scene).  The status must have been cleared by the caller.
int run_scene_stage(ucov_ctx *c, const SceneDev &sc, int64_t nbins, double *jp_out,
                    double *jx_out, bool jac_only, ucov_report *rep,
                    int64_t max_scene_cams = -1) {
  const int64_t n = sc.n, m = sc.m, t = sc.t;
  const int64_t N = 9 * n;
  const int64_t scan_tiles = (std::max(nbins, m) + 4095) / 4096 + 2;
  UCOV_TRY(ensure(c, c->cnt_p, 4 * m));
  UCOV_TRY(ensure(c, c->ptr_p, 8 * (m + 1)));
  UCOV_TRY(ensure(c, c->cur_p, 4 * m));
  UCOV_TRY(ensure(c, c->slot_key, 8 * t));
  UCOV_TRY(ensure(c, c->slot_obs, 4 * t));
  UCOV_TRY(ensure(c, c->slot_cam, 4 * t));
  UCOV_TRY(ensure(c, c->slot_pt, 4 * t));
  UCOV_TRY(ensure(c, c->rec, 8 * kRec * t));
  UCOV_TRY(ensure(c, c->scan_tmp, 8 * scan_tiles));
  SceneWork w{};
  w.cnt_p = as<int32_t>(c->cnt_p);
  w.ptr_p = as<int64_t>(c->ptr_p);
  w.cur_p = as<int32_t>(c->cur_p);
  w.slot_key = as<int64_t>(c->slot_key);
  w.slot_obs = as<int32_t>(c->slot_obs);
  w.slot_cam = as<int32_t>(c->slot_cam);
  w.slot_pt = as<int32_t>(c->slot_pt);
  w.rec = as<double>(c->rec);
  w.scan_tmp = as<int64_t>(c->scan_tmp);
  hipStream_t st = c->stream;

  mark(c, kEvStart, st);
  fill_i32(w.cnt_p, 0, m, st);
  fill_i32(w.cur_p, 0, m, st);
  launch_count_points(sc, w, c->ds, st);
  exclusive_scan(w.cnt_p, w.ptr_p, m, w.scan_tmp, st);
  launch_group_points(sc, w, c->ds, st);
  mark(c, kEvGrouped, st);
  launch_jacobians(sc, w, jp_out, jx_out, c->ds, st);
  UCOV_TRY(check_hip(c, "jacobian kernels"));
  if (jac_only) return sync_status(c, rep, "jacobians");

  UCOV_TRY(ensure(c, c->bin_cnt, 4 * nbins));
  UCOV_TRY(ensure(c, c->bin_ptr, 8 * (nbins + 1)));
  UCOV_TRY(ensure(c, c->bin_cur, 4 * nbins));
  UCOV_TRY(ensure(c, c->nzlist, sizeof(int2) * nbins));  // at most one entry per bin
  UCOV_TRY(ensure(c, c->nzcount, 8));
  UCOV_TRY(ensure(c, c->flag, 8));
  UCOV_TRY(ensure(c, c->nzpos, 8 * (nbins + 1)));
  w.bin_cnt = as<int32_t>(c->bin_cnt);
  w.bin_ptr = as<int64_t>(c->bin_ptr);
  w.bin_cur = as<int32_t>(c->bin_cur);
  w.nzlist = as<int2>(c->nzlist);
  w.nzcount = as<int64_t>(c->nzcount);
  w.nzpos = as<int64_t>(c->nzpos);
  launch_point_blocks(sc, w, c->ds, st);
  mark(c, kEvPoints, st);
  // camera-pair bins: camera-major with LDS counters where the largest
  // scene's cameras fit them, else one global atomic per pair
  const int64_t mc = max_scene_cams < 0 ? n : max_scene_cams;
  const bool cam_major = t > 0 && mc <= kCamHistMax;
  if (cam_major) {
    const size_t tmp_bytes = camera_lists_scratch(t);
    UCOV_TRY(ensure(c, c->cam_keys, 4 * t));
    UCOV_TRY(ensure(c, c->cam_slots, 4 * t));
    UCOV_TRY(ensure(c, c->cam_ptr, 8 * (n + 1)));
    UCOV_TRY(ensure(c, c->cam_tmp, std::max<size_t>(tmp_bytes, 8)));
    w.cam_keys = as<int32_t>(c->cam_keys);
    w.cam_slots = as<int32_t>(c->cam_slots);
    w.cam_ptr = as<int64_t>(c->cam_ptr);
    if (launch_camera_lists(sc, w, c->cam_tmp.p, tmp_bytes, st) != 0)
      return c->fail(UCOV_EDEVICE, "sorting the slots by camera");
    launch_pair_count_cam(sc, w, (int)mc, st);
  } else {
    fill_i32(w.bin_cnt, 0, nbins, st);
    launch_pair_count(sc, w, st);
  }
  exclusive_scan(w.bin_cnt, w.bin_ptr, nbins, w.scan_tmp, st);
  if (c->replay) launch_guard_pairs(w, nbins, c->pairs_cap, as<int32_t>(c->flag), c->ds, st);
  launch_nonzero_bins(sc, w, nbins, st);
  UCOV_TRY(check_hip(c, "point kernels"));
  int64_t npairs = c->pairs_cap;
  if (c->replay) {
    // the recorded sizes hold; the device checks that the scene did not grow
    launch_check_nonzero(w, c->n_nonzero, c->ds, st);
  } else {
    // the pair count sizes the next buffer: one host round trip
    hipMemcpyAsync(c->i64_host, w.bin_ptr + nbins, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    hipMemcpyAsync(c->i64_host + 1, w.nzcount, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    UCOV_TRY(sync_status(c, rep, "point blocks"));
    npairs = c->i64_host[0];
    c->n_nonzero = c->i64_host[1];
    c->pairs_cap = npairs;
    if (rep) rep->n_pairs = npairs;
  }
  UCOV_TRY(ensure(c, c->pairs, sizeof(int2) * npairs));
  UCOV_TRY(ensure(c, c->zdiag, 8 * 81 * n));
  UCOV_TRY(ensure(c, c->hc, 8 * 7 * N));
  w.pairs = as<int2>(c->pairs);
  w.zdiag = as<double>(c->zdiag);
  w.hc = as<double>(c->hc);
  // the camera-major fill keeps LDS cursors as int32 offsets within a row
  // a replay skips the fill when its scene outgrew the recorded pair list
  const int32_t *skip = c->replay ? as<int32_t>(c->flag) : nullptr;
  if (cam_major && npairs < ((int64_t)1 << 31))
    launch_pair_fill_cam(sc, w, (int)mc, nbins, npairs, skip, st);
  else
    launch_pair_fill(sc, w, nbins, npairs, skip, st);
  mark(c, kEvBins, st);
  launch_camera_diag(sc, w, c->ds, st);
  mark(c, kEvDiag, st);
  UCOV_TRY(check_hip(c, "schur kernels"));
  return UCOV_OK;
}

SceneWork scene_work(ucov_ctx *c) {
  SceneWork w{};
  w.cnt_p = as<int32_t>(c->cnt_p);
  w.ptr_p = as<int64_t>(c->ptr_p);
  w.cur_p = as<int32_t>(c->cur_p);
  w.slot_key = as<int64_t>(c->slot_key);
  w.slot_obs = as<int32_t>(c->slot_obs);
  w.slot_cam = as<int32_t>(c->slot_cam);
  w.slot_pt = as<int32_t>(c->slot_pt);
  w.rec = as<double>(c->rec);
  w.bin_cnt = as<int32_t>(c->bin_cnt);
  w.bin_ptr = as<int64_t>(c->bin_ptr);
  w.bin_cur = as<int32_t>(c->bin_cur);
  w.pairs = as<int2>(c->pairs);
  w.cam_keys = as<int32_t>(c->cam_keys);
  w.cam_slots = as<int32_t>(c->cam_slots);
  w.cam_ptr = as<int64_t>(c->cam_ptr);
  w.nzlist = as<int2>(c->nzlist);
  w.nzcount = as<int64_t>(c->nzcount);
  w.nzpos = as<int64_t>(c->nzpos);
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

int64_t single_bins(const SceneDev &sc) { return (int64_t)sc.n * (sc.n + 1) / 2; }

void clear_status(ucov_ctx *c) {
  fill_i32(reinterpret_cast<int32_t *>(c->ds), 0, 2, c->stream);
}

void reset_report(ucov_report *rep) {
  if (!rep) return;
  memset(rep, 0, sizeof *rep);
  rep->bad_index = -1;
  rep->bad_scene = -1;
}

void fill_defaults(const ucov_options *opt, ucov_options &o) {
  o.precision = UCOV_FP64;
  o.max_iter = 6;
  o.tol = 1e-10;
  o.alpha = 0.0;
  o.gauge = UCOV_GAUGE_CAMERA;
  o.flags = 0;
  if (opt) {
    o.precision = opt->precision;
    if (opt->max_iter > 0) o.max_iter = opt->max_iter;
    if (opt->tol > 0) o.tol = opt->tol;
    o.alpha = opt->alpha;
    o.gauge = opt->gauge;
    o.flags = opt->flags;
  }
}

// Entry points that take device pointers only reject UCOV_HOST_PTRS.
int device_only(ucov_ctx *c, const ucov_options &o) {
  if (o.flags == 0) return UCOV_OK;
  return c->fail(UCOV_EINVAL, "this entry point takes device pointers only (flags must be 0)");
}

// Mixed-precision inverse of A_s (Np x Np in c->amat): FP32 MFMA Cholesky
// inverse X0, then Newton-Schulz steps X <- X + X (I - A X) with the residual
// in FP64 and the correction on FP32 MFMA (UCOV_FP32_NS) or from split-BF16
// products on BF16 MFMA (UCOV_BF16X_NS), until |I - A X|_F / sqrt(N) <= tol.
int run_mixed(ucov_ctx *c, int64_t N, int64_t Np, const ucov_options &o, double *cov_out,
              ucov_report *rep) {
  hipStream_t st = c->stream;
  const size_t f32 = 4 * (size_t)Np * Np, f64 = 8 * (size_t)Np * Np;
  const bool split = o.precision == UCOV_BF16X_NS;
  UCOV_TRY(ensure(c, c->m_a32, f32));
  UCOV_TRY(ensure(c, c->m_x32, f32));
  if (split) {
    UCOV_TRY(ensure(c, c->m_split, split_bf16_scratch(Np)));
  } else {
    UCOV_TRY(ensure(c, c->m_r32, f32));
    UCOV_TRY(ensure(c, c->m_d32, f32));
  }
  UCOV_TRY(ensure(c, c->m_tmp32, 4 * std::max<int64_t>(1, spd_lower_inverse_scratch(Np))));
  UCOV_TRY(ensure(c, c->m_x64, f64));
  UCOV_TRY(ensure(c, c->m_r64, f64));
  UCOV_TRY(ensure(c, c->m_sum, 8 * ((size_t)Np + 1)));
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
    mixed_residual(Np, A, Np, as<double>(c->m_x64), as<double>(c->m_r64), as<double>(c->m_sum),
                   st);
    double h = 0.0;
    if (hipMemcpyAsync(&h, c->m_sum.p, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return c->fail(UCOV_EDEVICE, "residual readback");
    res = std::sqrt(h / (double)N);
    if (res <= o.tol || it >= o.max_iter) break;
    if (split)
      split_bf16_update(Np, as<double>(c->m_x64), as<double>(c->m_r64), c->m_split.p, st);
    else
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
  hipEventRecord(c->ev[kEvInverse], st);
  launch_extract_full(N, as<double>(c->m_x64), Np, as<double>(c->s), as<double>(c->q), N,
                      as<double>(c->alpha), o.gauge != UCOV_GAUGE_PAPER, cov_out, st);
  return UCOV_OK;
}

// Dense stage on the already assembled lower triangle of A_s in c->amat.
int run_dense_stage(ucov_ctx *c, int64_t N, const ucov_options &o, double *cov_out,
                    ucov_report *rep) {
  const int64_t Np = round_up(N, kTile);
  hipStream_t st = c->stream;
  double *A = as<double>(c->amat);
  launch_pad_identity(N, Np, A, Np, st);
  hipEventRecord(c->ev[kEvAssembled], st);
  if (o.precision == UCOV_FP64) {
    UCOV_TRY(ensure(c, c->tmat, 8 * std::max<int64_t>(1, spd_lower_inverse_scratch(Np))));
    spd_lower_inverse_fp64(A, Np, Np, as<double>(c->tmat), c->ds, st, c->small_for(Np));
    hipEventRecord(c->ev[kEvInverse], st);
    launch_extract(N, A, Np, as<double>(c->s), as<double>(c->q), N, as<double>(c->alpha),
                   o.gauge != UCOV_GAUGE_PAPER, cov_out, st);
  } else {
    UCOV_TRY(run_mixed(c, N, Np, o, cov_out, rep));
  }
  hipEventRecord(c->ev[kEvEnd], st);
  UCOV_TRY(check_hip(c, "dense kernels"));
  UCOV_TRY(sync_status(c, rep, "dense inverse"));
  if (rep) hipMemcpy(&rep->alpha, c->alpha.p, sizeof(double), hipMemcpyDeviceToHost);
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
  void *sp = nullptr;
  if (scratch_address(device, &sp) != UCOV_OK) {
    ucov_destroy(c);
    return UCOV_EDEVICE;
  }
  c->arena.base = static_cast<char *>(sp);
  c->arena.cap = UCOV_NOALLOC_SCRATCH_BYTES;
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
  Buf *bufs[] = {&c->cnt_p, &c->ptr_p, &c->cur_p, &c->slot_key, &c->slot_obs, &c->slot_cam, &c->slot_pt,
                 &c->rec, &c->bin_cnt, &c->bin_ptr, &c->bin_cur, &c->pairs, &c->scan_tmp, &c->nzlist, &c->nzcount, &c->nzpos, &c->flag,
                 &c->cam_keys, &c->cam_slots, &c->cam_ptr, &c->cam_tmp,
                 &c->zdiag, &c->hc, &c->q, &c->s, &c->alpha, &c->amat, &c->tmat,
                 &c->m_a32, &c->m_x32, &c->m_r32, &c->m_d32, &c->m_tmp32, &c->m_x64, &c->m_r64,
                 &c->m_sum, &c->m_split, &c->hp_cams, &c->hp_pts, &c->hp_oc, &c->hp_op,
                 &c->hp_info, &c->hp_out, &c->b_cams, &c->b_pts, &c->b_info, &c->b_oc, &c->b_op,
                 &c->b_cam_scene, &c->b_tab, &c->b_ds, &c->b_scratch, &c->f_hist, &c->f_ang, &c->f_covis,
                 &c->mlp_ws, &c->mlp_grad, &c->f_lab, &c->f_zero, &c->f_bscale, &c->sr_off, &c->sr_tmp, &c->pg_f, &c->sr_idx, &c->sr_cams, &c->sr_pts,
                 &c->sr_info, &c->sr_cand, &c->sr_chosen, &c->fc_x, &c->fc_part,
                 &c->fc_xq, &c->fc_k, &c->up_idx, &c->up_z, &c->up_jt, &c->up_b,
                 &c->up_t, &c->up_s, &c->up_tmp, &c->up_nj, &c->up_jn, &c->up_u, &c->up_g,
                 &c->up_v, &c->up_w};
  for (Buf *b : bufs)
    if (b->p) hipFree(b->p);
  if (c->h_stage) hipHostFree(c->h_stage);
  if (c->h_ds) hipHostFree(c->h_ds);
  spd_plan_destroy(c->plan);
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
  const SceneDev sc = scene_dev(scene);
  clear_status(c);
  return run_scene_stage(c, sc, single_bins(sc), jp, jx, true, nullptr);
}

int ucov_reduced_camera_matrix(ucov_ctx *c, const ucov_scene *scene, double *z, int64_t ldz,
                               ucov_report *rep) {
  if (!c) return UCOV_EINVAL;
  UCOV_TRY(check_scene(c, scene));
  const int64_t N = 9 * (int64_t)scene->n_cams;
  if (!z || ldz < N) return c->fail(UCOV_EINVAL, "bad output matrix");
  hipSetDevice(c->device);
  reset_report(rep);
  const SceneDev sc = scene_dev(scene);
  clear_status(c);
  UCOV_TRY(run_scene_stage(c, sc, single_bins(sc), nullptr, nullptr, false, rep));
  SceneWork w = scene_work(c);
  launch_assemble(sc, w, 0, z, ldz, c->n_nonzero, c->stream);
  UCOV_TRY(check_hip(c, "assemble"));
  return sync_status(c, rep, "reduced camera matrix");
}

int ucov_gauge_basis(ucov_ctx *c, const ucov_scene *scene, double *hc, double *q) {
  if (!c) return UCOV_EINVAL;
  UCOV_TRY(check_scene(c, scene));
  hipSetDevice(c->device);
  const SceneDev sc = scene_dev(scene);
  clear_status(c);
  UCOV_TRY(run_scene_stage(c, sc, single_bins(sc), nullptr, nullptr, false, nullptr));
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

}  // extern "C"

namespace {

int camera_covariance_dev(ucov_ctx *c, const ucov_scene *scene, const ucov_options *opt,
                          double *cov_out, ucov_report *rep);

// UCOV_HOST_PTRS: the scene and the output staged through device buffers.
int camera_covariance_impl(ucov_ctx *c, const ucov_scene *scene, const ucov_options *opt,
                           double *cov_out, ucov_report *rep) {
  if (!c) return UCOV_EINVAL;
  if (!opt || !(opt->flags & UCOV_HOST_PTRS))
    return camera_covariance_dev(c, scene, opt, cov_out, rep);
  if (opt->flags & ~UCOV_HOST_PTRS) return c->fail(UCOV_EINVAL, "unknown flags");
  UCOV_TRY(check_scene(c, scene));
  if (!cov_out) return c->fail(UCOV_EINVAL, "NULL output");
  hipSetDevice(c->device);
  const int64_t n = scene->n_cams, m = scene->n_pts, t = scene->n_obs;
  UCOV_TRY(ensure(c, c->hp_cams, 8 * 9 * (size_t)n));
  UCOV_TRY(ensure(c, c->hp_pts, 8 * 3 * (size_t)m));
  UCOV_TRY(ensure(c, c->hp_oc, 4 * (size_t)t));
  UCOV_TRY(ensure(c, c->hp_op, 4 * (size_t)t));
  if (scene->obs_info) UCOV_TRY(ensure(c, c->hp_info, 8 * 3 * (size_t)t));
  UCOV_TRY(ensure(c, c->hp_out, 8 * 81 * (size_t)n));
  hipStream_t st = c->stream;
  if (hipMemcpyAsync(c->hp_cams.p, scene->cams, 8 * 9 * n, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(c->hp_pts.p, scene->pts, 8 * 3 * m, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(c->hp_oc.p, scene->obs_cam, 4 * t, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(c->hp_op.p, scene->obs_pt, 4 * t, hipMemcpyHostToDevice, st) != hipSuccess ||
      (scene->obs_info &&
       hipMemcpyAsync(c->hp_info.p, scene->obs_info, 8 * 3 * t, hipMemcpyHostToDevice, st) != hipSuccess))
    return check_hip(c, "copying the scene to the device");
  ucov_scene d = *scene;
  d.cams = as<double>(c->hp_cams);
  d.pts = as<double>(c->hp_pts);
  d.obs_cam = as<int32_t>(c->hp_oc);
  d.obs_pt = as<int32_t>(c->hp_op);
  d.obs_info = scene->obs_info ? as<double>(c->hp_info) : nullptr;
  ucov_options o = *opt;
  o.flags = 0;
  UCOV_TRY(camera_covariance_dev(c, &d, &o, as<double>(c->hp_out), rep));
  if (hipMemcpyAsync(cov_out, c->hp_out.p, 8 * 81 * n, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return check_hip(c, "copying the blocks to the host");
  return UCOV_OK;
}

int camera_covariance_dev(ucov_ctx *c, const ucov_scene *scene, const ucov_options *opt,
                          double *cov_out, ucov_report *rep) {
  if (!c) return UCOV_EINVAL;
  UCOV_TRY(check_scene(c, scene));
  UCOV_TRY(check_fits(c, scene));
  if (!cov_out) return c->fail(UCOV_EINVAL, "NULL output");
  ucov_options o;
  fill_defaults(opt, o);
  UCOV_TRY(device_only(c, o));
  if (o.precision != UCOV_FP64 && o.precision != UCOV_FP32_NS && o.precision != UCOV_BF16X_NS)
    return c->fail(UCOV_EINVAL, "unknown precision");
  if (o.gauge != UCOV_GAUGE_CAMERA && o.gauge != UCOV_GAUGE_PAPER)
    return c->fail(UCOV_EINVAL, "unknown gauge");
  hipSetDevice(c->device);
  reset_report(rep);
  const SceneDev sc = scene_dev(scene);
  clear_status(c);
  UCOV_TRY(run_scene_stage(c, sc, single_bins(sc), nullptr, nullptr, false, rep));
  const int64_t N = 9 * (int64_t)scene->n_cams;
  const int64_t Np = round_up(N, kTile);
  UCOV_TRY(ensure(c, c->q, 8 * 7 * N));
  UCOV_TRY(ensure(c, c->s, 8 * N));
  UCOV_TRY(ensure(c, c->alpha, 8));
  UCOV_TRY(ensure(c, c->amat, 8 * Np * Np));
  if (o.gauge == UCOV_GAUGE_PAPER)
    UCOV_TRY(ensure(c, c->pg_f, 8 * paper_gauge_doubles(scene->n_pts)));
  SceneWork w = scene_work(c);
  if (o.gauge == UCOV_GAUGE_PAPER) {
    launch_paper_gauge(sc, w, as<double>(c->pg_f), c->ds, c->stream);
    launch_gauge(N, nullptr, w.q, w.zdiag, nullptr, 0, 1.0, w.s, w.alpha, c->ds, c->stream);
  } else {
    launch_gauge(N, w.hc, w.q, w.zdiag, nullptr, 0, o.alpha, w.s, w.alpha, c->ds, c->stream);
  }
  hipEventRecord(c->ev[kEvGauge], c->stream);
  launch_assemble(sc, w, 1, as<double>(c->amat), Np, c->n_nonzero, c->stream);
  UCOV_TRY(check_hip(c, "assemble"));
  UCOV_TRY(run_dense_stage(c, N, o, cov_out, rep));
  report_stages(c, rep);
  return UCOV_OK;
}

}  // namespace

extern "C" {

int ucov_camera_covariance(ucov_ctx *c, const ucov_scene *scene, const ucov_options *opt,
                           double *cov_out, ucov_report *rep) {
  return camera_covariance_impl(c, scene, opt, cov_out, rep);
}

// The same path with every buffer carved from the static scratch: no device
// or pinned allocation happens in this call (the status word, the pinned
// readback scalars and the events were made by ucov_create).
int ucov_camera_covariance_noalloc(ucov_ctx *c, const ucov_scene *scene,
                                   const ucov_options *opt, double *cov_out, ucov_report *rep) {
  if (!c) return UCOV_EINVAL;
  if (opt && opt->precision != UCOV_FP64)
    return c->fail(UCOV_EINVAL, "the allocation-free call supports UCOV_FP64 only");
  if (!c->arena.base) return c->fail(UCOV_EDEVICE, "no static scratch on this device");
  ArenaScope scope(c);
  return camera_covariance_impl(c, scene, opt, cov_out, rep);
}

int ucov_pinv_blocks(ucov_ctx *c, int64_t n, const double *z, int64_t ldz, const double *q,
                     const ucov_options *opt, double *cov_out, ucov_report *rep) {
  if (!c) return UCOV_EINVAL;
  if (n < 9 || n % 9 != 0 || !z || ldz < n || !q || !cov_out)
    return c->fail(UCOV_EINVAL, "bad dense arguments");
  ucov_options o;
  fill_defaults(opt, o);
  UCOV_TRY(device_only(c, o));
  if (o.precision != UCOV_FP64 && o.precision != UCOV_FP32_NS && o.precision != UCOV_BF16X_NS)
    return c->fail(UCOV_EINVAL, "unknown precision");
  hipSetDevice(c->device);
  reset_report(rep);
  const int64_t N = n, Np = round_up(N, kTile);
  UCOV_TRY(ensure(c, c->q, 8 * 7 * N));
  UCOV_TRY(ensure(c, c->s, 8 * N));
  UCOV_TRY(ensure(c, c->amat, 8 * Np * Np));
  hipStream_t st = c->stream;
  fill_i32(reinterpret_cast<int32_t *>(c->ds), 0, 2, st);
  hipMemcpyAsync(c->q.p, q, 8 * 7 * N, hipMemcpyDeviceToDevice, st);
  hipEventRecord(c->ev[kEvDiag], st);
  launch_gauge(N, nullptr, as<double>(c->q), nullptr, z, ldz, o.alpha, as<double>(c->s),
               as<double>(c->alpha), c->ds, st);
  launch_scale_dense(N, z, ldz, as<double>(c->q), as<double>(c->s), as<double>(c->alpha),
                     as<double>(c->amat), Np, st);
  o.gauge = UCOV_GAUGE_CAMERA;  // the caller's q is an orthonormal gauge basis
  UCOV_TRY(check_hip(c, "scale"));
  UCOV_TRY(run_dense_stage(c, N, o, cov_out, rep));
  if (rep) {
    rep->ms_gauge = ev_ms(c, kEvDiag, kEvAssembled);
    rep->ms_inverse = ev_ms(c, kEvAssembled, kEvInverse);
    rep->ms_extract = ev_ms(c, kEvInverse, kEvEnd);
  }
  return UCOV_OK;
}

// The whole camera covariance and every point's 3 x 3 covariance (Sec. 5.2:
// the points eliminated by block inversion and recovered from the camera
// covariance).  The dense stage keeps the full scaled inverse X = L^-T L^-1.
int ucov_full_covariance(ucov_ctx *c, const ucov_scene *scene, const ucov_options *opt,
                         double *cam_cov, int64_t ldc, double *pt_cov, ucov_report *rep) {
  if (!c) return UCOV_EINVAL;
  UCOV_TRY(check_scene(c, scene));
  const int64_t N = 9 * (int64_t)scene->n_cams;
  if (!cam_cov && !pt_cov) return c->fail(UCOV_EINVAL, "no output requested");
  if (cam_cov && ldc < N) return c->fail(UCOV_EINVAL, "bad leading dimension of cam_cov");
  ucov_options o;
  fill_defaults(opt, o);
  UCOV_TRY(device_only(c, o));
  if (o.precision != UCOV_FP64)
    return c->fail(UCOV_EINVAL, "the whole covariance supports UCOV_FP64 only");
  if (o.gauge != UCOV_GAUGE_CAMERA && o.gauge != UCOV_GAUGE_PAPER)
    return c->fail(UCOV_EINVAL, "unknown gauge");
  const bool paper = o.gauge == UCOV_GAUGE_PAPER;
  hipSetDevice(c->device);
  reset_report(rep);
  const SceneDev sc = scene_dev(scene);
  clear_status(c);
  UCOV_TRY(run_scene_stage(c, sc, single_bins(sc), nullptr, nullptr, false, rep));
  const int64_t Np = round_up(N, kTile);
  UCOV_TRY(ensure(c, c->q, 8 * 7 * N));
  UCOV_TRY(ensure(c, c->s, 8 * N));
  UCOV_TRY(ensure(c, c->amat, 8 * Np * Np));
  UCOV_TRY(ensure(c, c->fc_x, 8 * Np * Np));
  UCOV_TRY(ensure(c, c->tmat, 8 * std::max<int64_t>(1, spd_lower_inverse_scratch(Np))));
  if (paper) {
    UCOV_TRY(ensure(c, c->pg_f, 8 * paper_gauge_doubles(scene->n_pts)));
    if (pt_cov) {
      UCOV_TRY(ensure(c, c->fc_part, 8 * 7 * N * xq_splits(N)));
      UCOV_TRY(ensure(c, c->fc_xq, 8 * 7 * N));
      UCOV_TRY(ensure(c, c->fc_k, 8 * 49));
    }
  }
  SceneWork w = scene_work(c);
  hipStream_t st = c->stream;
  if (paper) {
    launch_paper_gauge(sc, w, as<double>(c->pg_f), c->ds, st);
    launch_gauge(N, nullptr, w.q, w.zdiag, nullptr, 0, 1.0, w.s, w.alpha, c->ds, st);
  } else {
    launch_gauge(N, w.hc, w.q, w.zdiag, nullptr, 0, o.alpha, w.s, w.alpha, c->ds, st);
  }
  hipEventRecord(c->ev[kEvGauge], st);
  double *A = as<double>(c->amat), *X = as<double>(c->fc_x);
  launch_assemble(sc, w, 1, A, Np, c->n_nonzero, st);
  launch_pad_identity(N, Np, A, Np, st);
  UCOV_TRY(check_hip(c, "assemble"));
  hipEventRecord(c->ev[kEvAssembled], st);
  spd_lower_inverse_fp64(A, Np, Np, as<double>(c->tmat), c->ds, st, c->small_for(Np));
  spd_inverse_from_factor(A, Np, Np, X, Np, st);
  hipEventRecord(c->ev[kEvInverse], st);
  if (cam_cov) launch_full_camera(N, X, Np, w.s, w.q, w.alpha, !paper, cam_cov, ldc, st);
  if (pt_cov) {
    if (paper) {
      double *xq = as<double>(c->fc_xq), *km = as<double>(c->fc_k);
      launch_xq(N, X, Np, w.s, w.q, as<double>(c->fc_part), xq, km, st);
      launch_point_cov(sc, w, X, Np, xq, as<double>(c->pg_f) + 28, km, true, pt_cov, st);
    } else {
      launch_point_cov(sc, w, X, Np, w.q, nullptr, nullptr, false, pt_cov, st);
    }
  }
  hipEventRecord(c->ev[kEvEnd], st);
  UCOV_TRY(check_hip(c, "whole covariance kernels"));
  UCOV_TRY(sync_status(c, rep, "whole covariance"));
  if (rep) hipMemcpy(&rep->alpha, c->alpha.p, sizeof(double), hipMemcpyDeviceToHost);
  report_stages(c, rep);
  return UCOV_OK;
}

// Incremental update (Sec. 6): the whole camera covariance after adding
// observations of existing points by existing cameras or by one new camera,
// by the Woodbury identity on the effective observation rows.
int ucov_update_covariance(ucov_ctx *c, const ucov_scene *scene, int64_t n_new,
                           const int32_t *new_cam, const int32_t *new_pt, const double *new_info,
                           const double *cam_new, double *cam_cov, int64_t ldc, double *new_cov,
                           double *new_cross, ucov_report *rep) {
  if (!c) return UCOV_EINVAL;
  UCOV_TRY(check_scene(c, scene));
  const int64_t n = scene->n_cams, m = scene->n_pts, N = 9 * n;
  if (n_new < 1 || !new_cam || !new_pt || !cam_cov || ldc < N)
    return c->fail(UCOV_EINVAL, "bad update arguments");
  if ((new_cov || new_cross) && !cam_new)
    return c->fail(UCOV_EINVAL, "new-camera outputs without a new camera");
  hipSetDevice(c->device);
  reset_report(rep);
  hipStream_t st = c->stream;
  // host bookkeeping of the new observations' indices
  std::vector<int32_t> hc(n_new), hp(n_new);
  if (hipMemcpyAsync(hc.data(), new_cam, 4 * n_new, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(hp.data(), new_pt, 4 * n_new, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return c->fail(UCOV_EDEVICE, "index readback");
  int64_t by_new = 0;
  for (int64_t a = 0; a < n_new; ++a) {
    if (hp[a] < 0 || hp[a] >= m || hc[a] < 0 || hc[a] > n || (hc[a] == n && !cam_new)) {
      if (rep) rep->bad_index = (int32_t)a;
      return c->fail(UCOV_EINVAL, "new observation index out of range");
    }
    by_new += hc[a] == n;
  }
  if (cam_new && by_new == 0) return c->fail(UCOV_EINVAL, "the new camera has no observations");
  std::vector<int32_t> ord(n_new), grp0(n_new);
  for (int64_t a = 0; a < n_new; ++a) ord[a] = (int32_t)a;
  std::sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
    return hp[x] != hp[y] ? hp[x] < hp[y] : (hc[x] != hc[y] ? hc[x] < hc[y] : x < y);
  });
  for (int64_t a = 0; a < n_new; ++a) {
    const bool same = a > 0 && hp[ord[a]] == hp[ord[a - 1]];
    if (same && hc[ord[a]] == hc[ord[a - 1]]) {
      if (rep) rep->bad_index = ord[a];
      return c->fail(UCOV_EINVAL, "duplicate new observation");
    }
    grp0[a] = same ? grp0[a - 1] : (int32_t)a;
  }
  // the old scene's point stage: Jacobians, V_j^-1, Y = J_X V^-1
  const SceneDev sc = scene_dev(scene);
  clear_status(c);
  UCOV_TRY(run_scene_stage(c, sc, 1, nullptr, nullptr, true, rep));
  SceneWork w = scene_work(c);
  launch_point_blocks(sc, w, c->ds, st);
  const int64_t Np = round_up(N, kTile), Kp = round_up(2 * n_new, kTile);
  UCOV_TRY(ensure(c, c->up_idx, 4 * 2 * n_new));
  UCOV_TRY(ensure(c, c->up_z, 8 * Np * Np));
  UCOV_TRY(ensure(c, c->up_jt, 8 * Np * Kp));
  UCOV_TRY(ensure(c, c->up_b, 8 * Np * Kp));
  UCOV_TRY(ensure(c, c->up_t, 8 * Np * Kp));
  UCOV_TRY(ensure(c, c->up_s, 8 * Kp * Kp));
  UCOV_TRY(ensure(c, c->up_tmp, 8 * std::max<int64_t>(1, spd_lower_inverse_scratch(Kp))));
  UCOV_TRY(ensure(c, c->up_nj, 8 * 24 * n_new));
  UCOV_TRY(ensure(c, c->up_jn, 8 * Kp * 64));
  if (cam_new) {
    UCOV_TRY(ensure(c, c->up_u, 8 * Kp * 64));
    UCOV_TRY(ensure(c, c->up_g, 8 * (64 * 64 + 2 * 81)));
    UCOV_TRY(ensure(c, c->up_v, 8 * Np * 64));
    UCOV_TRY(ensure(c, c->up_w, 8 * Np * 64));
  }
  int32_t *d_ord = as<int32_t>(c->up_idx), *d_grp = d_ord + n_new;
  if (hipMemcpyAsync(d_ord, ord.data(), 4 * n_new, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(d_grp, grp0.data(), 4 * n_new, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return c->fail(UCOV_EDEVICE, "index upload");
  double *Zp = as<double>(c->up_z), *jt = as<double>(c->up_jt), *B = as<double>(c->up_b),
         *T = as<double>(c->up_t), *S = as<double>(c->up_s), *jn = as<double>(c->up_jn),
         *nj = as<double>(c->up_nj);
  hipEventRecord(c->ev[kEvGauge], st);
  launch_copy_in(N, Np, cam_cov, ldc, Zp, st);
  fill_f64(jt, 0.0, Np * Kp, st);
  fill_f64(S, 0.0, Kp * Kp, st);
  fill_f64(jn, 0.0, Kp * 64, st);
  launch_new_jacobians(sc, n_new, d_ord, new_cam, new_pt, new_info, cam_new, nj, jn, Kp, c->ds,
                       st);
  launch_new_rows(sc, w, n_new, d_ord, new_cam, new_pt, d_grp, nj, jt, Np, S, Kp, c->ds, st);
  launch_pad_identity(2 * n_new, Kp, S, Kp, st);
  UCOV_TRY(check_hip(c, "update rows"));
  UCOV_TRY(sync_status(c, rep, "new observations"));
  hipEventRecord(c->ev[kEvAssembled], st);
  // B = Z^+ JtT, S += JtT^T B (lower), S = L L^T -> L^-1, T = B L^-T, Z^+ -= T T^T
  gemm_f64(false, false, false, Np, Kp, Np, Zp, Np, jt, Np, B, Np, 1.0, 0.0, kGemmFull, st);
  gemm_f64(true, false, true, Kp, Kp, Np, jt, Np, B, Np, S, Kp, 1.0, 1.0, kGemmFull, st);
  spd_lower_inverse_fp64(S, Kp, Kp, as<double>(c->up_tmp), c->ds, st);
  gemm_f64(false, true, false, Np, Kp, Kp, B, Np, S, Kp, T, Np, 1.0, 0.0, kGemmLeN, st);
  gemm_f64(false, true, false, Np, Np, Kp, T, Np, T, Np, Zp, Np, -1.0, 1.0, kGemmFull, st);
  if (cam_new) {
    // U = L^-1 J_n, C_n = (U^T U)^-1, V = T U, Z^+ += (V L_C)(V L_C)^T
    double *U = as<double>(c->up_u), *G = as<double>(c->up_g), *V = as<double>(c->up_v),
           *Wm = as<double>(c->up_w);
    double *cn = G + 64 * 64, *lc = cn + 81;
    gemm_f64(false, false, false, Kp, 64, Kp, S, Kp, jn, Kp, U, Kp, 1.0, 0.0, kGemmLeM, st);
    gemm_f64(true, false, false, 64, 64, Kp, U, Kp, U, Kp, G, 64, 1.0, 0.0, kGemmFull, st);
    gemm_f64(false, false, false, Np, 64, Kp, T, Np, U, Kp, V, Np, 1.0, 0.0, kGemmFull, st);
    launch_new_camera(G, cn, lc, N, Np, V, Wm, new_cross, c->ds, st);
    gemm_f64(false, true, false, Np, Np, 64, Wm, Np, Wm, Np, Zp, Np, 1.0, 1.0, kGemmFull, st);
    if (new_cov) hipMemcpyAsync(new_cov, cn, 8 * 81, hipMemcpyDeviceToDevice, st);
  }
  hipEventRecord(c->ev[kEvInverse], st);
  // errors found on the device (a factor that does not exist, a new camera
  // its observations do not determine) leave the caller's matrix untouched
  UCOV_TRY(check_hip(c, "update products"));
  UCOV_TRY(sync_status(c, rep, "covariance update"));
  launch_copy_out(N, Np, Zp, cam_cov, ldc, st);
  hipEventRecord(c->ev[kEvEnd], st);
  UCOV_TRY(check_hip(c, "update copy"));
  UCOV_TRY(sync_status(c, rep, "covariance update"));
  if (rep) {
    rep->ms_structure = ev_ms(c, kEvStart, kEvGauge);
    rep->ms_schur = ev_ms(c, kEvGauge, kEvAssembled);
    rep->ms_inverse = ev_ms(c, kEvAssembled, kEvInverse);
    rep->ms_extract = ev_ms(c, kEvInverse, kEvEnd);
  }
  return UCOV_OK;
}

// Tile schedule of the dense stage for matrices of size n: every candidate
// threshold for running the recursion's products on 32 x 32 instead of 64 x 64
// tiles is timed on a synthetic positive definite matrix of the padded size
// (best of three), and the fastest is kept for that size in this context.
int ucov_tune_dense(ucov_ctx *c, int64_t n, int64_t *threshold, float *ms) {
  if (!c) return UCOV_EINVAL;
  if (n < 1) return c->fail(UCOV_EINVAL, "n must be positive");
  hipSetDevice(c->device);
  const int64_t Np = round_up(n, kTile);
  UCOV_TRY(ensure(c, c->amat, 8 * Np * Np));
  UCOV_TRY(ensure(c, c->tmat, 8 * std::max<int64_t>(1, spd_lower_inverse_scratch(Np))));
  hipStream_t st = c->stream;
  clear_status(c);
  static const int64_t cand[] = {0, 256, 1024, 4096, (int64_t)1 << 40};
  int64_t best = kSmallTilesDefault;
  float best_ms = 0.0f;
  for (int64_t small : cand) {
    float t_min = 0.0f;
    for (int rep = 0; rep < 3; ++rep) {
      launch_tuning_matrix(Np, as<double>(c->amat), Np, st);
      hipEventRecord(c->ev[kEvTune0], st);
      spd_lower_inverse_fp64(as<double>(c->amat), Np, Np, as<double>(c->tmat), c->ds, st, small);
      hipEventRecord(c->ev[kEvTune1], st);
      if (hipEventSynchronize(c->ev[kEvTune1]) != hipSuccess)
        return c->fail(UCOV_EDEVICE, "tuning run");
      const float t = ev_ms(c, kEvTune0, kEvTune1);
      if (rep == 0 || t < t_min) t_min = t;
    }
    if (best_ms == 0.0f || t_min < best_ms) {
      best_ms = t_min;
      best = small;
    }
  }
  UCOV_TRY(check_hip(c, "tuning"));
  UCOV_TRY(sync_status(c, nullptr, "tuning"));
  c->small_tiles[Np] = best;
  if (threshold) *threshold = best;
  if (ms) *ms = best_ms;
  return UCOV_OK;
}

// The batched dense stage's tile schedule for scenes of sizes n[0..count):
// every candidate threshold is timed on synthetic positive definite matrices
// of those padded sizes run as one batched recursion (best of three), and the
// fastest is kept for that list of sizes.
int ucov_tune_batched(ucov_ctx *c, int32_t count, const int64_t *n, int64_t *threshold,
                      float *ms) {
  if (!c) return UCOV_EINVAL;
  if (count < 1 || !n) return c->fail(UCOV_EINVAL, "bad batch sizes");
  std::vector<int64_t> np(count), a_off(count + 1, 0);
  for (int s = 0; s < count; ++s) {
    if (n[s] < 1) return c->fail(UCOV_EINVAL, "sizes must be positive");
    np[s] = round_up(n[s], kTile);
    a_off[s + 1] = a_off[s] + np[s] * np[s];
  }
  hipSetDevice(c->device);
  hipStream_t st = c->stream;
  std::vector<int64_t> need(count), tmp_off(count + 1, 0);
  spd_batch_scratch(np.data(), count, need.data());
  for (int s = 0; s < count; ++s)
    tmp_off[s + 1] = tmp_off[s] + round_up(std::max<int64_t>(need[s], 1), 32);
  UCOV_TRY(ensure(c, c->amat, 8 * (size_t)a_off[count]));
  UCOV_TRY(ensure(c, c->b_scratch, 8 * (size_t)tmp_off[count]));
  UCOV_TRY(ensure(c, c->b_ds, sizeof(DevStatus) * count));
  DevStatus *bds = as<DevStatus>(c->b_ds);
  std::vector<SpdMat> mats(count);
  for (int s = 0; s < count; ++s)
    mats[s] = SpdMat{as<double>(c->amat) + a_off[s], np[s], np[s],
                     as<double>(c->b_scratch) + tmp_off[s], bds + s};
  if (!c->plan) c->plan = spd_plan_create();
  static const int64_t cand[] = {0, 256, 1024, 4096, (int64_t)1 << 40};
  int64_t best = 0;
  float best_ms = 0.0f;
  for (int64_t small : cand) {
    if (spd_plan_build(c->plan, mats.data(), count, st, small) != 0) {
      hipGetLastError();
      return c->fail(UCOV_ENOMEM, "batched inverse plan tables");
    }
    float t_min = 0.0f;
    for (int rep = 0; rep < 3; ++rep) {
      for (int s = 0; s < count; ++s) launch_tuning_matrix(np[s], as<double>(c->amat) + a_off[s], np[s], st);
      fill_i32(reinterpret_cast<int32_t *>(bds), 0, 2 * (int64_t)count, st);
      hipEventRecord(c->ev[kEvTune0], st);
      spd_plan_run(c->plan, st);
      hipEventRecord(c->ev[kEvTune1], st);
      if (hipEventSynchronize(c->ev[kEvTune1]) != hipSuccess)
        return c->fail(UCOV_EDEVICE, "batched tuning run");
      const float t = ev_ms(c, kEvTune0, kEvTune1);
      if (rep == 0 || t < t_min) t_min = t;
    }
    if (best_ms == 0.0f || t_min < best_ms) {
      best_ms = t_min;
      best = small;
    }
  }
  UCOV_TRY(check_hip(c, "batched tuning"));
  c->batch_small[np] = best;
  if (threshold) *threshold = best;
  if (ms) *ms = best_ms;
  return UCOV_OK;
}

int ucov_set_dense_threshold(ucov_ctx *c, int64_t n, int64_t threshold) {
  if (!c) return UCOV_EINVAL;
  if (n < 1 || threshold < 0) return c->fail(UCOV_EINVAL, "n must be positive, threshold >= 0");
  c->small_tiles[round_up(n, kTile)] = threshold;
  return UCOV_OK;
}

// Several independent scenes in one call.  The scene stage runs once over the
// concatenation (one launch per kernel for all scenes: camera-pair bins, the
// gauge basis and the dense matrices are kept per scene); the dense inverses
// of all scenes then run as one batched recursion whose every launch serves a
// node of the recursion for all the scenes that reach it.
}  // extern "C"

namespace {

// Offsets of the scenes of a batch in the concatenation.
struct BatchOffsets {
  std::vector<int32_t> cam_off, pt_off;
  std::vector<int64_t> obs_off;
};

// A failure of the scene stage names a global observation, point or camera:
// translate it into (scene, local index).
int localize_batch_error(ucov_ctx *c, const BatchOffsets &o, int rc, ucov_report *rep) {
  if (rc == UCOV_OK || !rep || rep->bad_index < 0) return rc;
  const int S = (int)o.cam_off.size() - 1;
  const int64_t g = rep->bad_index;
  int s = 0;
  int64_t base = 0;
  if (rc == UCOV_EINVAL) {
    s = (int)(std::upper_bound(o.obs_off.begin(), o.obs_off.end(), g) - o.obs_off.begin()) - 1;
    s = std::min(std::max(s, 0), S - 1);
    base = o.obs_off[s];
  } else if (rc == UCOV_EPOINT) {
    s = (int)(std::upper_bound(o.pt_off.begin(), o.pt_off.end(), (int32_t)g) - o.pt_off.begin()) - 1;
    s = std::min(std::max(s, 0), S - 1);
    base = o.pt_off[s];
  } else if (rc == UCOV_EGAUGE) {
    s = (int)(std::upper_bound(o.cam_off.begin(), o.cam_off.end(), (int32_t)g) - o.cam_off.begin()) - 1;
    s = std::min(std::max(s, 0), S - 1);
    base = o.cam_off[s];
  } else {
    return rc;
  }
  rep->bad_scene = s;
  rep->bad_index = (int32_t)(g - base);
  c->last_error += " in scene " + std::to_string(s) + ", local index " + std::to_string(g - base);
  return rc;
}

// Status of a batched solve once the stream has drained: the global status
// word (scene stage), then every scene's dense-stage status.
int batch_status(ucov_ctx *c, int S, const BatchOffsets &offs, ucov_report *rep) {
  hipStream_t st = c->stream;
  if (c->h_ds_cap < (size_t)S) {
    if (c->h_ds) hipHostFree(c->h_ds);
    c->h_ds = nullptr;
    c->h_ds_cap = 0;
    if (hipHostMalloc(&c->h_ds, sizeof(DevStatus) * S) != hipSuccess) {
      hipGetLastError();
      hipStreamSynchronize(st);
      return c->fail(UCOV_ENOMEM, "pinned status buffer");
    }
    c->h_ds_cap = S;
  }
  hipMemcpyAsync(c->h_ds, c->b_ds.p, sizeof(DevStatus) * S, hipMemcpyDeviceToHost, st);
  {
    const int rc = sync_status(c, rep, "batched solve");
    if (rc != UCOV_OK) return localize_batch_error(c, offs, rc, rep);
  }
  for (int s = 0; s < S; ++s) {
    if (c->h_ds[s].code != 0) {
      if (rep) {
        rep->bad_scene = s;
        rep->bad_index = c->h_ds[s].index;
      }
      char buf[160];
      snprintf(buf, sizeof buf, "dense inverse of scene %d (camera %d)", s, c->h_ds[s].index);
      return c->fail(c->h_ds[s].code, buf);
    }
  }
  return UCOV_OK;
}

}  // namespace

extern "C" {

int ucov_camera_covariance_batched(ucov_ctx *c, int32_t n_scenes, const ucov_scene *scenes,
                                   const ucov_options *opt, double *cov_out, double *alphas,
                                   ucov_report *rep) {
  if (!c) return UCOV_EINVAL;
  reset_report(rep);
  if (n_scenes < 1 || !scenes || !cov_out) return c->fail(UCOV_EINVAL, "bad batch arguments");
  ucov_options o;
  fill_defaults(opt, o);
  UCOV_TRY(device_only(c, o));
  if (o.precision != UCOV_FP64 || o.gauge != UCOV_GAUGE_CAMERA)
    return c->fail(UCOV_EINVAL, "batched calls support UCOV_FP64 with UCOV_GAUGE_CAMERA only");
  const int S = n_scenes;
  // host tables: offsets of every scene in the concatenation
  std::vector<int32_t> cam_off(S + 1), pt_off(S + 1);
  std::vector<int64_t> obs_off(S + 1), bin_off(S + 1), a_off(S + 1), a_ld(S);
  bool any_info = false;
  int64_t max_elems = 0;
  {
    int64_t nc = 0, np = 0, no = 0, nb = 0, na = 0;
    for (int s = 0; s < S; ++s) {
      const int rc = check_scene(c, &scenes[s]);
      if (rc != UCOV_OK) {
        if (rep) rep->bad_scene = s;
        return rc;
      }
      const ucov_scene &e = scenes[s];
      cam_off[s] = (int32_t)nc;
      pt_off[s] = (int32_t)np;
      obs_off[s] = no;
      bin_off[s] = nb;
      a_off[s] = na;
      const int64_t Np = round_up(9 * (int64_t)e.n_cams, kTile);
      a_ld[s] = Np;
      nc += e.n_cams;
      np += e.n_pts;
      no += e.n_obs;
      nb += (int64_t)e.n_cams * (e.n_cams + 1) / 2;
      na += Np * Np;
      any_info |= e.obs_info != nullptr;
      max_elems = std::max({max_elems, e.n_obs, 9 * (int64_t)e.n_cams, 3 * (int64_t)e.n_pts});
      if (nc > (int64_t)1 << 27 || np >= (int64_t)1 << 31 || no >= (int64_t)1 << 31)
        return c->fail(UCOV_EINVAL, "batch too large: at most 2^27 cameras and 2^31 - 1 points "
                                    "and observations in total");
    }
    cam_off[S] = (int32_t)nc;
    pt_off[S] = (int32_t)np;
    obs_off[S] = no;
    bin_off[S] = nb;
    a_off[S] = na;
  }
  const int64_t n = cam_off[S], m = pt_off[S], t = obs_off[S];
  const int64_t N = 9 * n;
  hipSetDevice(c->device);
  hipStream_t st = c->stream;

  // staged tables: [entries | cam_off | bin_off | a_off | a_ld], 8-byte aligned
  const size_t sz_tab = sizeof(BatchEntry) * S, sz_co = round_up(4 * (S + 1), 8),
               sz_bo = 8 * (S + 1), sz_ao = 8 * (S + 1), sz_ld = 8 * S;
  const size_t total = sz_tab + sz_co + sz_bo + sz_ao + sz_ld;
  if (c->h_stage_cap < total) {
    if (c->h_stage) hipHostFree(c->h_stage);
    c->h_stage = nullptr;
    c->h_stage_cap = 0;
    if (hipHostMalloc(&c->h_stage, total) != hipSuccess) {
      hipGetLastError();
      return c->fail(UCOV_ENOMEM, "pinned staging buffer");
    }
    c->h_stage_cap = total;
  }
  char *hs = static_cast<char *>(c->h_stage);
  BatchEntry *tab = reinterpret_cast<BatchEntry *>(hs);
  for (int s = 0; s < S; ++s) {
    const ucov_scene &e = scenes[s];
    tab[s] = BatchEntry{e.cams, e.pts, e.obs_info, e.obs_cam, e.obs_pt, e.n_cams, e.n_pts,
                        e.n_obs, cam_off[s], pt_off[s], obs_off[s]};
  }
  memcpy(hs + sz_tab, cam_off.data(), 4 * (S + 1));
  memcpy(hs + sz_tab + sz_co, bin_off.data(), sz_bo);
  memcpy(hs + sz_tab + sz_co + sz_bo, a_off.data(), sz_ao);
  memcpy(hs + sz_tab + sz_co + sz_bo + sz_ao, a_ld.data(), sz_ld);

  UCOV_TRY(ensure(c, c->b_tab, total));
  UCOV_TRY(ensure(c, c->b_cams, 8 * 9 * n));
  UCOV_TRY(ensure(c, c->b_pts, 8 * 3 * m));
  UCOV_TRY(ensure(c, c->b_oc, 4 * t));
  UCOV_TRY(ensure(c, c->b_op, 4 * t));
  UCOV_TRY(ensure(c, c->b_cam_scene, 4 * n));
  UCOV_TRY(ensure(c, c->b_ds, sizeof(DevStatus) * S));
  if (any_info) UCOV_TRY(ensure(c, c->b_info, 8 * 3 * t));
  char *dt = static_cast<char *>(c->b_tab.p);
  mark(c, kEvBatch, st);
  if (!c->replay) hipMemcpyAsync(dt, hs, total, hipMemcpyHostToDevice, st);
  clear_status(c);
  launch_concat_scenes(S, reinterpret_cast<const BatchEntry *>(dt), max_elems,
                       as<double>(c->b_cams), as<double>(c->b_pts),
                       any_info ? as<double>(c->b_info) : nullptr, as<int32_t>(c->b_oc),
                       as<int32_t>(c->b_op), as<int32_t>(c->b_cam_scene), c->ds, st);
  SceneDev sc;
  sc.n = (int)n;
  sc.m = (int)m;
  sc.t = t;
  sc.cams = as<double>(c->b_cams);
  sc.pts = as<double>(c->b_pts);
  sc.info = any_info ? as<double>(c->b_info) : nullptr;
  sc.oc = as<int32_t>(c->b_oc);
  sc.op = as<int32_t>(c->b_op);
  sc.n_scenes = S;
  sc.cam_scene = as<int32_t>(c->b_cam_scene);
  sc.cam_off = reinterpret_cast<const int32_t *>(dt + sz_tab);
  sc.bin_off = reinterpret_cast<const int64_t *>(dt + sz_tab + sz_co);
  sc.a_off = reinterpret_cast<const int64_t *>(dt + sz_tab + sz_co + sz_bo);
  sc.a_ld = reinterpret_cast<const int64_t *>(dt + sz_tab + sz_co + sz_bo + sz_ao);

  const BatchOffsets offs{cam_off, pt_off, obs_off};
  auto localize = [&](int rc) { return localize_batch_error(c, offs, rc, rep); };
  int64_t max_cams = 0;
  for (int s = 0; s < S; ++s) max_cams = std::max<int64_t>(max_cams, cam_off[s + 1] - cam_off[s]);
  {
    const int rc = run_scene_stage(c, sc, bin_off[S], nullptr, nullptr, false, rep, max_cams);
    if (rc != UCOV_OK) return localize(rc);
  }
  UCOV_TRY(ensure(c, c->q, 8 * 7 * N));
  UCOV_TRY(ensure(c, c->s, 8 * N));
  UCOV_TRY(ensure(c, c->alpha, 8 * S));
  UCOV_TRY(ensure(c, c->amat, 8 * std::max<int64_t>(1, a_off[S])));
  SceneWork w = scene_work(c);
  launch_gauge_scenes(sc, w.hc, w.q, w.zdiag, o.alpha, w.s, w.alpha, c->ds, st);
  mark(c, kEvGauge, st);
  launch_assemble(sc, w, 1, as<double>(c->amat), 0, c->n_nonzero, st, max_cams);
  mark(c, kEvAssembled, st);
  UCOV_TRY(check_hip(c, "batched assemble"));
  if (!c->replay) {
    const int rc = sync_status(c, rep, "batched gauge");
    if (rc != UCOV_OK) return localize(rc);
  }

  // dense stage: one batched recursion over all scenes (each launch serves a
  // node of the recursion for every scene that reaches it)
  std::vector<int64_t> need(S);
  spd_batch_scratch(a_ld.data(), S, need.data());
  std::vector<int64_t> tmp_off(S + 1, 0);
  for (int s = 0; s < S; ++s) tmp_off[s + 1] = tmp_off[s] + round_up(std::max<int64_t>(need[s], 1), 32);
  UCOV_TRY(ensure(c, c->b_scratch, 8 * (size_t)tmp_off[S]));
  DevStatus *bds = as<DevStatus>(c->b_ds);
  double *amat = as<double>(c->amat);
  std::vector<SpdMat> mats(S);
  int64_t max_np = 0;
  for (int s = 0; s < S; ++s) {
    mats[s] = SpdMat{amat + a_off[s], a_ld[s], a_ld[s], as<double>(c->b_scratch) + tmp_off[s], bds + s};
    max_np = std::max(max_np, a_ld[s]);
  }
  if (!c->plan) c->plan = spd_plan_create();
  if (!c->replay) {
    const int rc = spd_plan_build(c->plan, mats.data(), S, st, c->batch_small_for(a_ld));
    if (rc == -2) return c->fail(UCOV_EDEVICE, "internal error: batched inverse plan out of bounds");
    if (rc != 0) {
      hipGetLastError();
      return c->fail(UCOV_ENOMEM, "batched inverse plan tables");
    }
  }
  mark(c, kEvTune0, st);
  fill_i32(reinterpret_cast<int32_t *>(bds), 0, 2 * (int64_t)S, st);
  launch_pad_identity_scenes(S, max_np, sc.cam_off, sc.a_off, sc.a_ld, amat, st);
  spd_plan_run(c->plan, st);
  mark(c, kEvInverse, st);
  launch_extract_scenes(n, sc.cam_scene, sc.cam_off, sc.a_off, sc.a_ld, amat, w.s, w.q, w.alpha,
                        cov_out, st);
  mark(c, kEvEnd, st);
  UCOV_TRY(check_hip(c, "batched dense kernels"));
  if (c->replay) return UCOV_OK;  // the run of the recorded sequence checks the status
  UCOV_TRY(batch_status(c, S, offs, rep));
  if (alphas) hipMemcpy(alphas, c->alpha.p, 8 * (size_t)S, hipMemcpyDeviceToHost);
  if (rep) {
    hipMemcpy(&rep->alpha, c->alpha.p, sizeof(double), hipMemcpyDeviceToHost);
    report_stages(c, rep);
    rep->ms_structure += ev_ms(c, kEvBatch, kEvStart);
    rep->ms_inverse = ev_ms(c, kEvTune0, kEvInverse);
    rep->ms_total = ev_ms(c, kEvBatch, kEvEnd);
  }
  return UCOV_OK;
}

// ---- a batch recorded once and replayed ---------------------------------------

}  // extern "C"

struct ucov_batch {
  ucov_ctx *parent = nullptr;
  ucov_ctx *w = nullptr;          // private workspace that the graph uses
  hipStream_t cap = nullptr;      // stream the graph was recorded on
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int S = 0;
  BatchOffsets offs;
  ucov_report first{};            // report of the eager solve
};

extern "C" {

void ucov_batch_destroy(ucov_batch *b) {
  if (!b) return;
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->w) {
    b->w->stream = b->cap;
    ucov_destroy(b->w);
  }
  if (b->cap) hipStreamDestroy(b->cap);
  delete b;
}

int ucov_batch_create(ucov_ctx *c, int32_t n_scenes, const ucov_scene *scenes,
                      const ucov_options *opt, double *cov_out, ucov_batch **batch) {
  if (!c) return UCOV_EINVAL;
  if (!batch) return c->fail(UCOV_EINVAL, "NULL batch handle");
  *batch = nullptr;
  if (n_scenes < 1 || !scenes || !cov_out) return c->fail(UCOV_EINVAL, "bad batch arguments");
  hipSetDevice(c->device);
  ucov_batch *b = new ucov_batch();
  b->parent = c;
  b->S = n_scenes;
  if (ucov_create(&b->w, c->device) != UCOV_OK) {
    delete b;
    return c->fail(UCOV_ENOMEM, "private workspace of the batch");
  }
  b->w->small_tiles = c->small_tiles;
  b->w->batch_small = c->batch_small;
  if (hipStreamCreate(&b->cap) != hipSuccess) {
    hipGetLastError();
    ucov_batch_destroy(b);
    return c->fail(UCOV_EDEVICE, "stream of the batch");
  }
  ucov_ctx *w = b->w;
  w->stream = b->cap;
  // the eager solve validates the scenes, sizes every buffer and builds the
  // dense plan; its results are the first run's
  int rc = ucov_camera_covariance_batched(w, n_scenes, scenes, opt, cov_out, nullptr, &b->first);
  if (rc != UCOV_OK) {
    c->last_error = w->last_error;
    ucov_batch_destroy(b);
    return rc;
  }
  for (int s = 0; s <= n_scenes; ++s) {
    b->offs.cam_off.push_back(s ? b->offs.cam_off.back() + scenes[s - 1].n_cams : 0);
    b->offs.pt_off.push_back(s ? b->offs.pt_off.back() + scenes[s - 1].n_pts : 0);
    b->offs.obs_off.push_back(s ? b->offs.obs_off.back() + scenes[s - 1].n_obs : 0);
  }
  // record the same launches, with no host round trip, into a graph
  w->replay = true;
  if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    w->replay = false;
    hipGetLastError();
    ucov_batch_destroy(b);
    return c->fail(UCOV_EDEVICE, "beginning the graph capture");
  }
  rc = ucov_camera_covariance_batched(w, n_scenes, scenes, opt, cov_out, nullptr, nullptr);
  const hipError_t e = hipStreamEndCapture(b->cap, &b->graph);
  w->replay = false;
  if (rc != UCOV_OK || e != hipSuccess) {
    hipGetLastError();
    c->last_error = rc != UCOV_OK ? w->last_error : std::string("graph capture failed");
    ucov_batch_destroy(b);
    return rc != UCOV_OK ? rc : UCOV_EDEVICE;
  }
  if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
    hipGetLastError();
    ucov_batch_destroy(b);
    return c->fail(UCOV_EDEVICE, "graph instantiation");
  }
  *batch = b;
  return UCOV_OK;
}

int ucov_batch_run(ucov_batch *b, ucov_report *rep) {
  if (!b) return UCOV_EINVAL;
  reset_report(rep);
  ucov_ctx *c = b->parent, *w = b->w;
  hipSetDevice(w->device);
  w->stream = c->stream;  // the caller's stream
  hipEventRecord(w->ev[kEvTune0], w->stream);
  if (hipGraphLaunch(b->exec, w->stream) != hipSuccess) {
    hipGetLastError();
    return c->fail(UCOV_EDEVICE, "graph launch");
  }
  hipEventRecord(w->ev[kEvTune1], w->stream);
  const int rc = batch_status(w, b->S, b->offs, rep);
  if (rc != UCOV_OK) {
    c->last_error = w->last_error;
    return rc;
  }
  if (rep) {
    hipMemcpy(&rep->alpha, w->alpha.p, sizeof(double), hipMemcpyDeviceToHost);
    rep->n_pairs = b->first.n_pairs;
    rep->ms_total = ev_ms(w, kEvTune0, kEvTune1);
  }
  return UCOV_OK;
}

// ---- sub-reconstructions (Sec. 6) --------------------------------------------

int ucov_subrecon_covariance(ucov_ctx *c, const ucov_scene *scene, int32_t n_decomp,
                             const int32_t *groups, const ucov_options *opt, double *cov_out,
                             int32_t *chosen, int32_t *n_sub, ucov_report *rep) {
  if (!c) return UCOV_EINVAL;
  reset_report(rep);
  UCOV_TRY(check_scene(c, scene));
  if (n_decomp < 1 || !groups || !cov_out) return c->fail(UCOV_EINVAL, "bad sub-reconstruction arguments");
  const int64_t n = scene->n_cams, m = scene->n_pts, t = scene->n_obs;
  for (int64_t k = 0; k < (int64_t)n_decomp * n; ++k)
    if (groups[k] < 0 || groups[k] >= n) return c->fail(UCOV_EINVAL, "group id out of range");
  hipSetDevice(c->device);
  hipStream_t st = c->stream;
  const int64_t T = (int64_t)n_decomp * t;
  if (T >= ((int64_t)1 << 31))
    return c->fail(UCOV_EINVAL, "n_decomp x n_obs must be below 2^31");
  // sub-scenes in the order (decomposition, group by first appearance): per
  // camera and decomposition its sub-scene, its slot there and its row in the
  // concatenation of the sub-scenes' cameras
  std::vector<int32_t> gsub((size_t)n_decomp * n), cslot((size_t)n_decomp * n),
      pos((size_t)n_decomp * n), cam_src;
  std::vector<int64_t> cam_off{0};
  cam_src.reserve((size_t)n_decomp * n);
  for (int d = 0; d < n_decomp; ++d) {
    const int32_t *g = groups + (int64_t)d * n;
    std::vector<int32_t> gidx(n, -1), size;
    const int32_t base = (int32_t)cam_off.size() - 1;
    for (int64_t cam = 0; cam < n; ++cam) {
      if (gidx[g[cam]] < 0) {
        gidx[g[cam]] = (int32_t)size.size();
        size.push_back(0);
      }
      const int32_t sub = gidx[g[cam]];
      gsub[(size_t)d * n + cam] = base + sub;
      cslot[(size_t)d * n + cam] = size[sub]++;
    }
    std::vector<int64_t> first(size.size());
    for (size_t sub = 0; sub < size.size(); ++sub) {
      first[sub] = cam_off.back();
      cam_off.push_back(cam_off.back() + size[sub]);
    }
    cam_src.resize(cam_off.back());
    for (int64_t cam = 0; cam < n; ++cam) {
      const int64_t row = first[gidx[g[cam]]] + cslot[(size_t)d * n + cam];
      cam_src[row] = (int32_t)cam;
      pos[(size_t)d * n + cam] = (int32_t)row;
    }
  }
  const int S = (int)cam_off.size() - 1;
  const int64_t nt = cam_off.back();
  if (n_sub) *n_sub = S;
  // device index maps: cam_src | pos | gsub | cslot (n_decomp x n each), then
  // obs_src | loc_c | loc_p | pt_src (at most n_decomp x t each)
  const int64_t nd = (int64_t)n_decomp * n;
  UCOV_TRY(ensure(c, c->sr_idx, 4 * (size_t)(4 * nd + 4 * T)));
  UCOV_TRY(ensure(c, c->sr_off, 8 * 2 * (size_t)(S + 1)));
  UCOV_TRY(ensure(c, c->sr_tmp, subscene_select_scratch(T)));
  int32_t *idx = as<int32_t>(c->sr_idx);
  int32_t *d_cam_src = idx, *d_pos = idx + nd, *d_gsub = idx + 2 * nd, *d_cslot = idx + 3 * nd;
  int32_t *d_obs_src = idx + 4 * nd, *d_loc_c = d_obs_src + T, *d_loc_p = d_loc_c + T,
          *d_pt_src = d_loc_p + T;
  int64_t *d_obs_off = as<int64_t>(c->sr_off), *d_pt_off = d_obs_off + (S + 1);
  const std::pair<const std::vector<int32_t> *, int32_t *> up[] = {
      {&cam_src, d_cam_src}, {&pos, d_pos}, {&gsub, d_gsub}, {&cslot, d_cslot}};
  for (const auto &u : up)
    if (hipMemcpyAsync(u.second, u.first->data(), 4 * u.first->size(), hipMemcpyHostToDevice,
                       st) != hipSuccess)
      return check_hip(c, "sub-reconstruction index upload");
  clear_status(c);
  launch_subscene_select(t, n_decomp, (int32_t)n, (int32_t)m, S, scene->obs_cam, scene->obs_pt,
                         d_gsub, d_cslot, c->sr_tmp.p, d_obs_off, d_pt_off, d_obs_src, d_loc_c,
                         d_loc_p, d_pt_src, c->ds, st);
  UCOV_TRY(check_hip(c, "sub-scene selection"));
  std::vector<int64_t> offs(2 * (size_t)(S + 1));
  if (hipMemcpyAsync(offs.data(), d_obs_off, 8 * offs.size(), hipMemcpyDeviceToHost, st) !=
      hipSuccess)
    return check_hip(c, "sub-scene sizes");
  UCOV_TRY(sync_status(c, rep, "observation index out of range"));
  const int64_t *obs_off = offs.data(), *pt_off = offs.data() + (S + 1);
  const int64_t mt = pt_off[S], tt = obs_off[S];
  UCOV_TRY(ensure(c, c->sr_cams, 8 * 9 * (size_t)nt));
  UCOV_TRY(ensure(c, c->sr_pts, 8 * 3 * (size_t)std::max<int64_t>(mt, 1)));
  if (scene->obs_info) UCOV_TRY(ensure(c, c->sr_info, 8 * 3 * (size_t)std::max<int64_t>(tt, 1)));
  launch_gather_subscenes(nt, mt, tt, d_cam_src, d_pt_src, d_obs_src, scene->cams, scene->pts,
                          scene->obs_info, as<double>(c->sr_cams), as<double>(c->sr_pts),
                          scene->obs_info ? as<double>(c->sr_info) : nullptr, st);
  UCOV_TRY(check_hip(c, "sub-scene gather"));
  std::vector<ucov_scene> subs(S);
  for (int k = 0; k < S; ++k) {
    subs[k].n_cams = (int32_t)(cam_off[k + 1] - cam_off[k]);
    subs[k].n_pts = (int32_t)(pt_off[k + 1] - pt_off[k]);
    subs[k].n_obs = obs_off[k + 1] - obs_off[k];
    subs[k].cams = as<double>(c->sr_cams) + 9 * cam_off[k];
    subs[k].pts = as<double>(c->sr_pts) + 3 * pt_off[k];
    subs[k].obs_cam = d_loc_c + obs_off[k];
    subs[k].obs_pt = d_loc_p + obs_off[k];
    subs[k].obs_info = scene->obs_info ? as<double>(c->sr_info) + 3 * obs_off[k] : nullptr;
  }
  UCOV_TRY(ensure(c, c->sr_cand, 8 * 81 * (size_t)nt));
  UCOV_TRY(ucov_camera_covariance_batched(c, S, subs.data(), opt, as<double>(c->sr_cand),
                                          nullptr, rep));
  int32_t *d_chosen = nullptr;
  if (chosen) {
    UCOV_TRY(ensure(c, c->sr_chosen, 4 * (size_t)n));
    d_chosen = as<int32_t>(c->sr_chosen);
  }
  launch_min_trace(n, n_decomp, d_pos, as<double>(c->sr_cand), cov_out, d_chosen, st);
  if (chosen) hipMemcpyAsync(chosen, d_chosen, 4 * (size_t)n, hipMemcpyDeviceToHost, st);
  UCOV_TRY(check_hip(c, "minimum-trace choice"));
  if (hipStreamSynchronize(st) != hipSuccess) return check_hip(c, "sub-reconstructions");
  return UCOV_OK;
}

// ---- learned screener -------------------------------------------------------

int64_t ucov_mlp_param_count(void) { return mlp_param_count(); }

int ucov_screener_features(ucov_ctx *c, const ucov_scene *scene, float *feat) {
  if (!c) return UCOV_EINVAL;
  UCOV_TRY(check_scene(c, scene));
  if (!feat) return c->fail(UCOV_EINVAL, "NULL output");
  hipSetDevice(c->device);
  const SceneDev sc = scene_dev(scene);
  clear_status(c);
  UCOV_TRY(run_scene_stage(c, sc, single_bins(sc), nullptr, nullptr, false, nullptr));
  const int64_t n = sc.n;
  UCOV_TRY(ensure(c, c->f_hist, 4 * 8 * n));
  UCOV_TRY(ensure(c, c->f_ang, 8 * n));
  UCOV_TRY(ensure(c, c->f_covis, 4 * n));
  launch_screener_features(sc, scene_work(c), as<int32_t>(c->f_hist), as<double>(c->f_ang),
                           as<int32_t>(c->f_covis), feat, c->stream);
  UCOV_TRY(check_hip(c, "screener features"));
  return sync_status(c, nullptr, "screener features");
}

namespace {
int check_mlp_args(ucov_ctx *c, const float *params, int64_t batch, const float *x,
                   const float *mean, const float *stdv) {
  if (!params || !x || batch < 1 || batch > ((int64_t)1 << 24))
    return c->fail(UCOV_EINVAL, "bad MLP arguments (batch must be in [1, 2^24])");
  if ((mean == nullptr) != (stdv == nullptr))
    return c->fail(UCOV_EINVAL, "in_mean and in_std must both be given or both be NULL");
  return UCOV_OK;
}
}  // namespace

int ucov_mlp_forward(ucov_ctx *c, const float *params, int64_t batch, const float *x,
                     const float *in_mean, const float *in_std, float *y) {
  if (!c) return UCOV_EINVAL;
  UCOV_TRY(check_mlp_args(c, params, batch, x, in_mean, in_std));
  if (!y) return c->fail(UCOV_EINVAL, "NULL output");
  hipSetDevice(c->device);
  UCOV_TRY(ensure(c, c->mlp_ws, mlp_workspace_bytes(batch)));
  mlp_forward(params, batch, x, in_mean, in_std, y, c->mlp_ws.p, c->stream);
  UCOV_TRY(check_hip(c, "MLP forward"));
  if (hipStreamSynchronize(c->stream) != hipSuccess) return check_hip(c, "MLP forward");
  return UCOV_OK;
}

int ucov_mlp_gradient(ucov_ctx *c, const float *params, int64_t batch, const float *x,
                      const float *in_mean, const float *in_std, const float *target,
                      float *grad, float *loss) {
  if (!c) return UCOV_EINVAL;
  UCOV_TRY(check_mlp_args(c, params, batch, x, in_mean, in_std));
  if (!target || !grad) return c->fail(UCOV_EINVAL, "NULL target or gradient");
  hipSetDevice(c->device);
  UCOV_TRY(ensure(c, c->mlp_ws, mlp_workspace_bytes(batch)));
  mlp_gradient(params, batch, x, in_mean, in_std, target, grad, loss, c->mlp_ws.p, c->stream);
  UCOV_TRY(check_hip(c, "MLP gradient"));
  if (hipStreamSynchronize(c->stream) != hipSuccess) return check_hip(c, "MLP gradient");
  return UCOV_OK;
}

int ucov_mlp_train(ucov_ctx *c, float *params, float *adam_m, float *adam_v, int64_t step0,
                   float lr, int64_t batch, int64_t n_batches, const float *x,
                   const float *in_mean, const float *in_std, const float *target,
                   float *losses) {
  if (!c) return UCOV_EINVAL;
  UCOV_TRY(check_mlp_args(c, params, batch, x, in_mean, in_std));
  if (!adam_m || !adam_v || !target || n_batches < 1 || step0 < 1 || !(lr > 0.f))
    return c->fail(UCOV_EINVAL, "bad training arguments");
  hipSetDevice(c->device);
  const int64_t P = mlp_param_count();
  UCOV_TRY(ensure(c, c->mlp_ws, mlp_workspace_bytes(batch)));
  UCOV_TRY(ensure(c, c->mlp_grad, 4 * P));
  float *g = as<float>(c->mlp_grad);
  for (int64_t i = 0; i < n_batches; ++i) {
    mlp_gradient(params, batch, x + i * batch * UCOV_SCREENER_FEATURES, in_mean, in_std,
                 target + i * batch * UCOV_SCREENER_OUTPUTS, g, losses ? losses + i : nullptr,
                 c->mlp_ws.p, c->stream);
    mlp_adam(P, params, g, adam_m, adam_v, lr, step0 + i, c->stream);
  }
  UCOV_TRY(check_hip(c, "MLP training"));
  if (hipStreamSynchronize(c->stream) != hipSuccess) return check_hip(c, "MLP training");
  return UCOV_OK;
}

int ucov_screener_labels(ucov_ctx *c, int64_t n, const double *cov, const float *feat,
                         const double *scale, const float *out_mean, const float *out_std,
                         float *labels) {
  if (!c) return UCOV_EINVAL;
  if (n < 1 || !cov || !feat || !scale || !out_mean || !out_std || !labels)
    return c->fail(UCOV_EINVAL, "bad label arguments");
  hipSetDevice(c->device);
  UCOV_TRY(ensure(c, c->f_bscale, 8 * 9 * (size_t)n));
  clear_status(c);
  launch_block_scale(n, feat, as<double>(c->f_bscale), c->ds, c->stream);
  launch_labels(n, cov, as<double>(c->f_bscale), scale, out_mean, out_std, true, labels, c->ds,
                c->stream);
  UCOV_TRY(check_hip(c, "screener labels"));
  return sync_status(c, nullptr, "screener labels (a block is not positive definite)");
}

int ucov_screener_covariance(ucov_ctx *c, int64_t n, const float *y, const float *feat,
                             const double *scale, const float *out_mean, const float *out_std,
                             double *cov, double *spread) {
  if (!c) return UCOV_EINVAL;
  if (n < 1 || !y || !feat || !scale || !out_mean || !out_std || (!cov && !spread))
    return c->fail(UCOV_EINVAL, "bad screener covariance arguments");
  hipSetDevice(c->device);
  UCOV_TRY(ensure(c, c->f_bscale, 8 * 9 * (size_t)n));
  clear_status(c);
  launch_block_scale(n, feat, as<double>(c->f_bscale), c->ds, c->stream);
  launch_predicted_cov(n, y, as<double>(c->f_bscale), scale, out_mean, out_std, cov, spread,
                       c->stream);
  UCOV_TRY(check_hip(c, "screener covariance"));
  return sync_status(c, nullptr, "screener covariance (a Z_ii block is not positive definite)");
}

int ucov_screener_stats(ucov_ctx *c, int64_t n, const float *feat, const double *cov,
                        float *in_mean, float *in_std, double *scale, float *out_mean,
                        float *out_std) {
  if (!c) return UCOV_EINVAL;
  if (n < 2 || !feat || !cov || !in_mean || !in_std || !scale || !out_mean || !out_std)
    return c->fail(UCOV_EINVAL, "bad statistics arguments (n >= 2, every array given)");
  hipSetDevice(c->device);
  hipStream_t st = c->stream;
  UCOV_TRY(ensure(c, c->f_lab, 4 * UCOV_SCREENER_OUTPUTS * (size_t)n));
  UCOV_TRY(ensure(c, c->f_bscale, 8 * 9 * (size_t)n));
  UCOV_TRY(ensure(c, c->f_zero, 8 * UCOV_SCREENER_OUTPUTS));
  float *zero = as<float>(c->f_zero), *one = zero + UCOV_SCREENER_OUTPUTS;
  double *bsc = as<double>(c->f_bscale);
  clear_status(c);
  fill_i32(reinterpret_cast<int32_t *>(zero), 0, UCOV_SCREENER_OUTPUTS, st);
  fill_i32(reinterpret_cast<int32_t *>(one), 0x3f800000, UCOV_SCREENER_OUTPUTS, st);  // 1.0f
  launch_col_stats(n, UCOV_SCREENER_FEATURES, feat, in_mean, in_std, st);
  launch_block_scale(n, feat, bsc, c->ds, st);
  launch_diag_median(n, cov, bsc, scale, st);
  launch_labels(n, cov, bsc, scale, zero, one, false, as<float>(c->f_lab), c->ds, st);
  launch_col_robust(n, UCOV_SCREENER_OUTPUTS, as<float>(c->f_lab), out_mean, out_std, st);
  UCOV_TRY(check_hip(c, "screener statistics"));
  return sync_status(c, nullptr, "screener statistics (a block is not positive definite)");
}

}  // extern "C"

namespace {

// Screener file: a 64-byte header, the payload, and an FNV-1a hash of the
// payload (all little-endian as written by the host).
struct ScreenerHeader {
  char magic[8];      // "UCOVSCR1"
  uint32_t version;   // 1
  uint32_t n_in, n_hidden, n_out, n_scale;
  uint32_t has_adam;  // 1: Adam moments follow the statistics
  int64_t n_params;
  int64_t step;
  char pad[64 - 8 - 6 * 4 - 2 * 8];
};
static_assert(sizeof(ScreenerHeader) == 64, "screener header is 64 bytes");

uint64_t fnv1a(uint64_t h, const void *p, size_t len) {
  const unsigned char *b = static_cast<const unsigned char *>(p);
  for (size_t i = 0; i < len; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

struct Part {
  void *dev;
  size_t bytes;
};

std::vector<Part> screener_parts(const ucov_screener *s, bool adam) {
  const size_t P = (size_t)mlp_param_count();
  std::vector<Part> v = {{s->params, 4 * P},
                         {s->in_mean, 4 * UCOV_SCREENER_FEATURES},
                         {s->in_std, 4 * UCOV_SCREENER_FEATURES},
                         {s->out_mean, 4 * UCOV_SCREENER_OUTPUTS},
                         {s->out_std, 4 * UCOV_SCREENER_OUTPUTS},
                         {s->scale, 8 * 9}};
  if (adam) {
    v.push_back({s->adam_m, 4 * P});
    v.push_back({s->adam_v, 4 * P});
  }
  return v;
}

}  // namespace

extern "C" {

int ucov_screener_save(ucov_ctx *c, const char *path, const ucov_screener *s) {
  if (!c) return UCOV_EINVAL;
  if (!path || !s || !s->params || !s->in_mean || !s->in_std || !s->scale || !s->out_mean ||
      !s->out_std || (s->adam_m == nullptr) != (s->adam_v == nullptr) || s->step < 0)
    return c->fail(UCOV_EINVAL, "bad screener arguments");
  hipSetDevice(c->device);
  const bool adam = s->adam_m != nullptr;
  const std::vector<Part> parts = screener_parts(s, adam);
  size_t total = 0;
  for (const Part &p : parts) total += p.bytes;
  std::vector<unsigned char> payload(total);
  if (hipStreamSynchronize(c->stream) != hipSuccess) return check_hip(c, "screener save");
  size_t off = 0;
  for (const Part &p : parts) {
    if (hipMemcpy(payload.data() + off, p.dev, p.bytes, hipMemcpyDeviceToHost) != hipSuccess)
      return check_hip(c, "screener save (device read)");
    off += p.bytes;
  }
  ScreenerHeader h{};
  memcpy(h.magic, "UCOVSCR1", 8);
  h.version = 1;
  h.n_in = UCOV_SCREENER_FEATURES;
  h.n_hidden = 256;
  h.n_out = UCOV_SCREENER_OUTPUTS;
  h.n_scale = 9;
  h.has_adam = adam ? 1 : 0;
  h.n_params = mlp_param_count();
  h.step = s->step;
  const uint64_t hash = fnv1a(1469598103934665603ull, payload.data(), payload.size());
  FILE *f = fopen(path, "wb");
  if (!f) return c->fail(UCOV_EINVAL, std::string("cannot open ") + path + " for writing");
  const bool ok = fwrite(&h, sizeof h, 1, f) == 1 &&
                  fwrite(payload.data(), 1, payload.size(), f) == payload.size() &&
                  fwrite(&hash, sizeof hash, 1, f) == 1;
  if (fclose(f) != 0 || !ok) return c->fail(UCOV_EINVAL, std::string("cannot write ") + path);
  return UCOV_OK;
}

int ucov_screener_load(ucov_ctx *c, const char *path, ucov_screener *s) {
  if (!c) return UCOV_EINVAL;
  if (!path || !s || !s->params || !s->in_mean || !s->in_std || !s->scale || !s->out_mean ||
      !s->out_std || (s->adam_m == nullptr) != (s->adam_v == nullptr))
    return c->fail(UCOV_EINVAL, "bad screener arguments");
  hipSetDevice(c->device);
  FILE *f = fopen(path, "rb");
  if (!f) return c->fail(UCOV_EINVAL, std::string("cannot open ") + path);
  ScreenerHeader h{};
  if (fread(&h, sizeof h, 1, f) != 1 || memcmp(h.magic, "UCOVSCR1", 8) != 0 || h.version != 1 ||
      h.n_in != UCOV_SCREENER_FEATURES || h.n_hidden != 256 || h.n_out != UCOV_SCREENER_OUTPUTS ||
      h.n_scale != 9 || h.n_params != mlp_param_count() || h.has_adam > 1 || h.step < 0) {
    fclose(f);
    return c->fail(UCOV_EINVAL, std::string(path) + " is not a screener file of this network");
  }
  const bool want_adam = s->adam_m != nullptr;
  if (want_adam && !h.has_adam) {
    fclose(f);
    return c->fail(UCOV_EINVAL, std::string(path) + " holds no Adam moments");
  }
  const std::vector<Part> parts = screener_parts(s, h.has_adam != 0);
  size_t total = 0;
  for (const Part &p : parts) total += p.bytes;
  std::vector<unsigned char> payload(total);
  uint64_t hash = 0;
  const bool ok = fread(payload.data(), 1, total, f) == total && fread(&hash, sizeof hash, 1, f) == 1;
  fclose(f);
  if (!ok || hash != fnv1a(1469598103934665603ull, payload.data(), payload.size()))
    return c->fail(UCOV_EINVAL, std::string(path) + " is truncated or corrupt");
  if (hipStreamSynchronize(c->stream) != hipSuccess) return check_hip(c, "screener load");
  size_t off = 0;
  for (const Part &p : parts) {
    const bool skip = !want_adam && (p.dev == s->adam_m || p.dev == s->adam_v);
    if (!skip && hipMemcpy(p.dev, payload.data() + off, p.bytes, hipMemcpyHostToDevice) != hipSuccess)
      return check_hip(c, "screener load (device write)");
    off += p.bytes;
  }
  s->step = h.step;
  return UCOV_OK;
}

int ucov_split_bf16_update(ucov_ctx *c, int64_t n, double *x, const double *r) {
  if (!c) return UCOV_EINVAL;
  if (n < 64 || n % 64 != 0 || !x || !r)
    return c->fail(UCOV_EINVAL, "n must be a positive multiple of 64, x and r given");
  hipSetDevice(c->device);
  UCOV_TRY(ensure(c, c->m_split, split_bf16_scratch(n)));
  split_bf16_update(n, x, r, c->m_split.p, c->stream);
  UCOV_TRY(check_hip(c, "split-BF16 update"));
  if (hipStreamSynchronize(c->stream) != hipSuccess) return check_hip(c, "split-BF16 update");
  return UCOV_OK;
}

int ucov_plan_check(const int64_t *np, int32_t count, int64_t *n_launches) {
  if (!np || count < 1) return UCOV_EINVAL;
  for (int32_t s = 0; s < count; ++s)
    if (np[s] < 64 || np[s] % 64 != 0) return UCOV_EINVAL;
  std::string why;
  return spd_plan_check_host(np, count, &why, n_launches) == 0 ? UCOV_OK : UCOV_EDEVICE;
}

const char *ucov_strerror(int code) { return code_name(code); }

const char *ucov_last_error(const ucov_ctx *c) { return c ? c->last_error.c_str() : "no context"; }

}  // extern "C"

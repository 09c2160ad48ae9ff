// Scene stage of the camera covariance (steps a1-a3):
//   * observations grouped by point (counting sort on device),
//   * per-observation projection Jacobians (paper Sec. 5.1, projection),
//   * per-point 3x3 blocks V_j and their FP64 inverses (Sec. 5.2, A_p),
//   * camera-pair binning of the Schur-complement terms and their reduction
//     into Z = U - W V^-1 W^T (Sec. 5.2, Schur complement),
//   * the camera rows of the similarity nullspace with the rotation block
//     from J_r H_r = B (Sec. 5.1) and its Cholesky-QR2 orthonormalisation,
//   * Jacobi scaling of Z + a QQ^T (Sec. 5.2, conditioning).
#include <algorithm>

#include "camera_model.h"
#include "ucov_internal.h"
#include "../../include/ucov.h"

namespace ucov {

namespace {

constexpr int kBlk = 256;

typedef double d4 __attribute__((ext_vector_type(4)));

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

__device__ inline int64_t tri(int64_t i) { return i * (i + 1) / 2; }

// Lower-triangular camera-pair bin of cameras ci >= ck (of one scene).
__device__ inline int64_t bin_of(const SceneDev &sc, int ci, int ck) {
  if (!sc.cam_scene) return tri(ci) + ck;
  const int s = sc.cam_scene[ci];
  const int c0 = sc.cam_off[s];
  return sc.bin_off[s] + tri(ci - c0) + (ck - c0);
}

// ---------------------------------------------------------------------------
// fills and an exclusive scan of int32 counts into int64 offsets
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_f64(double *p, double v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ inline int64_t wave_incl_scan(int64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int64_t u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// Block-wide exclusive scan of the per-thread totals; returns the thread's
// exclusive prefix and writes the block total into *total.
__device__ inline int64_t block_excl_scan(int64_t v, int64_t *total) {
  __shared__ int64_t wsum[kScanThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int64_t inc = wave_incl_scan(v);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    int64_t w = lane < kScanThreads / 64 ? wsum[lane] : 0;
    int64_t wi = wave_incl_scan(w);
    if (lane < kScanThreads / 64) wsum[lane] = wi - w;
    if (lane == kScanThreads / 64 - 1) *total = wi;
  }
  __syncthreads();
  int64_t r = inc - v + wsum[wid];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const int32_t *in, int64_t *out,
                                                            int64_t len, int64_t *sums) {
  __shared__ int64_t total;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < len) ? (int64_t)in[base + k] : 0;
    s += v[k];
  }
  int64_t pre = block_excl_scan(s, &total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < len) out[base + k] = pre;
    pre += v[k];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// single block: exclusive scan of the tile sums, total at sums[ntiles]
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(int64_t *sums, int64_t ntiles) {
  __shared__ int64_t total;
  int64_t carry = 0;
  for (int64_t b = 0; b < ntiles; b += kScanThreads) {
    int64_t i = b + threadIdx.x;
    int64_t v = i < ntiles ? sums[i] : 0;
    int64_t pre = block_excl_scan(v, &total);
    if (i < ntiles) sums[i] = carry + pre;
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[ntiles] = carry;
}

__global__ void k_scan_add(int64_t *out, int64_t len, const int64_t *sums, int64_t ntiles) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) out[i] += sums[i / kScanTile];
  if (i == 0) out[len] = sums[ntiles];
}

// ---------------------------------------------------------------------------
// observations grouped by point
// ---------------------------------------------------------------------------
__global__ void k_count_points(SceneDev sc, int32_t *cnt_p, DevStatus *ds) {
  int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= sc.t) return;
  int c = sc.oc[o], j = sc.op[o];
  if (c < 0 || c >= sc.n || j < 0 || j >= sc.m) {
    report_error(ds, UCOV_EINVAL, (int)o);
    return;
  }
  atomicAdd(&cnt_p[j], 1);
}

// Each observation takes a slot of its point, with the sort key
// (camera << 32 | observation) of k_sort_points.
__global__ void k_fill_slots(SceneDev sc, const int64_t *ptr_p, int32_t *cur_p,
                             int64_t *slot_key) {
  int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= sc.t) return;
  int c = sc.oc[o], j = sc.op[o];
  if (c < 0 || c >= sc.n || j < 0 || j >= sc.m) return;
  int64_t pos = ptr_p[j] + atomicAdd(&cur_p[j], 1);
  slot_key[pos] = ((int64_t)c << 32) | (uint32_t)o;
}

// One thread per point: order its observations by camera, reject duplicate
// cameras and points with fewer than two observations.  Tracks of up to
// kSortCap observations are sorted as (camera, observation) keys in LDS
// (interleaved across the threads, read eight at a time); longer ones in
// place in global memory.
constexpr int kSortThreads = 128;
constexpr int kSortCap = 32;

__global__ __launch_bounds__(kSortThreads) void k_sort_points(SceneDev sc, const int64_t *ptr_p,
                                                              int64_t *slot_key, int32_t *slot_obs,
                                                              int32_t *slot_cam, int32_t *slot_pt,
                                                              DevStatus *ds) {
  __shared__ int64_t keys[kSortCap * kSortThreads];
  const int tid = threadIdx.x;
  int j = blockIdx.x * blockDim.x + tid;
  if (j >= sc.m) return;
  int64_t p0 = ptr_p[j], p1 = ptr_p[j + 1];
  const int64_t t = p1 - p0;
  if (t < 2) {
    report_error(ds, UCOV_EPOINT, j);
  }
  if (t <= kSortCap) {
    for (int a0 = 0; a0 < t; a0 += 8) {
      int64_t kk[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) kk[u] = a0 + u < t ? slot_key[p0 + a0 + u] : 0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (a0 + u < t) keys[(a0 + u) * kSortThreads + tid] = kk[u];
    }
    for (int a = 1; a < t; ++a) {
      const int64_t k = keys[a * kSortThreads + tid];
      int b = a - 1;
      while (b >= 0 && keys[b * kSortThreads + tid] > k) {
        keys[(b + 1) * kSortThreads + tid] = keys[b * kSortThreads + tid];
        --b;
      }
      keys[(b + 1) * kSortThreads + tid] = k;
    }
    int32_t prev = -1;
    for (int a = 0; a < t; ++a) {
      const int64_t k = keys[a * kSortThreads + tid];
      const int32_t c = (int32_t)(k >> 32), o = (int32_t)(k & 0xffffffff);
      if (c == prev) report_error(ds, UCOV_EINVAL, o);
      prev = c;
      slot_obs[p0 + a] = o;
      slot_cam[p0 + a] = c;
      slot_pt[p0 + a] = j;
    }
    return;
  }
  // insertion sort of a long segment's keys in place
  for (int64_t a = p0 + 1; a < p1; ++a) {
    const int64_t k = slot_key[a];
    int64_t b = a - 1;
    while (b >= p0 && slot_key[b] > k) {
      slot_key[b + 1] = slot_key[b];
      --b;
    }
    slot_key[b + 1] = k;
  }
  int32_t prev = -1;
  for (int64_t a = p0; a < p1; ++a) {
    const int64_t k = slot_key[a];
    const int32_t c = (int32_t)(k >> 32), o = (int32_t)(k & 0xffffffff);
    if (c == prev) report_error(ds, UCOV_EINVAL, o);
    prev = c;
    slot_obs[a] = o;
    slot_cam[a] = c;
    slot_pt[a] = j;
  }
}

// step a1: projection Jacobians -- projection_jacobian() in camera_model.h

// One thread per slot: Jacobians, whitened by the upper Cholesky factor L of
// the information block (L^T L = Sigma_u^-1), written into the slot record.
// Only the first ptr_p[m] slots are filled (observations with out-of-range
// indices are never placed), so every slot loop is bounded by that count.
// The workgroup's records pass through LDS so that the stores are coalesced
// (a record's 24 values are contiguous; one thread per record would store
// with a 256-byte stride across the lanes).  A slot with an error reports it
// and gets zeros (the call fails on the reported status).
constexpr int kJacPitch = 25;  // LDS doubles per staged record

__global__ __launch_bounds__(kBlk) void k_jacobians(SceneDev sc, const int64_t *ptr_p,
                                                    const int32_t *slot_obs,
                                                    const int32_t *slot_cam,
                                                    const int32_t *slot_pt, double *rec,
                                                    double *jp_out, double *jx_out, DevStatus *ds) {
  __shared__ double tile[kBlk * kJacPitch];
  const int64_t count = ptr_p[sc.m];
  const int64_t s0 = (int64_t)blockIdx.x * blockDim.x;
  const int64_t s = s0 + threadIdx.x;
  double val[24];
#pragma unroll
  for (int k = 0; k < 24; ++k) val[k] = 0.0;
  auto compute = [&]() {
    const int32_t o = slot_obs[s];
    const int i = slot_cam[s], j = slot_pt[s];
    double cam[9], X[3];
#pragma unroll
    for (int k = 0; k < 9; ++k) cam[k] = sc.cams[9 * (int64_t)i + k];
#pragma unroll
    for (int k = 0; k < 3; ++k) X[k] = sc.pts[3 * (int64_t)j + k];
    if (!finite9(cam, 9) || !finite9(X, 3)) {
      report_error(ds, UCOV_EINVAL, o);
      return;
    }
    double l00 = 1.0, l01 = 0.0, l11 = 1.0;
    if (sc.info) {
      const double ia = sc.info[3 * (int64_t)o], ib = sc.info[3 * (int64_t)o + 1],
                   ic = sc.info[3 * (int64_t)o + 2];
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
    if (jp_out) {
#pragma unroll
      for (int p = 0; p < 2; ++p) {
#pragma unroll
        for (int k = 0; k < 9; ++k) jp_out[18 * (int64_t)o + 9 * p + k] = J.jp[p][k];
#pragma unroll
        for (int k = 0; k < 3; ++k) jx_out[6 * (int64_t)o + 3 * p + k] = J.jx[p][k];
      }
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      val[kRecJP + k] = l00 * J.jp[0][k] + l01 * J.jp[1][k];
      val[kRecJP + 9 + k] = l11 * J.jp[1][k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      val[kRecJX + k] = l00 * J.jx[0][k] + l01 * J.jx[1][k];
      val[kRecJX + 3 + k] = l11 * J.jx[1][k];
    }
  };
  if (s < count) compute();
#pragma unroll
  for (int k = 0; k < 24; ++k) tile[threadIdx.x * kJacPitch + k] = val[k];
  __syncthreads();
  const int64_t nslots = min((int64_t)blockDim.x, count - s0);
  for (int64_t e = threadIdx.x; e < nslots * 24; e += blockDim.x) {
    const int64_t sl = e / 24, k = e % 24;
    rec[(s0 + sl) * kRec + k] = tile[sl * kJacPitch + k];
  }
}

// ---------------------------------------------------------------------------
// step a2 (points): V_j = sum J_X^T J_X, FP64 Cholesky inverse, Y = J_X V^-1
// ---------------------------------------------------------------------------
// A point block is rejected when its Cholesky factor does not exist or its
// smallest squared pivot is at most 1e-14 times its trace.
__global__ void k_point_blocks(SceneDev sc, const int64_t *ptr_p, double *rec, DevStatus *ds) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= sc.m) return;
  const int64_t p0 = ptr_p[j], p1 = ptr_p[j + 1];
  if (p1 - p0 < 2) return;
  double v00 = 0, v01 = 0, v02 = 0, v11 = 0, v12 = 0, v22 = 0;
  for (int64_t s = p0; s < p1; ++s) {
    const double *x = rec + s * kRec + kRecJX;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const double a = x[3 * p], b = x[3 * p + 1], c = x[3 * p + 2];
      v00 += a * a;
      v01 += a * b;
      v02 += a * c;
      v11 += b * b;
      v12 += b * c;
      v22 += c * c;
    }
  }
  const double tr = v00 + v11 + v22;
  const double thr = 1e-14 * tr;
  // V = L L^T
  const double d0 = v00;
  if (!(d0 > thr)) {
    report_error(ds, UCOV_EPOINT, j);
    return;
  }
  const double L00 = sqrt(d0);
  const double L10 = v01 / L00, L20 = v02 / L00;
  const double d1 = v11 - L10 * L10;
  if (!(d1 > thr)) {
    report_error(ds, UCOV_EPOINT, j);
    return;
  }
  const double L11 = sqrt(d1);
  const double L21 = (v12 - L20 * L10) / L11;
  const double d2 = v22 - L20 * L20 - L21 * L21;
  if (!(d2 > thr)) {
    report_error(ds, UCOV_EPOINT, j);
    return;
  }
  const double L22 = sqrt(d2);
  // M = L^-1 (lower)
  const double M00 = 1.0 / L00, M11 = 1.0 / L11, M22 = 1.0 / L22;
  const double M10 = -L10 * M00 * M11;
  const double M21 = -L21 * M11 * M22;
  const double M20 = -(L20 * M00 + L21 * M10) * M22;
  // V^-1 = M^T M
  const double w00 = M00 * M00 + M10 * M10 + M20 * M20;
  const double w01 = M10 * M11 + M20 * M21;
  const double w02 = M20 * M22;
  const double w11 = M11 * M11 + M21 * M21;
  const double w12 = M21 * M22;
  const double w22 = M22 * M22;
  for (int64_t s = p0; s < p1; ++s) {
    double *r = rec + s * kRec;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const double a = r[kRecJX + 3 * p], b = r[kRecJX + 3 * p + 1], c = r[kRecJX + 3 * p + 2];
      r[kRecY + 3 * p + 0] = a * w00 + b * w01 + c * w02;
      r[kRecY + 3 * p + 1] = a * w01 + b * w11 + c * w12;
      r[kRecY + 3 * p + 2] = a * w02 + b * w12 + c * w22;
    }
  }
}

// ---------------------------------------------------------------------------
// camera-pair bins: every ordered pair (a, b) of observations of one point
// with cam(a) >= cam(b) contributes to block Z(cam a, cam b)
// ---------------------------------------------------------------------------
// The first pair that lands in a bin also appends (i, k) to the list of
// non-empty bins.
__global__ void k_pair_count(SceneDev sc, const int64_t *ptr_p, const int32_t *slot_cam,
                             const int32_t *slot_pt, int32_t *bin_cnt) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= ptr_p[sc.m]) return;
  const int64_t p0 = ptr_p[slot_pt[a]];
  const int ci = slot_cam[a];
  for (int64_t b = p0; b <= a; ++b) atomicAdd(&bin_cnt[bin_of(sc, ci, slot_cam[b])], 1);
}

// Camera pair (i, k) of a bin (inverse of bin_of).
__device__ inline int2 bin_pair(const SceneDev &sc, int64_t bin) {
  int64_t local = bin;
  int base = 0;
  if (sc.cam_scene) {  // the scene: last s with bin_off[s] <= bin
    int lo = 0, hi = sc.n_scenes;
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      if (sc.bin_off[mid] <= bin) lo = mid;
      else hi = mid;
    }
    local = bin - sc.bin_off[lo];
    base = sc.cam_off[lo];
  }
  int64_t i = (int64_t)((sqrt(8.0 * (double)local + 1.0) - 1.0) * 0.5);
  while (tri(i + 1) <= local) ++i;
  while (tri(i) > local) --i;
  return make_int2(base + (int)i, base + (int)(local - tri(i)));
}

__global__ void k_nz_flag(int64_t nbins, const int32_t *bin_cnt, int32_t *flag) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nbins) flag[b] = bin_cnt[b] > 0 ? 1 : 0;
}

// The non-empty bins in bin order (camera i major within a scene), so that
// the waves of k_bin_blocks that run side by side share camera i's records.
__global__ void k_nz_compact(SceneDev sc, int64_t nbins, const int32_t *bin_cnt,
                             const int64_t *nzpos, int2 *nzlist, int64_t *nzcount) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b == 0) nzcount[0] = nzpos[nbins];
  if (b < nbins && bin_cnt[b] > 0) nzlist[nzpos[b]] = bin_pair(sc, b);
}

// Both fills write nothing when the pair count (*total) exceeds the capacity
// of the pair list or the overflow flag *skip is set (a replayed launch
// sequence whose scene grew: its bins were emptied and the error reported).
__global__ void k_pair_fill(SceneDev sc, const int64_t *ptr_p, const int32_t *slot_cam,
                            const int32_t *slot_pt, const int64_t *bin_ptr, int32_t *bin_cur,
                            int2 *pairs, const int64_t *total, int64_t cap, const int32_t *skip) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= ptr_p[sc.m] || *total > cap || (skip && *skip)) return;
  const int64_t p0 = ptr_p[slot_pt[a]];
  const int ci = slot_cam[a];
  for (int64_t b = p0; b <= a; ++b) {
    const int64_t bin = bin_of(sc, ci, slot_cam[b]);
    const int64_t pos = bin_ptr[bin] + atomicAdd(&bin_cur[bin], 1);
    pairs[pos] = make_int2((int)a, (int)b);
  }
}

// Camera-major construction of the same bins, for scenes of at most
// kCamHistMax cameras: the pairs (a, b), b <= a in a point, of the slots a of
// camera i all fall in bin row i, so one workgroup per camera counts them
// and then places them with LDS counters over the scene's cameras k <= i, and
// no global atomics are needed.  The slots of each camera come from a stable
// radix sort of the slots by camera (ascending slot order within a camera,
// below).
// (Grouping the slots with one global atomic per slot instead was measured
// slower: 500 cameras share ~300 000 increments.)
constexpr int kCamThreads = 256;

// ---------------------------------------------------------------------------
// Stable LSD radix sort of the slots by camera, 8 bits per pass: per block of
// kRadixItems keys a digit histogram, one exclusive scan over (digit, block),
// then a scatter in which every key's rank among the equal digits before it
// in its block comes from wave ballots (lanes with the same digit are found
// by matching the 8 digit bits) and per-wave running counts.  No atomics
// decide a position, so the order is the same on every call, and equal keys
// keep their input order (slots ascending within a camera).
// ---------------------------------------------------------------------------
constexpr int kRadixThreads = 256;
constexpr int kRadixSteps = 16;  // 64-key steps per wave
constexpr int kRadixItems = kRadixThreads * kRadixSteps;
constexpr int kRadixPerWave = 64 * kRadixSteps;

// Only the first *count of the t slots hold observations (the rest belong to
// rejected input), so every kernel of the sort stops there (count null: all
// t keys).
__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(int64_t t_max, const int64_t *count,
                                                            const int32_t *keys, int shift,
                                                            int64_t nblocks, int32_t *hist) {
  __shared__ int32_t cnt[256];
  const int64_t t = count ? min(t_max, *count) : t_max;
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixItems;
  for (int k = threadIdx.x; k < kRadixItems; k += kRadixThreads) {
    const int64_t e = base + k;
    if (e < t) atomicAdd(&cnt[((uint32_t)keys[e] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// vals_in null: the value of a key is its input position.
__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(
    int64_t t_max, const int64_t *count, const int32_t *keys_in, const int32_t *vals_in,
    int shift, int64_t nblocks, const int64_t *offs, int32_t *keys_out, int32_t *vals_out) {
  __shared__ int32_t wcnt[kRadixThreads / 64][256];
  __shared__ int32_t wpre[kRadixThreads / 64][256];
  const int64_t t = count ? min(t_max, *count) : t_max;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int d = threadIdx.x; d < 256 * (kRadixThreads / 64); d += kRadixThreads) wcnt[d >> 8][d & 255] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixItems + (int64_t)w * kRadixPerWave;
  const uint64_t below = (1ull << lane) - 1ull;
  int32_t key[kRadixSteps], rank[kRadixSteps];
#pragma unroll
  for (int st = 0; st < kRadixSteps; ++st) {
    const int64_t e = base + st * 64 + lane;
    const bool valid = e < t;
    const int32_t k = valid ? keys_in[e] : 0;
    const unsigned d = ((uint32_t)k >> shift) & 255u;
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t ones = __ballot(valid && ((d >> b) & 1u));
      same &= ((d >> b) & 1u) ? ones : ~ones;
    }
    int32_t before = 0;
    if (valid) before = wcnt[w][d];
    // all lanes have read before the lowest lane of each digit group writes
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (valid && (same & below) == 0) wcnt[w][d] = before + (int32_t)__popcll(same);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    key[st] = k;
    rank[st] = before + (int32_t)__popcll(same & below);
  }
  __syncthreads();
  {
    const int d = threadIdx.x;  // 256 threads, one per digit
    int32_t run = 0;
#pragma unroll
    for (int v = 0; v < kRadixThreads / 64; ++v) {
      wpre[v][d] = run;
      run += wcnt[v][d];
    }
  }
  __syncthreads();
#pragma unroll
  for (int st = 0; st < kRadixSteps; ++st) {
    const int64_t e = base + st * 64 + lane;
    if (e >= t) continue;
    const unsigned d = ((uint32_t)key[st] >> shift) & 255u;
    const int64_t dest = offs[(int64_t)d * nblocks + blockIdx.x] + wpre[w][d] + rank[st];
    keys_out[dest] = key[st];
    vals_out[dest] = vals_in ? vals_in[e] : (int32_t)e;
  }
}

// cam_ptr[c] = first position of camera c in the sorted camera keys, c <= n.
__global__ void k_cam_bounds(int n, int64_t t_max, const int64_t *count, const int32_t *cam_sorted,
                             int64_t *cam_ptr) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c > n) return;
  int64_t lo = 0, hi = min(t_max, *count);
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (cam_sorted[mid] < c) lo = mid + 1;
    else hi = mid;
  }
  cam_ptr[c] = lo;
}

// Bin row i: bin_cnt[bin(i, k)] for every camera k <= i of the scene.
__global__ __launch_bounds__(kCamThreads) void k_pair_count_cam(
    SceneDev sc, const int64_t *cam_ptr, const int32_t *cam_slots, const int64_t *ptr_p,
    const int32_t *slot_cam, const int32_t *slot_pt, int32_t *bin_cnt) {
  extern __shared__ int32_t hist[];
  const int i = blockIdx.x;
  const int c0 = sc.cam_scene ? sc.cam_off[sc.cam_scene[i]] : 0;
  const int nk = i - c0 + 1;
  for (int k = threadIdx.x; k < nk; k += blockDim.x) hist[k] = 0;
  __syncthreads();
  // the cameras of a point ascend along its slots and share its scene, so
  // slot_cam[b] - c0 lies in [0, nk) for b <= a
  for (int64_t e = cam_ptr[i] + threadIdx.x; e < cam_ptr[i + 1]; e += blockDim.x) {
    const int a = cam_slots[e];
    for (int64_t b = ptr_p[slot_pt[a]]; b <= a; ++b) atomicAdd(&hist[slot_cam[b] - c0], 1);
  }
  __syncthreads();
  const int64_t row = bin_of(sc, i, c0);
  for (int k = threadIdx.x; k < nk; k += blockDim.x) bin_cnt[row + k] = hist[k];
}

// One wave per camera: every LDS cursor increment of the row then comes from
// one wave, whose atomic instructions the LDS resolves in a fixed lane order,
// so the pairs of a bin are placed in the same order on every call and the
// bin sums that follow are bitwise reproducible.
constexpr int kFillThreads = 64;

__global__ __launch_bounds__(kFillThreads) void k_pair_fill_cam(
    SceneDev sc, const int64_t *cam_ptr, const int32_t *cam_slots, const int64_t *ptr_p,
    const int32_t *slot_cam, const int32_t *slot_pt, const int64_t *bin_ptr, int2 *pairs,
    const int64_t *total, int64_t cap, const int32_t *skip) {
  extern __shared__ int32_t cur[];  // next position of each bin, from the row's start
  if (*total > cap || (skip && *skip)) return;
  const int i = blockIdx.x;
  const int c0 = sc.cam_scene ? sc.cam_off[sc.cam_scene[i]] : 0;
  const int nk = i - c0 + 1;
  const int64_t row = bin_of(sc, i, c0);
  const int64_t base = bin_ptr[row];  // int32 offsets: the host launches this below 2^31 pairs
  for (int k = threadIdx.x; k < nk; k += blockDim.x) cur[k] = (int32_t)(bin_ptr[row + k] - base);
  __syncthreads();
  for (int64_t e = cam_ptr[i] + threadIdx.x; e < cam_ptr[i + 1]; e += blockDim.x) {
    const int a = cam_slots[e];
    for (int64_t b = ptr_p[slot_pt[a]]; b <= a; ++b) {
      const int k = slot_cam[b] - c0;
      pairs[base + atomicAdd(&cur[k], 1)] = make_int2(a, (int)b);
    }
  }
}

// ---------------------------------------------------------------------------
// per camera: diagonal block Z_ii and the rotation rows of the nullspace
// ---------------------------------------------------------------------------
constexpr int kDiagVals = 45 + 6 + 9;  // Z_ii upper triangle, J_r^T J_r, J_r^T B
constexpr int kDiagWaves = 2;           // waves per camera in k_camera_diag

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Sums over the 64 lanes of a wave of 64 values per lane, lane l ending
// with the sum of value l: at distance d = 32, 16, .., 1 every lane keeps the
// half of its remaining values that bit d of its lane index selects and
// adds its partner's copy of that half (63 exchanges instead of 6 per value).
template <int V>
__device__ inline void wave_sums_halving(double (&x)[64], int lane) {
  if constexpr (V > 1) {
    constexpr int H = V / 2;
    const bool up = lane & H;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const double keep = up ? x[H + i] : x[i], send = up ? x[i] : x[H + i];
      x[i] = keep + __shfl_xor(send, H, 64);
    }
    wave_sums_halving<H>(x, lane);
  }
}

// Z_ii = sum over the observations a of camera i of J_P^T (I - Y J_X^T) J_P
// (whitened), i.e. U_i minus the point-eliminated terms.  The rotation
// nullspace block solves J_r H_r = B in least squares over the camera's
// observation rows, B = -J_X [X_j - C_i]x (the known rows of H in the rotation
// columns are [C_i]x for the centre and [X_j]x for the points, and J_C = -J_X).
template <int W>
__global__ __launch_bounds__(64 * W) void k_camera_diag(SceneDev sc, const int64_t *bin_ptr,
                                                       const int2 *pairs, const double *rec,
                                                       const int32_t *slot_pt, double *zdiag,
                                                       double *hc, DevStatus *ds) {
  const int i = blockIdx.x;
  const int64_t bin = bin_of(sc, i, i);
  const int64_t e0 = bin_ptr[bin], e1 = bin_ptr[bin + 1];
  double acc[64];  // kDiagVals sums, padded for the halving exchange
#pragma unroll
  for (int k = 0; k < 64; ++k) acc[k] = 0.0;
  const double C0 = sc.cams[9 * (int64_t)i + 3], C1 = sc.cams[9 * (int64_t)i + 4],
               C2 = sc.cams[9 * (int64_t)i + 5];
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 64 * W) {
    const int a = pairs[e].x;
    // the record's first 30 values (J_P, J_X, Y) with 16-byte loads
    const double2 *r2 = reinterpret_cast<const double2 *>(rec + (int64_t)a * kRec);
    double rv[30];
#pragma unroll
    for (int h = 0; h < 15; ++h) {
      const double2 t = r2[h];
      rv[2 * h] = t.x;
      rv[2 * h + 1] = t.y;
    }
    double jp[2][9], jx[2][3], y[2][3];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
#pragma unroll
      for (int k = 0; k < 9; ++k) jp[p][k] = rv[kRecJP + 9 * p + k];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        jx[p][k] = rv[kRecJX + 3 * p + k];
        y[p][k] = rv[kRecY + 3 * p + k];
      }
    }
    // M = I - Y J_X^T (2x2, symmetric)
    double M[2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q)
        M[p][q] = (p == q ? 1.0 : 0.0) - (y[p][0] * jx[q][0] + y[p][1] * jx[q][1] + y[p][2] * jx[q][2]);
    double T[2][9];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int k = 0; k < 9; ++k) T[p][k] = M[p][0] * jp[0][k] + M[p][1] * jp[1][k];
    int idx = 0;
#pragma unroll
    for (int rr = 0; rr < 9; ++rr)
#pragma unroll
      for (int cc = rr; cc < 9; ++cc) acc[idx++] += jp[0][rr] * T[0][cc] + jp[1][rr] * T[1][cc];
    // rotation nullspace normal equations
    const int j = slot_pt[a];
    const double v0 = sc.pts[3 * (int64_t)j] - C0, v1 = sc.pts[3 * (int64_t)j + 1] - C1,
                 v2 = sc.pts[3 * (int64_t)j + 2] - C2;
    double B[2][3];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      // -(jx [v]x): row p of jx times [v]x, negated
      B[p][0] = -(jx[p][1] * v2 - jx[p][2] * v1);
      B[p][1] = -(jx[p][2] * v0 - jx[p][0] * v2);
      B[p][2] = -(jx[p][0] * v1 - jx[p][1] * v0);
    }
#pragma unroll
    for (int rr = 0; rr < 3; ++rr)
#pragma unroll
      for (int cc = rr; cc < 3; ++cc) acc[idx++] += jp[0][rr] * jp[0][cc] + jp[1][rr] * jp[1][cc];
#pragma unroll
    for (int rr = 0; rr < 3; ++rr)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) acc[idx++] += jp[0][rr] * B[0][cc] + jp[1][rr] * B[1][cc];
  }
  __shared__ double part[W][64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  wave_sums_halving<64>(acc, lane);
  part[wid][lane] = acc[0];  // this wave's sum of value `lane`
  __syncthreads();
  __shared__ double tot[kDiagVals];
  if (threadIdx.x < kDiagVals) {
    const int k = threadIdx.x;
    double v = part[0][k];
#pragma unroll
    for (int w = 1; w < W; ++w) v += part[w][k];
    tot[k] = v;
  }
  __syncthreads();
  // diagonal block, full 9x9 row-major
  for (int u = threadIdx.x; u < 81; u += 64 * W) {
    const int rr = u / 9, cc = u % 9;
    const int a = rr < cc ? rr : cc, b = rr < cc ? cc : rr;
    const int idx = a * 9 - a * (a - 1) / 2 + (b - a);
    zdiag[81 * (int64_t)i + u] = tot[idx];
  }
  if (threadIdx.x == 0) {
    if (e1 == e0) report_error(ds, UCOV_EGAUGE, i);
    const double *N = tot + 45;  // 00 01 02 11 12 22
    const double *R = tot + 51;  // row-major 3x3
    const double n00 = N[0], n01 = N[1], n02 = N[2], n11 = N[3], n12 = N[4], n22 = N[5];
    // Cholesky of the 3x3 normal matrix, pivots checked against its trace
    const double thr = 1e-14 * (n00 + n11 + n22);
    double L00 = 0, L10 = 0, L20 = 0, L11 = 0, L21 = 0, L22 = 0;
    bool ok = n00 > thr;
    if (ok) {
      L00 = sqrt(n00);
      L10 = n01 / L00;
      L20 = n02 / L00;
      const double d1 = n11 - L10 * L10;
      ok = d1 > thr;
      if (ok) {
        L11 = sqrt(d1);
        L21 = (n12 - L20 * L10) / L11;
        const double d2 = n22 - L20 * L20 - L21 * L21;
        ok = d2 > thr;
        if (ok) L22 = sqrt(d2);
      }
    }
    if (!ok) report_error(ds, UCOV_EGAUGE, i);
    const int64_t Nn = 9 * (int64_t)sc.n;
    const int64_t row0 = 9 * (int64_t)i;
    for (int cc = 0; cc < 3; ++cc) {
      // solve L L^T h = R[:, cc]
      double h0 = 0, h1 = 0, h2 = 0;
      if (ok) {
        const double y0 = R[0 * 3 + cc] / L00;
        const double y1 = (R[1 * 3 + cc] - L10 * y0) / L11;
        const double y2 = (R[2 * 3 + cc] - L20 * y0 - L21 * y1) / L22;
        h2 = y2 / L22;
        h1 = (y1 - L21 * h2) / L11;
        h0 = (y0 - L10 * h1 - L20 * h2) / L00;
      }
      hc[(3 + cc) * Nn + row0 + 0] = h0;
      hc[(3 + cc) * Nn + row0 + 1] = h1;
      hc[(3 + cc) * Nn + row0 + 2] = h2;
    }
    // rotation rows, translation and scale columns: zero
    for (int rr = 0; rr < 3; ++rr) {
      for (int cc = 0; cc < 3; ++cc) hc[cc * Nn + row0 + rr] = 0.0;
      hc[6 * Nn + row0 + rr] = 0.0;
    }
    // centre rows: [I | [C]x | C]
    const double Cv[3] = {C0, C1, C2};
    const double Cx[3][3] = {{0, -C2, C1}, {C2, 0, -C0}, {-C1, C0, 0}};
    for (int rr = 0; rr < 3; ++rr) {
      for (int cc = 0; cc < 3; ++cc) {
        hc[cc * Nn + row0 + 3 + rr] = rr == cc ? 1.0 : 0.0;
        hc[(3 + cc) * Nn + row0 + 3 + rr] = Cx[rr][cc];
      }
      hc[6 * Nn + row0 + 3 + rr] = Cv[rr];
    }
    // intrinsics rows: zero
    for (int rr = 6; rr < 9; ++rr)
      for (int cc = 0; cc < 7; ++cc) hc[cc * Nn + row0 + rr] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// step a3: Cholesky-QR2 orthonormalisation, gauge weight, Jacobi scaling
// ---------------------------------------------------------------------------
constexpr int kGaugeThreads = 512;

// Lane l's value of x on every lane (scalar lane reads).
__device__ inline double lane_bcast(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double block_sum(double v, double *red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < kGaugeThreads / 64; ++k) s += red[k];
  return s;
}

// Gram matrix G = A^T A of an N x 7 column-major matrix, then R = chol(G)
// (G = R^T R) and A <- A R^-1, written into out.  Returns false if G is not
// positive definite.
__device__ __forceinline__ bool cholqr_pass(int64_t N, int64_t ld, const double *A, double *out, double *red,
                            double *Gs, double *Ri) {
  double g[28];
#pragma unroll
  for (int k = 0; k < 28; ++k) g[k] = 0.0;
  for (int64_t p = threadIdx.x; p < N; p += kGaugeThreads) {
    double row[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) row[c] = A[c * ld + p];
    int idx = 0;
#pragma unroll
    for (int a = 0; a < 7; ++a)
#pragma unroll
      for (int b = a; b < 7; ++b) g[idx++] += row[a] * row[b];
  }
  // one reduction pass for all 28 sums: wave sums, then across the waves
  __shared__ double part[kGaugeThreads / 64][28];
  {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 28; ++k) {
      const double v = wave_sum(g[k]);
      if (lane == 0) part[wid][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 28) {
      double v = 0.0;
      for (int w = 0; w < kGaugeThreads / 64; ++w) v += part[w][threadIdx.x];
      Gs[threadIdx.x] = v;
    }
    __syncthreads();
  }
  __shared__ int okflag;
  // the 7 x 7 factorisation and its inverse on wave 0, in registers: lane
  // r < 7 holds row r (of G, then L, then L^-1), columns broadcast by lane
  // reads; R = L^T, Ri = R^-1 = (L^-1)^T
  if (threadIdx.x < 64) {
    const int r = threadIdx.x;
    double l[7], y[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      const int lo = r < c ? r : c, hi = r < c ? c : r;  // upper-packed (lo, hi)
      l[c] = r < 7 ? Gs[lo * 7 - lo * (lo - 1) / 2 + (hi - lo)] : 0.0;
      y[c] = r == c ? 1.0 : 0.0;
    }
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      const double piv = lane_bcast(l[j], j);
      ok = ok && piv > 0.0;
      const double d = sqrt(piv);
      const double w = r == j ? d : l[j] / d;  // L[r][j] for r >= j
#pragma unroll
      for (int c = j + 1; c < 7; ++c) l[c] -= w * lane_bcast(w, c);
      l[j] = r >= j ? w : 0.0;
    }
    // forward elimination with M = L diag(L)^-1: row r > j loses M[r][j]
    // times row j; row r of L^-1 is then row r over L[r][r]
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const double f = r > j ? l[j] / lane_bcast(l[j], j) : 0.0;
#pragma unroll
      for (int c = 0; c < j; ++c) y[c] -= f * lane_bcast(y[c], j);
      y[j] -= f;
    }
    double lrr = 1.0;
#pragma unroll
    for (int k = 0; k < 7; ++k) lrr = r == k ? l[k] : lrr;
    if (r < 7) {
#pragma unroll
      for (int c = 0; c < 7; ++c) Ri[c * 7 + r] = ok ? y[c] / lrr : 0.0;
    }
    if (r == 0) okflag = ok ? 1 : 0;
  }
  __syncthreads();
  if (!okflag) return false;
  for (int64_t p = threadIdx.x; p < N; p += kGaugeThreads) {
    double row[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) row[c] = A[c * ld + p];
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < 7; ++k) v += row[k] * Ri[k * 7 + c];
      out[c * ld + p] = v;
    }
  }
  __syncthreads();
  return true;
}

// One workgroup per scene.  Scene s owns the rows [row0, row0 + N) of the
// N_total x 7 matrices hc and q (leading dimension ld); diag(Z) of its rows
// comes from the per-camera blocks zdiag (camera = row / 9) or, when that is
// null, from the dense zdense (single scene).
__device__ void gauge_scene(int64_t row0, int64_t N, int64_t ld, const double *hc, double *q,
                            const double *zdiag, const double *zdense, int64_t ldz,
                            double user_alpha, double *s, double *alpha_out, DevStatus *ds,
                            double *red, double *Gs, double *Ri) {
  if (hc) {
    if (!cholqr_pass(N, ld, hc + row0, q + row0, red, Gs, Ri) ||
        !cholqr_pass(N, ld, q + row0, q + row0, red, Gs, Ri)) {
      if (threadIdx.x == 0) report_error(ds, UCOV_EGAUGE, (int)(row0 / 9));
      return;
    }
  }
  // a = 7 / sum_p sum_k Q_pk^2 / Z_pp unless given
  double part = 0.0;
  for (int64_t pl = threadIdx.x; pl < N; pl += kGaugeThreads) {
    const int64_t p = row0 + pl;
    const double zpp = zdiag ? zdiag[81 * (p / 9) + 10 * (p % 9)] : zdense[pl * ldz + pl];
    double qq = 0.0;
#pragma unroll
    for (int c = 0; c < 7; ++c) qq += q[c * ld + p] * q[c * ld + p];
    part += qq / zpp;
  }
  const double tot = block_sum(part, red);
  const double a = user_alpha > 0.0 ? user_alpha : 7.0 / tot;
  if (threadIdx.x == 0) *alpha_out = a;
  for (int64_t pl = threadIdx.x; pl < N; pl += kGaugeThreads) {
    const int64_t p = row0 + pl;
    const double zpp = zdiag ? zdiag[81 * (p / 9) + 10 * (p % 9)] : zdense[pl * ldz + pl];
    double qq = 0.0;
#pragma unroll
    for (int c = 0; c < 7; ++c) qq += q[c * ld + p] * q[c * ld + p];
    const double dA = zpp + a * qq;
    if (!(dA > 0.0) || !isfinite(dA)) {
      report_error(ds, UCOV_EGAUGE, (int)(p / 9));
      s[p] = 0.0;
    } else {
      s[p] = 1.0 / sqrt(dA);
    }
  }
}

__global__ __launch_bounds__(kGaugeThreads) void k_gauge(int64_t N, const double *hc,
                                                        double *q, const double *zdiag,
                                                        const double *zdense, int64_t ldz,
                                                        double user_alpha, double *s,
                                                        double *alpha_out, DevStatus *ds) {
  __shared__ double red[kGaugeThreads / 64];
  __shared__ double Gs[28];
  __shared__ double Ri[49];
  gauge_scene(0, N, N, hc, q, zdiag, zdense, ldz, user_alpha, s, alpha_out, ds, red, Gs, Ri);
}

__global__ __launch_bounds__(kGaugeThreads) void k_gauge_scenes(SceneDev sc, const double *hc,
                                                               double *q, const double *zdiag,
                                                               double user_alpha, double *s,
                                                               double *alpha, DevStatus *ds) {
  __shared__ double red[kGaugeThreads / 64];
  __shared__ double Gs[28];
  __shared__ double Ri[49];
  const int si = blockIdx.x;
  const int64_t row0 = 9 * (int64_t)sc.cam_off[si];
  const int64_t N = 9 * (int64_t)(sc.cam_off[si + 1] - sc.cam_off[si]);
  gauge_scene(row0, N, 9 * (int64_t)sc.n, hc, q, zdiag, nullptr, 0, user_alpha, s, alpha + si,
              ds, red, Gs, Ri);
}

// ---------------------------------------------------------------------------
// The paper's gauge: (M^+)_cc = (Z + G F^-1 G^T)^-1 with G = H_c - W V^-1 H_p
// and F = H_p^T V^-1 H_p, H_p the point rows [I, [X_j]x, X_j] of the
// similarity nullspace (Sec. 4, Sec. 5.2: the points eliminated with the full
// nullspace; the term vanishes from the inverse as the constraint weight
// grows).  Written as P P^T with P = G L_F^-T, it takes the place of a Q Q^T.
// ---------------------------------------------------------------------------

// F_j = H_p^T V_j^-1 H_p per point (V_j from the point's whitened J_X rows),
// 28 upper-triangle values summed per workgroup into fpart (28 per
// workgroup); k_paper_fsum adds the workgroups' sums in a fixed order.
__global__ __launch_bounds__(256) void k_paper_f(SceneDev sc, const int64_t *ptr_p,
                                                const double *rec, double *fpart) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  double acc[28];
#pragma unroll
  for (int k = 0; k < 28; ++k) acc[k] = 0.0;
  if (j < sc.m && ptr_p[j + 1] - ptr_p[j] >= 2) {
    double v00 = 0, v01 = 0, v02 = 0, v11 = 0, v12 = 0, v22 = 0;
    for (int64_t a = ptr_p[j]; a < ptr_p[j + 1]; ++a) {
      const double *x = rec + a * kRec + kRecJX;
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const double u = x[3 * p], v = x[3 * p + 1], w = x[3 * p + 2];
        v00 += u * u; v01 += u * v; v02 += u * w;
        v11 += v * v; v12 += v * w; v22 += w * w;
      }
    }
    // V = L L^T (its pivots were checked by the point blocks), M = L^-1
    const double L00 = sqrt(v00), L10 = v01 / L00, L20 = v02 / L00;
    const double L11 = sqrt(v11 - L10 * L10), L21 = (v12 - L20 * L10) / L11;
    const double L22 = sqrt(v22 - L20 * L20 - L21 * L21);
    const double M00 = 1.0 / L00, M11 = 1.0 / L11, M22 = 1.0 / L22;
    const double M10 = -L10 * M00 * M11, M21 = -L21 * M11 * M22;
    const double M20 = -(L20 * M00 + L21 * M10) * M22;
    const double X0 = sc.pts[3 * (int64_t)j], X1 = sc.pts[3 * (int64_t)j + 1],
                 X2 = sc.pts[3 * (int64_t)j + 2];
    // H_p rows: [I, [X]x, X]
    const double H[3][7] = {{1, 0, 0, 0, -X2, X1, X0},
                            {0, 1, 0, X2, 0, -X0, X1},
                            {0, 0, 1, -X1, X0, 0, X2}};
    const double M[3][3] = {{M00, 0, 0}, {M10, M11, 0}, {M20, M21, M22}};
    double R[3][7];  // M H_p, so F_j = R^T R
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 7; ++c) R[r][c] = M[r][0] * H[0][c] + M[r][1] * H[1][c] + M[r][2] * H[2][c];
    int k = 0;
#pragma unroll
    for (int a = 0; a < 7; ++a)
#pragma unroll
      for (int b = a; b < 7; ++b) acc[k++] = R[0][a] * R[0][b] + R[1][a] * R[1][b] + R[2][a] * R[2][b];
  }
  __shared__ double part[4][28];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 28; ++k) {
    const double v = wave_sum(acc[k]);
    if (lane == 0) part[wid][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 28) {
    const int k = threadIdx.x;
    fpart[28 * (int64_t)blockIdx.x + k] = part[0][k] + part[1][k] + part[2][k] + part[3][k];
  }
}

// f[k] = sum over the nb workgroup sums of k_paper_f, in a fixed order (each
// thread a fixed stride of workgroups, then a fixed tree): the same bits on
// every call.
constexpr int kFsumThreads = 256;

__global__ __launch_bounds__(kFsumThreads) void k_paper_fsum(int64_t nb, const double *fpart,
                                                           double *f) {
  __shared__ double red[kFsumThreads];
  for (int k = 0; k < 28; ++k) {
    double v = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += kFsumThreads) v += fpart[28 * b + k];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int h = kFsumThreads / 2; h > 0; h >>= 1) {
      if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) f[k] = red[0];
    __syncthreads();
  }
}

// G_i = H_c,i - sum over camera i's observations of J_P^T (Y H_p,j) (Y =
// J_X V^-1 from the slot record), one workgroup per camera over the slots of
// its diagonal camera-pair bin; written to q (N x 7, leading dimension N).
__global__ __launch_bounds__(256) void k_paper_g(SceneDev sc, const int64_t *bin_ptr,
                                                const int2 *pairs, const double *rec,
                                                const int32_t *slot_pt, const double *hc,
                                                double *q) {
  const int i = blockIdx.x;
  const int64_t bin = bin_of(sc, i, i);
  const int64_t N = 9 * (int64_t)sc.n;
  double acc[63];
#pragma unroll
  for (int k = 0; k < 63; ++k) acc[k] = 0.0;
  for (int64_t e = bin_ptr[bin] + threadIdx.x; e < bin_ptr[bin + 1]; e += blockDim.x) {
    const int a = pairs[e].x;
    const double *r = rec + (int64_t)a * kRec;
    const int j = slot_pt[a];
    const double X0 = sc.pts[3 * (int64_t)j], X1 = sc.pts[3 * (int64_t)j + 1],
                 X2 = sc.pts[3 * (int64_t)j + 2];
    double yh[2][7];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const double y0 = r[kRecY + 3 * p], y1 = r[kRecY + 3 * p + 1], y2 = r[kRecY + 3 * p + 2];
      yh[p][0] = y0;
      yh[p][1] = y1;
      yh[p][2] = y2;
      yh[p][3] = y1 * X2 - y2 * X1;  // y [X]x
      yh[p][4] = -y0 * X2 + y2 * X0;
      yh[p][5] = y0 * X1 - y1 * X0;
      yh[p][6] = y0 * X0 + y1 * X1 + y2 * X2;
    }
#pragma unroll
    for (int rr = 0; rr < 9; ++rr) {
      const double p0 = r[kRecJP + rr], p1 = r[kRecJP + 9 + rr];
#pragma unroll
      for (int c = 0; c < 7; ++c) acc[7 * rr + c] += p0 * yh[0][c] + p1 * yh[1][c];
    }
  }
  __shared__ double part[4][63];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 63; ++k) {
    const double v = wave_sum(acc[k]);
    if (lane == 0) part[wid][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 63) {
    const int rr = threadIdx.x / 7, c = threadIdx.x % 7;
    const int64_t row = 9 * (int64_t)i + rr;
    const double g = part[0][threadIdx.x] + part[1][threadIdx.x] + part[2][threadIdx.x] +
                     part[3][threadIdx.x];
    q[c * N + row] = hc[c * N + row] - g;
  }
}

// F = L_F L_F^T (one thread; L_F stored row-major after F's 28 values),
// then every row of q replaced by L_F^-1 applied to it (P = G L_F^-T); the
// gauge weight is 1.
__global__ __launch_bounds__(1024) void k_paper_p(int64_t N, double *f, double *q,
                                                 double *alpha, DevStatus *ds) {
  __shared__ double L[7][7];
  __shared__ int ok;
  if (threadIdx.x == 0) {
    double F[7][7];
    int k = 0;
    for (int a = 0; a < 7; ++a)
      for (int b = a; b < 7; ++b, ++k) F[a][b] = F[b][a] = f[k];
    double tr = 0.0;
    for (int a = 0; a < 7; ++a) tr += F[a][a];
    ok = 1;
    for (int a = 0; a < 7; ++a) {
      for (int b = 0; b <= a; ++b) {
        double s = F[a][b];
        for (int c = 0; c < b; ++c) s -= L[a][c] * L[b][c];
        if (a == b) {
          if (!(s > 1e-14 * tr)) {
            ok = 0;
            s = 1.0;
          }
          L[a][a] = sqrt(s);
        } else {
          L[a][b] = s / L[b][b];
        }
      }
      for (int b = a + 1; b < 7; ++b) L[a][b] = 0.0;
    }
    if (!ok) report_error(ds, UCOV_EGAUGE, -1);
    for (int a = 0; a < 7; ++a)
      for (int b = 0; b < 7; ++b) f[28 + 7 * a + b] = L[a][b];
    alpha[0] = 1.0;
  }
  __syncthreads();
  if (!ok) return;
  for (int64_t p = threadIdx.x; p < N; p += blockDim.x) {
    double x[7];
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      double s = q[a * N + p];
#pragma unroll
      for (int c = 0; c < a; ++c) s -= L[a][c] * x[c];
      x[a] = s / L[a][a];
    }
#pragma unroll
    for (int a = 0; a < 7; ++a) q[a * N + p] = x[a];
  }
}

// ---------------------------------------------------------------------------
// assembly of Z (mode 0) or S (Z + a QQ^T) S (mode 1)
//
// k_fill_empty writes the camera blocks without Schur terms (Z_ik = 0): zeros
// in mode 0, the scaled gauge term in mode 1; one thread per row of a camera's
// 9 columns, with coalesced column stores.  k_bin_blocks takes one wave per non-empty
// bin (i, k) and writes that whole 9x9 block.
// ---------------------------------------------------------------------------
// One workgroup per camera k (its 9 columns) and chunk of kFillRows rows of
// the column's scene: each thread takes one row r, loads its 7 Q values,
// scale and bin test once and writes its entries r >= c in the 9 columns
// (column stores coalesced across the threads).  The scene gives the matrix
// (offset a_off[s], leading dimension a_ld[s]) and the row range.
constexpr int kFillRows = 1024;

__global__ __launch_bounds__(256) void k_fill_empty(SceneDev sc, const int32_t *bin_cnt,
                                                   const double *q, const double *s,
                                                   const double *alpha, int mode, double *out,
                                                   int64_t ld) {
  const int64_t N = 9 * (int64_t)sc.n;  // rows of q (all scenes)
  const int kc = blockIdx.x;
  const int64_t gc0 = 9 * (int64_t)kc;
  int si = 0;
  int64_t row0 = 0, Ns = N, off = 0, lds = ld;
  if (sc.cam_scene) {
    si = sc.cam_scene[kc];
    row0 = 9 * (int64_t)sc.cam_off[si];
    Ns = 9 * (int64_t)(sc.cam_off[si + 1] - sc.cam_off[si]);
    off = sc.a_off[si];
    lds = sc.a_ld[si];
  }
  const int64_t c0 = gc0 - row0;  // first column in the scene
  const int64_t r_begin = c0 + (int64_t)blockIdx.y * kFillRows;
  if (r_begin >= Ns) return;
  const int64_t r_end = min(Ns, r_begin + kFillRows);
  __shared__ double qcs[9][7], scs[9];
  const int tid = threadIdx.x;
  if (tid < 63) qcs[tid / 7][tid % 7] = mode ? q[(tid % 7) * N + gc0 + tid / 7] : 0.0;
  if (tid < 9) scs[tid] = mode ? s[gc0 + tid] : 0.0;
  __syncthreads();
  const double a = mode ? alpha[si] : 0.0;
  double *o = out + off;
  for (int64_t r = r_begin + tid; r < r_end; r += blockDim.x) {
    const int64_t gr = row0 + r;
    if (bin_cnt[bin_of(sc, (int)(gr / 9), kc)] != 0) continue;
    const int jmax = (int)min((int64_t)8, r - c0);  // columns c0 + j <= r
    if (mode == 0) {
      for (int j = 0; j <= jmax; ++j) {
        o[r + (c0 + j) * lds] = 0.0;
        o[(c0 + j) + r * lds] = 0.0;
      }
      continue;
    }
    double qr[7];
#pragma unroll
    for (int h = 0; h < 7; ++h) qr[h] = q[h * N + gr];
    const double sr = s[gr];
    for (int j = 0; j <= jmax; ++j) {
      double g = 0.0;
#pragma unroll
      for (int h = 0; h < 7; ++h) g += qr[h] * qcs[j][h];
      o[r + (c0 + j) * lds] = sr * (a * g) * scs[j];
    }
  }
}

__global__ __launch_bounds__(256) void k_concat(const BatchEntry *tab, double *cams, double *pts,
                                               double *info, int32_t *oc, int32_t *op,
                                               int32_t *cam_scene, DevStatus *ds) {
  const BatchEntry e = tab[blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = i0; i < e.t; i += stride) {
    int c = e.oc[i], p = e.op[i];
    if (c < 0 || c >= e.n || p < 0 || p >= e.m) {
      report_error(ds, UCOV_EINVAL, (int)(e.obs0 + i));
      c = 0;
      p = 0;
    }
    oc[e.obs0 + i] = e.cam0 + c;
    op[e.obs0 + i] = e.pt0 + p;
    if (info) {
#pragma unroll
      for (int k = 0; k < 3; ++k)
        info[3 * (e.obs0 + i) + k] = e.info ? e.info[3 * i + k] : (k == 1 ? 0.0 : 1.0);
    }
  }
  for (int64_t i = i0; i < 9 * (int64_t)e.n; i += stride) cams[9 * (int64_t)e.cam0 + i] = e.cams[i];
  for (int64_t i = i0; i < 3 * (int64_t)e.m; i += stride) pts[3 * (int64_t)e.pt0 + i] = e.pts[i];
  for (int64_t i = i0; i < e.n; i += stride) cam_scene[e.cam0 + i] = (int32_t)blockIdx.y;
}

// Off-diagonal block Z_ik = -sum_e J_P,a^T K_e J_P,b with K_e = Y_a J_X,b^T
// (2x2), written as -A^T B with A the stacked J_P,a (2E x 9) and B the stacked
// K_e J_P,b (2E x 9): an FP64 MFMA (16x16x4) contraction over the pair
// dimension, two pairs per instruction, rows and columns padded 9 -> 16.
// Lane l supplies A[kk][l%16] and B[kk][l%16] with kk = l/16 = 2 (pair) + row.
// (6 waves per SIMD: 80 registers without spills; more waves in flight
// beat deeper loads per wave here, and 8 waves spill)
// LDS writes of a wave visible to its own later reads (and its reads done
// before later writes): a wave's LDS accesses run in issue order, so a
// fence and a wave barrier suffice, no workgroup barrier.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(256, 6) void k_bin_blocks(SceneDev sc, const int2 *nzlist,
                                                   const int64_t *nzcount, const int64_t *bin_ptr,
                                                   const int2 *pairs, const double *rec,
                                                   const double *zdiag, const double *q,
                                                   const double *s, const double *alpha,
                                                   int mode, double *out, int64_t ld) {
  // Workgroups go round-robin to the 8 dies (XCDs); give each die a
  // contiguous run of the bin-ordered list (the grid is a multiple of 8), so
  // one die's L2 keeps a camera's records while its bins are reduced.
  __shared__ double lrec[4][8][2][kRec];  // per wave: 8 pairs x (record a, record b)
  const unsigned per = gridDim.x / 8;
  const unsigned logical = (blockIdx.x % 8) * per + blockIdx.x / 8;
  const int64_t w = (int64_t)logical * 4 + (threadIdx.x >> 6);
  if (w >= *nzcount) return;
  const int lane = threadIdx.x & 63;
  const int2 ik = nzlist[w];
  const int i = ik.x, k = ik.y;
  const int64_t N = 9 * (int64_t)sc.n;
  d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  const int col = lane & 15, kk = lane >> 4, p = kk & 1;
  if (i != k) {
    const int64_t bin = bin_of(sc, i, k);
    const int64_t e0 = bin_ptr[bin], e1 = bin_ptr[bin + 1];
    // 8 pairs (4 MFMAs) per iteration.  The wave first copies the 8 pairs'
    // two slot records into its LDS slot with 16-byte loads (8 lanes per
    // pair: 4 per record, 8 doubles each), then every lane reads its
    // operands there: 4 vector loads per lane and iteration instead of 48
    // narrow ones that mostly fetched the same values across 16 lanes.
    constexpr int U = 4;
    double(*my)[2][kRec] = lrec[threadIdx.x >> 6];
    const int q_ld = lane >> 3, part = lane & 7;
    for (int64_t e = e0; e < e1; e += 2 * U) {
      if (e + q_ld < e1) {
        const int2 pp = pairs[e + q_ld];
        const int slot = (part >> 2) ? pp.y : pp.x;
        const double2 *src =
            reinterpret_cast<const double2 *>(rec + (int64_t)slot * kRec + (part & 3) * 8);
        double2 *dst = reinterpret_cast<double2 *>(&my[q_ld][part >> 2][(part & 3) * 8]);
        const double2 v0 = src[0], v1 = src[1], v2 = src[2], v3 = src[3];
        dst[0] = v0;
        dst[1] = v1;
        dst[2] = v2;
        dst[3] = v3;
      }
      wave_lds_sync();
      double av[U], bv[U];
#pragma unroll
      for (int h = 0; h < U; ++h) {
        const int q = 2 * h + (kk >> 1);
        av[h] = 0.0;
        bv[h] = 0.0;
        if (e + q < e1 && col < 9) {
          const double *ra = my[q][0];
          const double *rb = my[q][1];
          av[h] = ra[kRecJP + 9 * p + col];
          const double y0 = ra[kRecY + 3 * p], y1 = ra[kRecY + 3 * p + 1], y2 = ra[kRecY + 3 * p + 2];
          const double k0 = y0 * rb[kRecJX + 0] + y1 * rb[kRecJX + 1] + y2 * rb[kRecJX + 2];
          const double k1 = y0 * rb[kRecJX + 3] + y1 * rb[kRecJX + 4] + y2 * rb[kRecJX + 5];
          bv[h] = k0 * rb[kRecJP + col] + k1 * rb[kRecJP + 9 + col];
        }
      }
      wave_lds_sync();  // the operands are read before the next copy
#pragma unroll
      for (int h = 0; h < U; h += 2) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[h], bv[h], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[h + 1], bv[h + 1], acc1, 0, 0, 0);
      }
    }
  }
  int si = 0;
  int64_t row0 = 0, off = 0, lds = ld;
  if (sc.cam_scene) {
    si = sc.cam_scene[i];
    row0 = 9 * (int64_t)sc.cam_off[si];
    off = sc.a_off[si];
    lds = sc.a_ld[si];
  }
  const double a = mode ? alpha[si] : 0.0;
  double *o = out + off;
  // gauge block Q_i Q_k^T (9 x 7 times 7 x 9) as two more 4-deep MFMA steps:
  // lane l supplies Q_i[l % 16][h] and Q_k[l % 16][h] with h = 4 t + l / 16
  d4 g4 = {0.0, 0.0, 0.0, 0.0};
  if (mode) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int h = 4 * t + (lane >> 4);
      const bool in = col < 9 && h < 7;
      const double qa = in ? q[h * N + 9 * (int64_t)i + col] : 0.0;
      const double qb = in ? q[h * N + 9 * (int64_t)k + col] : 0.0;
      g4 = __builtin_amdgcn_mfma_f64_16x16x4f64(qa, qb, g4, 0, 0, 0);
    }
  }
  const double sc_col = (mode && col < 9) ? s[9 * (int64_t)k + col] : 0.0;
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const int row = 4 * v + (lane >> 4);
    if (row >= 9 || col >= 9) continue;
    const double z = (i == k) ? zdiag[81 * (int64_t)i + 9 * row + col] : -(acc0[v] + acc1[v]);
    const int64_t pr = 9 * (int64_t)i + row, pc = 9 * (int64_t)k + col;  // global rows
    const int64_t lr = pr - row0, lc = pc - row0;                        // rows in the scene
    if (mode == 0) {
      o[lr + lc * lds] = z;
      o[lc + lr * lds] = z;
    } else {
      o[lr + lc * lds] = s[pr] * (z + a * g4[v]) * sc_col;
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, kBlk)), dim3(kBlk), 0, st, p, v, n);
}
void fill_f64(double *p, double v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(n, kBlk)), dim3(kBlk), 0, st, p, v, n);
}

void exclusive_scan(const int32_t *in, int64_t *out, int64_t len, int64_t *tmp,
                    hipStream_t st) {
  const int64_t ntiles = (len + kScanTile - 1) / kScanTile;
  if (ntiles > 0)
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(kScanThreads), 0, st, in,
                       out, len, tmp);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, st, tmp, ntiles);
  hipLaunchKernelGGL(k_scan_add, dim3(blocks_for(len + 1, kBlk)), dim3(kBlk), 0, st, out, len,
                     tmp, ntiles);
}

void launch_count_points(const SceneDev &sc, SceneWork &w, DevStatus *ds, hipStream_t st) {
  hipLaunchKernelGGL(k_count_points, dim3(blocks_for(sc.t, kBlk)), dim3(kBlk), 0, st, sc,
                     w.cnt_p, ds);
}

void launch_group_points(const SceneDev &sc, SceneWork &w, DevStatus *ds, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_slots, dim3(blocks_for(sc.t, kBlk)), dim3(kBlk), 0, st, sc,
                     w.ptr_p, w.cur_p, w.slot_key);
  hipLaunchKernelGGL(k_sort_points, dim3(blocks_for(sc.m, kSortThreads)), dim3(kSortThreads), 0,
                     st, sc, w.ptr_p, w.slot_key, w.slot_obs, w.slot_cam, w.slot_pt, ds);
}

void launch_jacobians(const SceneDev &sc, SceneWork &w, double *jp_out, double *jx_out,
                      DevStatus *ds, hipStream_t st) {
  hipLaunchKernelGGL(k_jacobians, dim3(blocks_for(sc.t, kBlk)), dim3(kBlk), 0, st, sc,
                     w.ptr_p, w.slot_obs, w.slot_cam, w.slot_pt, w.rec, jp_out, jx_out, ds);
}

void launch_point_blocks(const SceneDev &sc, SceneWork &w, DevStatus *ds, hipStream_t st) {
  hipLaunchKernelGGL(k_point_blocks, dim3(blocks_for(sc.m, kBlk)), dim3(kBlk), 0, st, sc,
                     w.ptr_p, w.rec, ds);
}

void launch_pair_count(const SceneDev &sc, SceneWork &w, hipStream_t st) {
  hipLaunchKernelGGL(k_pair_count, dim3(blocks_for(sc.t, kBlk)), dim3(kBlk), 0, st, sc,
                     w.ptr_p, w.slot_cam, w.slot_pt, w.bin_cnt);
}

void launch_nonzero_bins(const SceneDev &sc, SceneWork &w, int64_t nbins, hipStream_t st) {
  hipLaunchKernelGGL(k_nz_flag, dim3(blocks_for(nbins, kBlk)), dim3(kBlk), 0, st, nbins, w.bin_cnt,
                     w.bin_cur);
  exclusive_scan(w.bin_cur, w.nzpos, nbins, w.scan_tmp, st);
  hipLaunchKernelGGL(k_nz_compact, dim3(blocks_for(nbins, kBlk)), dim3(kBlk), 0, st, sc, nbins,
                     w.bin_cnt, w.nzpos, w.nzlist, w.nzcount);
  fill_i32(w.bin_cur, 0, nbins, st);
}

void launch_pair_fill(const SceneDev &sc, SceneWork &w, int64_t nbins, int64_t cap,
                      const int32_t *skip, hipStream_t st) {
  hipLaunchKernelGGL(k_pair_fill, dim3(blocks_for(sc.t, kBlk)), dim3(kBlk), 0, st, sc,
                     w.ptr_p, w.slot_cam, w.slot_pt, w.bin_ptr, w.bin_cur, w.pairs,
                     w.bin_ptr + nbins, cap, skip);
}

namespace {
// A replayed launch sequence was sized by the call that recorded it.  When
// the scene's pair count exceeds the pair list, every bin is emptied (so no
// kernel reads or writes pairs beyond the list) and UCOV_EINVAL is reported;
// more non-empty bins than recorded are reported as well (the bin reduction's
// grid covers the recorded count only).
__global__ void k_pairs_overflow(const int64_t *pairs, int64_t pairs_cap, int32_t *flag,
                                 DevStatus *ds) {
  *flag = *pairs > pairs_cap;
  if (*flag) report_error(ds, UCOV_EINVAL, -1);
}

__global__ void k_empty_bins_if(const int32_t *flag, int64_t nbins, int32_t *bin_cnt,
                                int64_t *bin_ptr) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (!*flag || b > nbins) return;
  if (b < nbins) bin_cnt[b] = 0;
  bin_ptr[b] = 0;
}

__global__ void k_check_nonzero(const int64_t *nz, int64_t nz_cap, DevStatus *ds) {
  if (*nz > nz_cap) report_error(ds, UCOV_EINVAL, -1);
}
}  // namespace

void launch_guard_pairs(SceneWork &w, int64_t nbins, int64_t pairs_cap, int32_t *flag,
                        DevStatus *ds, hipStream_t st) {
  hipLaunchKernelGGL(k_pairs_overflow, dim3(1), dim3(1), 0, st, w.bin_ptr + nbins, pairs_cap, flag,
                     ds);
  hipLaunchKernelGGL(k_empty_bins_if, dim3(blocks_for(nbins + 1, kBlk)), dim3(kBlk), 0, st, flag,
                     nbins, w.bin_cnt, w.bin_ptr);
}

void launch_check_nonzero(const SceneWork &w, int64_t nz_cap, DevStatus *ds, hipStream_t st) {
  hipLaunchKernelGGL(k_check_nonzero, dim3(1), dim3(1), 0, st, w.nzcount, nz_cap, ds);
}

// Scratch of the camera sort: ping-pong keys and values (t each), the
// (digit, block) histogram, its int64 offsets and the scan's tile sums.
struct RadixScratch {
  int32_t *keys, *vals, *hist;
  int64_t *offs, *scan;
};

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static RadixScratch radix_layout(void *tmp, int64_t t) {
  const int64_t nb = (t + kRadixItems - 1) / kRadixItems, len = 256 * nb;
  char *p = static_cast<char *>(tmp);
  RadixScratch r;
  r.keys = reinterpret_cast<int32_t *>(p);
  p += align256(4 * (size_t)t);
  r.vals = reinterpret_cast<int32_t *>(p);
  p += align256(4 * (size_t)t);
  r.hist = reinterpret_cast<int32_t *>(p);
  p += align256(4 * (size_t)len);
  r.offs = reinterpret_cast<int64_t *>(p);
  p += align256(8 * (size_t)(len + 1));
  r.scan = reinterpret_cast<int64_t *>(p);
  return r;
}

size_t camera_lists_scratch(int64_t t) {
  const int64_t nb = (t + kRadixItems - 1) / kRadixItems, len = 256 * nb;
  const int64_t scan_tiles = (len + 4095) / 4096 + 2;
  return 2 * align256(4 * (size_t)t) + align256(4 * (size_t)len) + align256(8 * (size_t)(len + 1)) +
         8 * (size_t)scan_tiles;
}

// Stable sort of t (key, value) pairs by the low `bits` bits of the
// non-negative keys, 8 bits per pass; the first *count pairs (count null:
// all t).  vals null: the values are the input positions.  keys and keys_out
// must not alias.
static void radix_sort_pairs(int64_t t, const int64_t *count, const int32_t *keys,
                             const int32_t *vals, int bits, int32_t *keys_out, int32_t *vals_out,
                             void *tmp, hipStream_t st) {
  const int passes = std::max(1, (bits + 7) / 8);
  const int64_t nb = (t + kRadixItems - 1) / kRadixItems;
  const RadixScratch r = radix_layout(tmp, t);
  const int32_t *kin = keys, *vin = vals;
  for (int p = 0; p < passes; ++p) {
    // the last pass writes the output, the one before it the scratch
    const bool to_out = (passes - 1 - p) % 2 == 0;
    int32_t *kout = to_out ? keys_out : r.keys, *vout = to_out ? vals_out : r.vals;
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kRadixThreads), 0, st, t, count,
                       kin, 8 * p, nb, r.hist);
    exclusive_scan(r.hist, r.offs, 256 * nb, r.scan, st);
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kRadixThreads), 0, st, t, count,
                       kin, vin, 8 * p, nb, r.offs, kout, vout);
    kin = kout;
    vin = vout;
  }
}

static int bits_for(int64_t n) {
  int bits = 1;
  while (bits < 31 && ((int64_t)1 << bits) < n) ++bits;
  return bits;
}

int launch_camera_lists(const SceneDev &sc, SceneWork &w, void *tmp, size_t tmp_bytes,
                        hipStream_t st) {
  const int64_t t = sc.t;
  if (tmp_bytes < camera_lists_scratch(t)) return -1;
  const int64_t *count = w.ptr_p + sc.m;  // slots placed by the point grouping
  radix_sort_pairs(t, count, w.slot_cam, nullptr, bits_for(sc.n), w.cam_keys, w.cam_slots, tmp,
                   st);
  hipLaunchKernelGGL(k_cam_bounds, dim3(blocks_for((int64_t)sc.n + 1, kBlk)), dim3(kBlk), 0, st,
                     sc.n, sc.t, count, w.cam_keys, w.cam_ptr);
  return 0;
}

void launch_pair_count_cam(const SceneDev &sc, SceneWork &w, int max_scene_cams,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_pair_count_cam, dim3(sc.n), dim3(kCamThreads),
                     sizeof(int32_t) * max_scene_cams, st, sc, w.cam_ptr, w.cam_slots, w.ptr_p,
                     w.slot_cam, w.slot_pt, w.bin_cnt);
}

void launch_pair_fill_cam(const SceneDev &sc, SceneWork &w, int max_scene_cams, int64_t nbins,
                          int64_t cap, const int32_t *skip, hipStream_t st) {
  hipLaunchKernelGGL(k_pair_fill_cam, dim3(sc.n), dim3(kFillThreads),
                     sizeof(int32_t) * max_scene_cams, st, sc, w.cam_ptr, w.cam_slots, w.ptr_p,
                     w.slot_cam, w.slot_pt, w.bin_ptr, w.pairs, w.bin_ptr + nbins, cap, skip);
}

void launch_camera_diag(const SceneDev &sc, SceneWork &w, DevStatus *ds, hipStream_t st) {
  hipLaunchKernelGGL(k_camera_diag<kDiagWaves>, dim3(sc.n), dim3(64 * kDiagWaves), 0, st, sc,
                     w.bin_ptr, w.pairs, w.rec, w.slot_pt, w.zdiag, w.hc, ds);
}

void launch_gauge(int64_t N, const double *hc, double *q, const double *zdiag,
                  const double *zdense, int64_t ldz, double user_alpha, double *s,
                  double *alpha, DevStatus *ds, hipStream_t st) {
  hipLaunchKernelGGL(k_gauge, dim3(1), dim3(kGaugeThreads), 0, st, N, hc, q, zdiag, zdense,
                     ldz, user_alpha, s, alpha, ds);
}

void launch_concat_scenes(int n_scenes, const BatchEntry *tab, int64_t max_elems, double *cams,
                          double *pts, double *info, int32_t *oc, int32_t *op,
                          int32_t *cam_scene, DevStatus *ds, hipStream_t st) {
  const unsigned bx = (unsigned)std::min<int64_t>(std::max<int64_t>(1, (max_elems + 255) / 256), 1024);
  hipLaunchKernelGGL(k_concat, dim3(bx, (unsigned)n_scenes), dim3(256), 0, st, tab, cams, pts,
                     info, oc, op, cam_scene, ds);
}

int64_t paper_gauge_doubles(int64_t m) { return kPaperF + 28 * blocks_for(m, 256); }

void launch_paper_gauge(const SceneDev &sc, SceneWork &w, double *f, DevStatus *ds,
                        hipStream_t st) {
  const int64_t N = 9 * (int64_t)sc.n;
  const int64_t nb = blocks_for(sc.m, 256);
  double *fpart = f + kPaperF;
  hipLaunchKernelGGL(k_paper_f, dim3(nb), dim3(256), 0, st, sc, w.ptr_p, w.rec, fpart);
  hipLaunchKernelGGL(k_paper_fsum, dim3(1), dim3(kFsumThreads), 0, st, nb, fpart, f);
  hipLaunchKernelGGL(k_paper_g, dim3(sc.n), dim3(256), 0, st, sc, w.bin_ptr, w.pairs, w.rec,
                     w.slot_pt, w.hc, w.q);
  hipLaunchKernelGGL(k_paper_p, dim3(1), dim3(1024), 0, st, N, f, w.q, w.alpha, ds);
}

// ---------------------------------------------------------------------------
// sub-reconstructions (Sec. 6): gather sub-scenes out of a parent scene and
// keep, per parent camera, the candidate block with the smallest trace
// ---------------------------------------------------------------------------
namespace {

__global__ void k_gather_subscenes(int64_t n, int64_t m, int64_t t, const int32_t *cam_src,
                                   const int32_t *pt_src, const int32_t *obs_src,
                                   const double *pcams, const double *ppts, const double *pinfo,
                                   double *cams, double *pts, double *info) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 9 * n) cams[i] = pcams[9 * (int64_t)cam_src[i / 9] + i % 9];
  if (i < 3 * m) pts[i] = ppts[3 * (int64_t)pt_src[i / 3] + i % 3];
  if (pinfo && i < 3 * t) info[i] = pinfo[3 * (int64_t)obs_src[i / 3] + i % 3];
}

// pos[d * n + c]: row of parent camera c's block in decomposition d
__global__ void k_min_trace(int64_t n, int n_decomp, const int32_t *pos, const double *cand,
                            double *cov, int32_t *chosen) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  int best = -1;
  double bt = 0.0;
  for (int d = 0; d < n_decomp; ++d) {
    const double *b = cand + 81 * (int64_t)pos[(int64_t)d * n + c];
    double tr = 0.0;
    for (int a = 0; a < 9; ++a) tr += b[10 * a];
    if (best < 0 || tr < bt) {
      best = d;
      bt = tr;
    }
  }
  const double *b = cand + 81 * (int64_t)pos[(int64_t)best * n + c];
  for (int k = 0; k < 81; ++k) cov[81 * c + k] = b[k];
  if (chosen) chosen[c] = best;
}

// ---- the sub-scenes' observations, chosen on the device --------------------
// A candidate is one observation o in one decomposition d, e = d t + o.  The
// candidates are sorted stably by point, then by sub-scene (the camera's
// group), so each (sub-scene, point) pair becomes one run, in sub-scene
// order, points ascending, observations ascending; a run of at least two
// observations is kept: that point belongs to the sub-scene.

// keys: the point of each candidate; out-of-range indices are reported
// (the first observation's index) and read as 0.
__global__ void k_sub_point_keys(int64_t t, int n_decomp, int32_t n, int32_t m,
                                 const int32_t *oc, const int32_t *op, int32_t *key,
                                 DevStatus *ds) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n_decomp * t) return;
  const int64_t o = e % t;
  const int32_t c = oc[o], j = op[o];
  const bool bad = c < 0 || c >= n || j < 0 || j >= m;
  if (bad && e < t) report_error(ds, UCOV_EINVAL, (int)o);
  key[e] = bad ? 0 : j;
}

// keys: the sub-scene of each candidate (after the sort by point)
__global__ void k_sub_group_keys(int64_t T, int64_t t, int32_t n, const int32_t *oc,
                                 const int32_t *gsub, const int32_t *cand, int32_t *key) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T) return;
  const int64_t e = cand[i], d = e / t;
  const int32_t c = min(max(oc[e % t], 0), n - 1);
  key[i] = gsub[d * n + c];
}

__device__ inline int32_t cand_point(const int32_t *op, const int32_t *cand, int64_t t,
                                     int64_t i, int32_t m) {
  return min(max(op[cand[i] % t], 0), m - 1);
}

// head[i]: candidate i starts a (sub-scene, point) run
__global__ void k_sub_heads(int64_t T, int64_t t, int32_t m, const int32_t *op,
                            const int32_t *sub, const int32_t *cand, int32_t *head) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T) return;
  head[i] = i == 0 || sub[i] != sub[i - 1] ||
            cand_point(op, cand, t, i, m) != cand_point(op, cand, t, i - 1, m);
}

// start[r] = first candidate of run r (run = inclusive scan of head - 1), and
// start[#runs] = T
__global__ void k_sub_run_starts(int64_t T, const int32_t *head, const int64_t *run,
                                 int64_t *start) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < T && head[i]) start[run[i]] = i;
  if (i == T) start[run[T]] = T;
}

// keep[i]: i's run holds at least two observations; khead[i]: i is the head
// of a kept run (a point of the sub-scene)
__global__ void k_sub_keep(int64_t T, const int32_t *head, const int64_t *run,
                           const int64_t *start, int32_t *keep, int32_t *khead) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T) return;
  const int64_t r = run[i] + head[i] - 1;
  const bool k = start[r + 1] - start[r] >= 2;
  keep[i] = k;
  khead[i] = k && head[i];
}

// Per sub-scene s <= S: the first kept observation and kept point, from the
// first candidate of a sub-scene >= s (binary search on the sorted keys).
__global__ void k_sub_offsets(int32_t S, int64_t T, const int32_t *sub, const int64_t *qpos,
                              const int64_t *kpos, int64_t *obs_off, int64_t *pt_off) {
  const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s > S) return;
  int64_t lo = 0, hi = T;
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (sub[mid] < s) lo = mid + 1;
    else hi = mid;
  }
  obs_off[s] = qpos[lo];
  pt_off[s] = kpos[lo];
}

// The kept candidates: parent observation, camera slot and point index in
// their sub-scene; each kept point's parent index.
__global__ void k_sub_emit(int64_t T, int64_t t, int32_t n, int32_t m, const int32_t *oc,
                           const int32_t *op, const int32_t *cslot, const int32_t *sub,
                           const int32_t *cand, const int32_t *keep, const int32_t *khead,
                           const int64_t *qpos, const int64_t *kpos, const int64_t *pt_off,
                           int32_t *obs_src, int32_t *loc_c, int32_t *loc_p, int32_t *pt_src) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T || !keep[i]) return;
  const int64_t e = cand[i], d = e / t, o = e % t;
  const int64_t kp = kpos[i] + khead[i] - 1;  // the run's point
  const int64_t q = qpos[i];
  obs_src[q] = (int32_t)o;
  loc_c[q] = cslot[d * n + min(max(oc[o], 0), n - 1)];
  loc_p[q] = (int32_t)(kp - pt_off[sub[i]]);
  if (khead[i]) pt_src[kp] = cand_point(op, cand, t, i, m);
}

}  // namespace

void launch_gather_subscenes(int64_t n, int64_t m, int64_t t, const int32_t *cam_src,
                             const int32_t *pt_src, const int32_t *obs_src, const double *pcams,
                             const double *ppts, const double *pinfo, double *cams, double *pts,
                             double *info, hipStream_t st) {
  const int64_t len = std::max({9 * n, 3 * m, pinfo ? 3 * t : (int64_t)0});
  hipLaunchKernelGGL(k_gather_subscenes, dim3(blocks_for(len, kBlk)), dim3(kBlk), 0, st, n, m, t,
                     cam_src, pt_src, obs_src, pcams, ppts, pinfo, cams, pts, info);
}

size_t subscene_select_scratch(int64_t T) {
  const int64_t tiles = (T + 1 + kScanTile - 1) / kScanTile + 2;
  return camera_lists_scratch(T) + 6 * align256(4 * (size_t)T) + 4 * align256(8 * (size_t)(T + 1)) +
         align256(8 * (size_t)tiles);
}

void launch_subscene_select(int64_t t, int n_decomp, int32_t n, int32_t m, int32_t S,
                            const int32_t *oc, const int32_t *op, const int32_t *gsub,
                            const int32_t *cslot, void *tmp, int64_t *obs_off, int64_t *pt_off,
                            int32_t *obs_src, int32_t *loc_c, int32_t *loc_p, int32_t *pt_src,
                            DevStatus *ds, hipStream_t st) {
  const int64_t T = (int64_t)n_decomp * t;
  char *p = static_cast<char *>(tmp);
  void *rtmp = p;
  p += camera_lists_scratch(T);
  auto take32 = [&]() {
    int32_t *r = reinterpret_cast<int32_t *>(p);
    p += align256(4 * (size_t)T);
    return r;
  };
  auto take64 = [&]() {
    int64_t *r = reinterpret_cast<int64_t *>(p);
    p += align256(8 * (size_t)(T + 1));
    return r;
  };
  int32_t *k0 = take32(), *k1 = take32(), *v1 = take32(), *cand = take32(), *head = take32(),
          *keep = take32();
  int32_t *khead = head;  // the heads are not needed once the runs are known
  int64_t *run = take64(), *start = take64(), *qpos = take64(), *kpos = take64();
  int64_t *scan_tmp = reinterpret_cast<int64_t *>(p);
  const unsigned g = blocks_for(T, kBlk), g1 = blocks_for(T + 1, kBlk);
  hipLaunchKernelGGL(k_sub_point_keys, dim3(g), dim3(kBlk), 0, st, t, n_decomp, n, m, oc, op, k0,
                     ds);
  radix_sort_pairs(T, nullptr, k0, nullptr, bits_for(m), k1, v1, rtmp, st);
  hipLaunchKernelGGL(k_sub_group_keys, dim3(g), dim3(kBlk), 0, st, T, t, n, oc, gsub, v1, k0);
  int32_t *sub = k1;
  radix_sort_pairs(T, nullptr, k0, v1, bits_for((int64_t)S), sub, cand, rtmp, st);
  hipLaunchKernelGGL(k_sub_heads, dim3(g), dim3(kBlk), 0, st, T, t, m, op, sub, cand, head);
  exclusive_scan(head, run, T, scan_tmp, st);
  hipLaunchKernelGGL(k_sub_run_starts, dim3(g1), dim3(kBlk), 0, st, T, head, run, start);
  hipLaunchKernelGGL(k_sub_keep, dim3(g), dim3(kBlk), 0, st, T, head, run, start, keep, khead);
  exclusive_scan(keep, qpos, T, scan_tmp, st);
  exclusive_scan(khead, kpos, T, scan_tmp, st);
  hipLaunchKernelGGL(k_sub_offsets, dim3(blocks_for((int64_t)S + 1, kBlk)), dim3(kBlk), 0, st, S,
                     T, sub, qpos, kpos, obs_off, pt_off);
  hipLaunchKernelGGL(k_sub_emit, dim3(g), dim3(kBlk), 0, st, T, t, n, m, oc, op, cslot, sub, cand,
                     keep, khead, qpos, kpos, pt_off, obs_src, loc_c, loc_p, pt_src);
}

void launch_min_trace(int64_t n, int n_decomp, const int32_t *pos, const double *cand,
                      double *cov, int32_t *chosen, hipStream_t st) {
  hipLaunchKernelGGL(k_min_trace, dim3(blocks_for(n, kBlk)), dim3(kBlk), 0, st, n, n_decomp, pos,
                     cand, cov, chosen);
}

void launch_gauge_scenes(const SceneDev &sc, const double *hc, double *q, const double *zdiag,
                         double user_alpha, double *s, double *alpha, DevStatus *ds,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_gauge_scenes, dim3((unsigned)sc.n_scenes), dim3(kGaugeThreads), 0, st, sc,
                     hc, q, zdiag, user_alpha, s, alpha, ds);
}

void launch_assemble(const SceneDev &sc, SceneWork &w, int mode, double *out, int64_t ld,
                     int64_t n_nonzero, hipStream_t st, int64_t max_scene_cams) {
  const int64_t rows = 9 * (max_scene_cams < 0 ? (int64_t)sc.n : max_scene_cams);
  hipLaunchKernelGGL(k_fill_empty, dim3((unsigned)sc.n, (unsigned)((rows + kFillRows - 1) / kFillRows)),
                     dim3(256), 0, st, sc, w.bin_cnt, w.q, w.s, w.alpha, mode, out, ld);
  if (n_nonzero > 0)
    hipLaunchKernelGGL(k_bin_blocks, dim3((blocks_for(n_nonzero, 4) + 7) / 8 * 8), dim3(256), 0, st, sc,
                       w.nzlist, w.nzcount, w.bin_ptr, w.pairs, w.rec, w.zdiag, w.q, w.s,
                       w.alpha, mode, out, ld);
}

}  // namespace ucov

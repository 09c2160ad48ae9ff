"""ctypes binding of the ucov C-ABI (argument marshalling only).

Every computation runs in the HIP kernels of ``lib/libucov.so``; this module
only passes device pointers of torch tensors and the current HIP stream.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libucov.so")

OK, EINVAL, EPOINT, EGAUGE, ENOCONV, EDEVICE, ENOMEM = 0, -1, -2, -3, -4, -5, -6
ERROR_NAMES = {EINVAL: "EINVAL", EPOINT: "EPOINT", EGAUGE: "EGAUGE", ENOCONV: "ENOCONV",
               EDEVICE: "EDEVICE", ENOMEM: "ENOMEM"}
FP64, FP32_NS, BF16X_NS = 0, 1, 2
GAUGE_CAMERA, GAUGE_PAPER = 0, 1


class Scene(ctypes.Structure):
    _fields_ = [("n_cams", ctypes.c_int32), ("n_pts", ctypes.c_int32), ("n_obs", ctypes.c_int64),
                ("cams", ctypes.c_void_p), ("pts", ctypes.c_void_p),
                ("obs_cam", ctypes.c_void_p), ("obs_pt", ctypes.c_void_p),
                ("obs_info", ctypes.c_void_p)]


class ScreenerStruct(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p), ("in_mean", ctypes.c_void_p),
                ("in_std", ctypes.c_void_p), ("scale", ctypes.c_void_p),
                ("out_mean", ctypes.c_void_p), ("out_std", ctypes.c_void_p),
                ("adam_m", ctypes.c_void_p), ("adam_v", ctypes.c_void_p),
                ("step", ctypes.c_int64)]


HOST_PTRS = 1


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("tol", ctypes.c_double), ("alpha", ctypes.c_double), ("gauge", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class Report(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("bad_index", ctypes.c_int32),
                ("ns_iters", ctypes.c_int32), ("ns_residual", ctypes.c_double),
                ("n_pairs", ctypes.c_int64),
                ("ms_structure", ctypes.c_float), ("ms_schur", ctypes.c_float),
                ("ms_gauge", ctypes.c_float), ("ms_inverse", ctypes.c_float),
                ("ms_extract", ctypes.c_float), ("bad_scene", ctypes.c_int32),
                ("ms_total", ctypes.c_float)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


EXPORTS = ["ucov_create", "ucov_set_stream", "ucov_destroy", "ucov_camera_covariance",
           "ucov_camera_covariance_batched",
           "ucov_jacobians", "ucov_reduced_camera_matrix", "ucov_gauge_basis",
           "ucov_pinv_blocks", "ucov_strerror", "ucov_last_error",
           "ucov_mlp_param_count", "ucov_screener_features", "ucov_mlp_forward",
           "ucov_mlp_gradient", "ucov_mlp_train", "ucov_screener_labels",
           "ucov_screener_covariance", "ucov_plan_check", "ucov_subrecon_covariance",
           "ucov_full_covariance", "ucov_update_covariance", "ucov_tune_dense",
           "ucov_camera_covariance_noalloc", "ucov_screener_stats", "ucov_screener_save",
           "ucov_screener_load", "ucov_split_bf16_update", "ucov_set_dense_threshold",
           "ucov_tune_batched", "ucov_batch_create", "ucov_batch_run", "ucov_batch_destroy"]

N_FEATURES, N_OUTPUTS = 55, 45

_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"ucov HIP library not built: {path} is missing "
                          "(run __graft_entry__.build() or python paper_1808_02414_amd/build.py)")
    lib = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "ucov_create": (ctypes.c_int, [ctypes.POINTER(P), ctypes.c_int]),
        "ucov_set_stream": (ctypes.c_int, [P, P]),
        "ucov_destroy": (None, [P]),
        "ucov_camera_covariance": (ctypes.c_int, [P, ctypes.POINTER(Scene), ctypes.POINTER(Options),
                                                  P, ctypes.POINTER(Report)]),
        "ucov_camera_covariance_noalloc": (ctypes.c_int, [P, ctypes.POINTER(Scene),
                                                          ctypes.POINTER(Options), P,
                                                          ctypes.POINTER(Report)]),
        "ucov_camera_covariance_batched": (ctypes.c_int, [P, I32, ctypes.POINTER(Scene),
                                                          ctypes.POINTER(Options), P,
                                                          ctypes.POINTER(D), ctypes.POINTER(Report)]),
        "ucov_full_covariance": (ctypes.c_int, [P, ctypes.POINTER(Scene), ctypes.POINTER(Options),
                                                P, I64, P, ctypes.POINTER(Report)]),
        "ucov_update_covariance": (ctypes.c_int, [P, ctypes.POINTER(Scene), I64, P, P, P, P, P, I64,
                                                  P, P, ctypes.POINTER(Report)]),
        "ucov_tune_dense": (ctypes.c_int, [P, I64, ctypes.POINTER(I64), ctypes.POINTER(ctypes.c_float)]),
        "ucov_jacobians": (ctypes.c_int, [P, ctypes.POINTER(Scene), P, P]),
        "ucov_reduced_camera_matrix": (ctypes.c_int, [P, ctypes.POINTER(Scene), P, I64,
                                                      ctypes.POINTER(Report)]),
        "ucov_gauge_basis": (ctypes.c_int, [P, ctypes.POINTER(Scene), P, P]),
        "ucov_pinv_blocks": (ctypes.c_int, [P, I64, P, I64, P, ctypes.POINTER(Options), P,
                                            ctypes.POINTER(Report)]),
        "ucov_mlp_param_count": (I64, []),
        "ucov_screener_features": (ctypes.c_int, [P, ctypes.POINTER(Scene), P]),
        "ucov_mlp_forward": (ctypes.c_int, [P, P, I64, P, P, P, P]),
        "ucov_mlp_gradient": (ctypes.c_int, [P, P, I64, P, P, P, P, P, P]),
        "ucov_mlp_train": (ctypes.c_int, [P, P, P, P, I64, ctypes.c_float, I64, I64, P, P, P,
                                          P, P]),
        "ucov_screener_labels": (ctypes.c_int, [P, I64, P, P, P, P, P, P]),
        "ucov_screener_covariance": (ctypes.c_int, [P, I64, P, P, P, P, P, P, P]),
        "ucov_plan_check": (ctypes.c_int, [P, I32, P]),
        "ucov_split_bf16_update": (ctypes.c_int, [P, I64, P, P]),
        "ucov_set_dense_threshold": (ctypes.c_int, [P, I64, I64]),
        "ucov_tune_batched": (ctypes.c_int, [P, I32, P, ctypes.POINTER(I64),
                                             ctypes.POINTER(ctypes.c_float)]),
        "ucov_batch_create": (ctypes.c_int, [P, I32, ctypes.POINTER(Scene), ctypes.POINTER(Options),
                                             P, ctypes.POINTER(P)]),
        "ucov_batch_run": (ctypes.c_int, [P, ctypes.POINTER(Report)]),
        "ucov_batch_destroy": (None, [P]),
        "ucov_screener_stats": (ctypes.c_int, [P, I64, P, P, P, P, P, P, P]),
        "ucov_screener_save": (ctypes.c_int, [P, ctypes.c_char_p, ctypes.POINTER(ScreenerStruct)]),
        "ucov_screener_load": (ctypes.c_int, [P, ctypes.c_char_p, ctypes.POINTER(ScreenerStruct)]),
        "ucov_subrecon_covariance": (ctypes.c_int, [P, ctypes.POINTER(Scene), I32, P,
                                                    ctypes.POINTER(Options), P, P, P,
                                                    ctypes.POINTER(Report)]),
        "ucov_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "ucov_last_error": (ctypes.c_char_p, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    del D
    _lib = lib
    return lib


def plan_check(np_sizes):
    """Host-only check of the batched inverse plan (see ucov_plan_check):
    returns (ok, number of launches)."""
    lib = load()
    arr = (ctypes.c_int64 * len(np_sizes))(*[int(x) for x in np_sizes])
    nl = ctypes.c_int64(0)
    rc = lib.ucov_plan_check(arr, len(np_sizes), ctypes.byref(nl))
    if rc == EINVAL:
        raise ValueError("sizes must be positive multiples of 64")
    return rc == OK, int(nl.value)


class UcovError(RuntimeError):
    def __init__(self, code: int, message: str, index: int = -1, scene: int = -1):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {message}")
        self.code = code
        self.kind = ERROR_NAMES.get(code, str(code))
        self.index = index
        self.scene = scene


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("ucov needs a GPU: torch.cuda.is_available() is False")
    return torch


class DeviceScene:
    """A reconstruction resident in device memory (torch tensors)."""

    def __init__(self, cams, pts, obs_cam, obs_pt, obs_info=None):
        self.cams, self.pts, self.obs_cam, self.obs_pt, self.obs_info = cams, pts, obs_cam, obs_pt, obs_info

    @classmethod
    def from_scene(cls, scene, device="cuda:0"):
        torch = _torch()

        def t(a, dt):
            return torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(device)

        info = None if scene.obs_info is None else t(scene.obs_info, torch.float64)
        return cls(t(scene.cams, torch.float64), t(scene.pts, torch.float64),
                   t(scene.obs_cam, torch.int32), t(scene.obs_pt, torch.int32), info)

    @property
    def n_cams(self):
        return int(self.cams.shape[0])

    @property
    def n_pts(self):
        return int(self.pts.shape[0])

    def struct(self) -> Scene:
        for a in (self.cams, self.pts, self.obs_cam, self.obs_pt):
            assert a.is_cuda and a.is_contiguous()
        return Scene(self.cams.shape[0], self.pts.shape[0], self.obs_cam.shape[0],
                     self.cams.data_ptr(), self.pts.data_ptr(), self.obs_cam.data_ptr(),
                     self.obs_pt.data_ptr(),
                     None if self.obs_info is None else self.obs_info.data_ptr())


class Context:
    """One ucov context on one device; calls use torch's current stream."""

    def __init__(self, device: int = 0):
        self.torch = _torch()
        self.lib = load()
        self.device = device
        h = ctypes.c_void_p()
        rc = self.lib.ucov_create(ctypes.byref(h), device)
        if rc != OK:
            raise UcovError(rc, "ucov_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.ucov_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        s = self.torch.cuda.current_stream(self.device).cuda_stream
        self.lib.ucov_set_stream(self.h, ctypes.c_void_p(s))

    def _check(self, rc, rep=None):
        if rc != OK:
            msg = self.lib.ucov_last_error(self.h).decode()
            raise UcovError(rc, msg, rep.bad_index if rep is not None else -1,
                            rep.bad_scene if rep is not None else -1)

    def camera_covariance(self, scene: DeviceScene, precision=FP64, alpha=0.0, tol=0.0,
                          max_iter=0, out=None, gauge=GAUGE_CAMERA):
        """(n, 9, 9) float64 covariance blocks on the device, and the report."""
        torch = self.torch
        n = scene.n_cams
        if out is None:
            out = torch.empty((n, 9, 9), dtype=torch.float64, device=scene.cams.device)
        opt = Options(precision, max_iter, tol, alpha, gauge)
        rep = Report()
        self._stream()
        sc = scene.struct()
        rc = self.lib.ucov_camera_covariance(self.h, ctypes.byref(sc), ctypes.byref(opt),
                                             out.data_ptr(), ctypes.byref(rep))
        self._check(rc, rep)
        return out, rep.as_dict()

    def camera_covariance_noalloc(self, scene: DeviceScene, out, alpha=0.0,
                                  gauge=GAUGE_CAMERA):
        """``camera_covariance`` in FP64 with the library's static scratch
        instead of its workspace (no device allocation in the call); ``out``
        is the caller's (n, 9, 9) float64 device tensor.  Returns out and the
        report."""
        torch = self.torch
        assert out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()
        assert out.shape == (scene.n_cams, 9, 9)
        opt = Options(FP64, 0, 0.0, alpha, gauge)
        rep = Report()
        self._stream()
        sc = scene.struct()
        rc = self.lib.ucov_camera_covariance_noalloc(self.h, ctypes.byref(sc), ctypes.byref(opt),
                                                     out.data_ptr(), ctypes.byref(rep))
        self._check(rc, rep)
        return out, rep.as_dict()

    def camera_covariance_host(self, scene, precision=FP64, alpha=0.0, gauge=GAUGE_CAMERA):
        """``camera_covariance`` on a scene held in host memory (numpy arrays of
        a ``scenegen.Scene``: cams, pts, obs_cam, obs_pt, obs_info): the library
        stages it through device buffers (UCOV_HOST_PTRS).  Returns (n, 9, 9)
        float64 numpy blocks and the report."""
        arrs = [np.ascontiguousarray(scene.cams, np.float64), np.ascontiguousarray(scene.pts, np.float64),
                np.ascontiguousarray(scene.obs_cam, np.int32), np.ascontiguousarray(scene.obs_pt, np.int32)]
        info = None if scene.obs_info is None else np.ascontiguousarray(scene.obs_info, np.float64)
        out = np.empty((arrs[0].shape[0], 9, 9), np.float64)
        sc = Scene(arrs[0].shape[0], arrs[1].shape[0], arrs[2].shape[0], arrs[0].ctypes.data,
                   arrs[1].ctypes.data, arrs[2].ctypes.data, arrs[3].ctypes.data,
                   None if info is None else info.ctypes.data)
        opt = Options(precision, 0, 0.0, alpha, gauge, HOST_PTRS)
        rep = Report()
        self._stream()
        rc = self.lib.ucov_camera_covariance(self.h, ctypes.byref(sc), ctypes.byref(opt),
                                             out.ctypes.data, ctypes.byref(rep))
        self._check(rc, rep)
        return out, rep.as_dict()

    def full_covariance(self, scene: DeviceScene, cameras=True, points=True, alpha=0.0,
                        gauge=GAUGE_CAMERA):
        """The whole camera covariance (N, N) and the point covariances
        (m, 3, 3) as float64 device tensors (None where not requested), and the
        report."""
        torch = self.torch
        dev = scene.cams.device
        N = 9 * scene.n_cams
        cam = torch.empty((N, N), dtype=torch.float64, device=dev) if cameras else None
        pts = torch.empty((scene.n_pts, 3, 3), dtype=torch.float64, device=dev) if points else None
        opt = Options(FP64, 0, 0.0, alpha, gauge)
        rep = Report()
        self._stream()
        sc = scene.struct()
        # column-major N x N with leading dimension N is the row-major tensor's transpose;
        # the matrix is symmetric
        rc = self.lib.ucov_full_covariance(self.h, ctypes.byref(sc), ctypes.byref(opt),
                                           cam.data_ptr() if cam is not None else None, N,
                                           pts.data_ptr() if pts is not None else None,
                                           ctypes.byref(rep))
        self._check(rc, rep)
        return cam, pts, rep.as_dict()

    def update_covariance(self, scene: DeviceScene, cam_cov, new_cam, new_pt, new_info=None,
                          cam_new=None):
        """Update the whole camera covariance ``cam_cov`` ((N, N) float64
        device tensor, as from ``full_covariance``) in place for the new
        observations (device int32 tensors; optional (k, 3) information and
        a new camera's 9 parameters).  Returns (cam_cov, new camera's 9 x 9
        covariance or None, its (N, 9) cross-covariance or None, report)."""
        torch = self.torch
        dev = scene.cams.device
        N = 9 * scene.n_cams
        assert cam_cov.shape == (N, N) and cam_cov.dtype == torch.float64 and cam_cov.is_contiguous()
        k = int(new_cam.numel())
        ncov = ncross = None
        if cam_new is not None:
            ncov = torch.empty((9, 9), dtype=torch.float64, device=dev)
            ncross = torch.empty((N, 9), dtype=torch.float64, device=dev)
        rep = Report()
        self._stream()
        sc = scene.struct()
        ptr = lambda t: None if t is None else t.data_ptr()  # noqa: E731
        rc = self.lib.ucov_update_covariance(self.h, ctypes.byref(sc), k, ptr(new_cam), ptr(new_pt),
                                             ptr(new_info), ptr(cam_new), cam_cov.data_ptr(), N,
                                             ptr(ncov), ptr(ncross), ctypes.byref(rep))
        self._check(rc, rep)
        return cam_cov, ncov, ncross, rep.as_dict()

    def tune_dense(self, n: int):
        """Pick the dense stage's tile schedule for matrices of size n (9 per
        camera); returns (threshold, milliseconds of the chosen schedule)."""
        th = ctypes.c_int64()
        ms = ctypes.c_float()
        self._stream()
        self._check(self.lib.ucov_tune_dense(self.h, int(n), ctypes.byref(th), ctypes.byref(ms)))
        return int(th.value), float(ms.value)

    def tune_batched(self, sizes):
        """Pick the batched dense stage's tile schedule for scenes of matrix
        sizes ``sizes`` (9 per camera, scene order); returns (threshold, ms)."""
        arr = (ctypes.c_int64 * len(sizes))(*[int(x) for x in sizes])
        th = ctypes.c_int64()
        ms = ctypes.c_float()
        self._stream()
        self._check(self.lib.ucov_tune_batched(self.h, len(sizes), arr, ctypes.byref(th),
                                               ctypes.byref(ms)))
        return int(th.value), float(ms.value)

    def set_dense_threshold(self, n: int, threshold: int):
        """Use a known tile-schedule threshold for matrices of size n."""
        self._check(self.lib.ucov_set_dense_threshold(self.h, int(n), int(threshold)))

    def camera_covariance_batched(self, scenes, alpha=0.0, out=None):
        """Covariance blocks of independent scenes in one call: a list of
        (n_s, 9, 9) views into one (sum n_s, 9, 9) device tensor, the per-scene
        gauge weights and the report."""
        torch = self.torch
        sizes = [s.n_cams for s in scenes]
        total = sum(sizes)
        if out is None:
            out = torch.empty((total, 9, 9), dtype=torch.float64, device=scenes[0].cams.device)
        arr = (Scene * len(scenes))(*[s.struct() for s in scenes])
        alphas = (ctypes.c_double * len(scenes))()
        opt = Options(FP64, 0, 0.0, alpha, GAUGE_CAMERA)
        rep = Report()
        self._stream()
        rc = self.lib.ucov_camera_covariance_batched(self.h, len(scenes), arr, ctypes.byref(opt),
                                                     out.data_ptr(), alphas, ctypes.byref(rep))
        self._check(rc, rep)
        views, o = [], 0
        for n in sizes:
            views.append(out[o:o + n])
            o += n
        return views, list(alphas), rep.as_dict()

    def batch(self, scenes, alpha=0.0, out=None):
        """A batch recorded once (eager solve, then a captured graph) and
        replayed by ``Batch.run()``; its blocks are written to ``out``."""
        return Batch(self, scenes, alpha, out)

    def subrecon_covariance(self, scene: DeviceScene, groups, alpha=0.0):
        """Per-camera blocks from sub-reconstructions: groups is an
        (n_decomp, n_cams) integer array of group ids; returns the (n, 9, 9)
        minimum-trace blocks, the decomposition chosen per camera, the number of
        sub-reconstructions and the report of the batched solve."""
        torch = self.torch
        g = np.ascontiguousarray(np.asarray(groups, dtype=np.int32).reshape(-1, scene.n_cams))
        out = torch.empty((scene.n_cams, 9, 9), dtype=torch.float64, device=scene.cams.device)
        chosen = np.zeros(scene.n_cams, dtype=np.int32)
        n_sub = ctypes.c_int32(0)
        opt = Options(FP64, 0, 0.0, alpha, GAUGE_CAMERA)
        rep = Report()
        self._stream()
        sc = scene.struct()
        rc = self.lib.ucov_subrecon_covariance(
            self.h, ctypes.byref(sc), g.shape[0], g.ctypes.data, ctypes.byref(opt), out.data_ptr(),
            chosen.ctypes.data, ctypes.byref(n_sub), ctypes.byref(rep))
        self._check(rc, rep)
        return out, chosen, int(n_sub.value), rep.as_dict()

    def jacobians(self, scene: DeviceScene):
        torch = self.torch
        t = scene.obs_cam.shape[0]
        jp = torch.empty((t, 2, 9), dtype=torch.float64, device=scene.cams.device)
        jx = torch.empty((t, 2, 3), dtype=torch.float64, device=scene.cams.device)
        self._stream()
        sc = scene.struct()
        self._check(self.lib.ucov_jacobians(self.h, ctypes.byref(sc), jp.data_ptr(), jx.data_ptr()))
        return jp, jx

    def reduced_camera_matrix(self, scene: DeviceScene):
        torch = self.torch
        N = 9 * scene.n_cams
        z = torch.empty((N, N), dtype=torch.float64, device=scene.cams.device)
        rep = Report()
        self._stream()
        sc = scene.struct()
        self._check(self.lib.ucov_reduced_camera_matrix(self.h, ctypes.byref(sc), z.data_ptr(), N,
                                                        ctypes.byref(rep)), rep)
        return z.T, rep.as_dict()  # column-major storage

    def gauge_basis(self, scene: DeviceScene):
        torch = self.torch
        N = 9 * scene.n_cams
        hc = torch.empty((7, N), dtype=torch.float64, device=scene.cams.device)
        q = torch.empty((7, N), dtype=torch.float64, device=scene.cams.device)
        self._stream()
        sc = scene.struct()
        self._check(self.lib.ucov_gauge_basis(self.h, ctypes.byref(sc), hc.data_ptr(), q.data_ptr()))
        return hc.T, q.T

    def pinv_blocks(self, z, q, alpha=0.0, precision=FP64):
        """Diagonal 9x9 blocks of Z^+ for a symmetric z (N, N) with null space
        spanned by the orthonormal columns of q (N, 7)."""
        torch = self.torch
        N = z.shape[0]
        zc = z.contiguous()  # symmetric: row-major storage is its own column-major form
        qc = q.T.contiguous()
        out = torch.empty((N // 9, 9, 9), dtype=torch.float64, device=z.device)
        opt = Options(precision, 0, 0.0, alpha, GAUGE_CAMERA)
        rep = Report()
        self._stream()
        self._check(self.lib.ucov_pinv_blocks(self.h, N, zc.data_ptr(), N, qc.data_ptr(),
                                              ctypes.byref(opt), out.data_ptr(), ctypes.byref(rep)), rep)
        return out, rep.as_dict()

    def split_bf16_update(self, x, r):
        """x += x r in place (n x n float64 device tensors, n a multiple of 64;
        row-major tensors are passed as their column-major transposes, so the
        call computes x^T += x^T r^T on the stored arrays)."""
        torch = self.torch
        n = x.shape[0]
        assert x.shape == (n, n) and r.shape == (n, n)
        self._stream()
        self._check(self.lib.ucov_split_bf16_update(self.h, n, self._dev(x, torch.float64),
                                                    self._dev(r, torch.float64)))
        return x

    # ---- learned screener ---------------------------------------------------

    def mlp_param_count(self) -> int:
        return int(self.lib.ucov_mlp_param_count())

    @staticmethod
    def _ptr(t):
        return None if t is None else t.data_ptr()

    def _dev(self, t, dtype):
        assert t.is_cuda and t.dtype == dtype and t.is_contiguous(), (t.device, t.dtype)
        return t.data_ptr()

    def screener_features(self, scene: DeviceScene):
        """(n, 55) float32 features of every camera."""
        torch = self.torch
        f = torch.empty((scene.n_cams, N_FEATURES), dtype=torch.float32, device=scene.cams.device)
        self._stream()
        sc = scene.struct()
        self._check(self.lib.ucov_screener_features(self.h, ctypes.byref(sc), f.data_ptr()))
        return f

    def mlp_forward(self, params, x, in_mean=None, in_std=None):
        torch = self.torch
        f32 = torch.float32
        y = torch.empty((x.shape[0], N_OUTPUTS), dtype=f32, device=x.device)
        self._stream()
        self._check(self.lib.ucov_mlp_forward(
            self.h, self._dev(params, f32), x.shape[0], self._dev(x, f32),
            None if in_mean is None else self._dev(in_mean, f32),
            None if in_std is None else self._dev(in_std, f32), y.data_ptr()))
        return y

    def mlp_gradient(self, params, x, target, in_mean=None, in_std=None):
        torch = self.torch
        f32 = torch.float32
        g = torch.empty_like(params)
        loss = torch.zeros(1, dtype=f32, device=x.device)
        self._stream()
        self._check(self.lib.ucov_mlp_gradient(
            self.h, self._dev(params, f32), x.shape[0], self._dev(x, f32),
            None if in_mean is None else self._dev(in_mean, f32),
            None if in_std is None else self._dev(in_std, f32), self._dev(target, f32),
            g.data_ptr(), loss.data_ptr()))
        return g, float(loss.item())

    def mlp_train(self, params, adam_m, adam_v, step0, lr, batch, x, target,
                  in_mean=None, in_std=None):
        """Adam steps over consecutive batches of (x, target) (rows beyond the
        last whole batch are not used); returns the per-batch losses."""
        torch = self.torch
        f32 = torch.float32
        nb = x.shape[0] // batch
        losses = torch.zeros(nb, dtype=f32, device=x.device)
        self._stream()
        self._check(self.lib.ucov_mlp_train(
            self.h, self._dev(params, f32), self._dev(adam_m, f32), self._dev(adam_v, f32),
            int(step0), float(lr), int(batch), int(nb), self._dev(x, f32),
            None if in_mean is None else self._dev(in_mean, f32),
            None if in_std is None else self._dev(in_std, f32), self._dev(target, f32),
            losses.data_ptr()))
        return losses

    def screener_labels(self, cov, features, scale, out_mean, out_std):
        """Standardised log-Cholesky labels (n, 45) of covariances (n, 9, 9)
        normalised by each camera's scale (from its features (n, 55))."""
        torch = self.torch
        n = cov.shape[0]
        lab = torch.empty((n, N_OUTPUTS), dtype=torch.float32, device=cov.device)
        self._stream()
        rc = self.lib.ucov_screener_labels(self.h, n, self._dev(cov, torch.float64),
                                           self._dev(features, torch.float32),
                                           self._dev(scale, torch.float64),
                                           self._dev(out_mean, torch.float32),
                                           self._dev(out_std, torch.float32), lab.data_ptr())
        self._check(rc)
        return lab

    def screener_stats(self, features, covs):
        """Standardisation statistics of a training set (features (n, 55)
        float32, covariances (n, 9, 9) float64): in_mean, in_std, scale,
        out_mean, out_std as device tensors."""
        torch = self.torch
        dev = features.device
        n = features.shape[0]
        in_mean = torch.empty(N_FEATURES, dtype=torch.float32, device=dev)
        in_std = torch.empty_like(in_mean)
        scale = torch.empty(9, dtype=torch.float64, device=dev)
        out_mean = torch.empty(N_OUTPUTS, dtype=torch.float32, device=dev)
        out_std = torch.empty_like(out_mean)
        self._stream()
        self._check(self.lib.ucov_screener_stats(
            self.h, n, self._dev(features, torch.float32), self._dev(covs, torch.float64),
            in_mean.data_ptr(), in_std.data_ptr(), scale.data_ptr(), out_mean.data_ptr(),
            out_std.data_ptr()))
        return in_mean, in_std, scale, out_mean, out_std

    def _screener_struct(self, t, step=0):
        ptr = self._ptr
        return ScreenerStruct(ptr(t["params"]), ptr(t["in_mean"]), ptr(t["in_std"]),
                              ptr(t["scale"]), ptr(t["out_mean"]), ptr(t["out_std"]),
                              ptr(t.get("adam_m")), ptr(t.get("adam_v")), int(step))

    def screener_save(self, path: str, tensors: dict, step: int = 0):
        """Write a screener (dict of device tensors: params, in_mean, in_std,
        scale, out_mean, out_std and optionally adam_m, adam_v) to ``path``."""
        self._stream()
        st = self._screener_struct(tensors, step)
        self._check(self.lib.ucov_screener_save(self.h, os.fsencode(path), ctypes.byref(st)))

    def screener_load(self, path: str, adam: bool = False, device="cuda"):
        """Read a screener file into new device tensors; returns (dict, step)."""
        torch = self.torch
        P = self.mlp_param_count()
        f32, f64 = torch.float32, torch.float64
        t = {"params": torch.empty(P, dtype=f32, device=device),
             "in_mean": torch.empty(N_FEATURES, dtype=f32, device=device),
             "in_std": torch.empty(N_FEATURES, dtype=f32, device=device),
             "scale": torch.empty(9, dtype=f64, device=device),
             "out_mean": torch.empty(N_OUTPUTS, dtype=f32, device=device),
             "out_std": torch.empty(N_OUTPUTS, dtype=f32, device=device)}
        if adam:
            t["adam_m"] = torch.empty(P, dtype=f32, device=device)
            t["adam_v"] = torch.empty(P, dtype=f32, device=device)
        self._stream()
        st = self._screener_struct(t)
        self._check(self.lib.ucov_screener_load(self.h, os.fsencode(path), ctypes.byref(st)))
        return t, int(st.step)

    def screener_covariance(self, y, features, scale, out_mean, out_std):
        """Predicted (n, 9, 9) covariances and (n,) spreads from network
        outputs y (n, 45) and the cameras' features (n, 55)."""
        torch = self.torch
        n = y.shape[0]
        cov = torch.empty((n, 9, 9), dtype=torch.float64, device=y.device)
        spread = torch.empty(n, dtype=torch.float64, device=y.device)
        self._stream()
        self._check(self.lib.ucov_screener_covariance(
            self.h, n, self._dev(y, torch.float32), self._dev(features, torch.float32),
            self._dev(scale, torch.float64), self._dev(out_mean, torch.float32),
            self._dev(out_std, torch.float32), cov.data_ptr(), spread.data_ptr()))
        return cov, spread


class Batch:
    """ucov_batch_create / ucov_batch_run / ucov_batch_destroy: the scenes'
    tensors and the output stay referenced while the batch lives."""

    def __init__(self, ctx: Context, scenes, alpha=0.0, out=None):
        torch = ctx.torch
        self.ctx = ctx
        self.scenes = list(scenes)
        total = sum(s.n_cams for s in self.scenes)
        if out is None:
            out = torch.empty((total, 9, 9), dtype=torch.float64, device=self.scenes[0].cams.device)
        assert out.shape == (total, 9, 9) and out.is_contiguous() and out.dtype == torch.float64
        self.out = out
        self._arr = (Scene * len(self.scenes))(*[s.struct() for s in self.scenes])
        opt = Options(FP64, 0, 0.0, alpha, GAUGE_CAMERA)
        h = ctypes.c_void_p()
        ctx._stream()
        ctx._check(ctx.lib.ucov_batch_create(ctx.h, len(self.scenes), self._arr, ctypes.byref(opt),
                                             out.data_ptr(), ctypes.byref(h)))
        self.h = h

    def views(self):
        out, o = [], 0
        for s in self.scenes:
            out.append(self.out[o:o + s.n_cams])
            o += s.n_cams
        return out

    def run(self):
        """Replay on the current stream; returns the report."""
        rep = Report()
        self.ctx._stream()
        self.ctx._check(self.ctx.lib.ucov_batch_run(self.h, ctypes.byref(rep)), rep)
        return rep.as_dict()

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.ucov_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

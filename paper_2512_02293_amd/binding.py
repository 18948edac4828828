"""Thin ctypes binding of the HIP library (include/vi_ba.h).

Argument marshalling only: device arrays are torch tensors on the GPU (their
data pointers are passed through), host arrays are NumPy, and every step of
the computation runs in the library's HIP kernels.  Loading fails loudly when
the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from ._build import LIB_PATH

VI_OK, VI_EINVAL, VI_ENOMEM, VI_EDEVICE, VI_ENOTPD, VI_ENONFINITE, VI_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
VI_PREC_FP64, VI_PREC_MIXED = 0, 1
STATUS_NAMES = {0: "VI_OK", -1: "VI_EINVAL", -2: "VI_ENOMEM", -3: "VI_EDEVICE", -4: "VI_ENOTPD",
                -5: "VI_ENONFINITE", -6: "VI_EUNSUPPORTED"}
NUM_STAGES = 6
STAGE_NAMES = ["vis_gram_imu", "local", "assemble", "cholesky", "backsub_retract", "final_cost"]
PREINT_DOUBLES = 154


class ViError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Camera(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("H", C.c_int32), ("W", C.c_int32), ("gravity", C.c_double * 3), ("T_bc", C.c_double * 7)]


class ImuNoise(C.Structure):
    _fields_ = [("sigma_g", C.c_double), ("sigma_a", C.c_double), ("sigma_bgw", C.c_double),
                ("sigma_baw", C.c_double)]


class State(C.Structure):
    _fields_ = [("n_kf", C.c_int32), ("pose", C.c_void_p), ("vel", C.c_void_p), ("bias", C.c_void_p),
                ("invdepth", C.c_void_p)]


class Edges(C.Structure):
    _fields_ = [("n_edges", C.c_int32), ("ii", C.c_void_p), ("jj", C.c_void_p), ("target", C.c_void_p),
                ("weight", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("n_fixed", C.c_int32), ("use_imu", C.c_int32), ("bias_mode", C.c_int32),
                ("precision", C.c_int32), ("invdepth_f32", C.c_int32), ("reserved", C.c_int32),
                ("lm_lambda", C.c_double), ("depth_eta", C.c_double), ("z_min", C.c_double), ("d_min", C.c_double)]


class Report(C.Structure):
    _fields_ = [("cost_before", C.c_double), ("cost_after", C.c_double), ("n_valid", C.c_int64),
                ("iters_done", C.c_int32), ("tile_px", C.c_int32), ("dxi", C.c_void_p), ("dd", C.c_void_p),
                ("costs", C.c_void_p), ("stage_ms", C.c_void_p)]


class Window(C.Structure):
    _fields_ = [("cam", Camera), ("state", State), ("edges", Edges), ("imu", C.c_void_p),
                ("report", C.POINTER(Report))]


class InertialInit(C.Structure):
    _fields_ = [("n_kf", C.c_int32), ("pose_vis", C.c_void_p), ("imu", C.c_void_p), ("vel_vis", C.c_void_p),
                ("bias", C.c_void_p), ("rot_wg", C.c_void_p), ("log_scale", C.c_void_p), ("cost", C.c_void_p)]


class RelPoses(C.Structure):
    _fields_ = [("n_rel", C.c_int32), ("ii", C.c_void_p), ("jj", C.c_void_p), ("meas", C.c_void_p),
                ("info", C.c_void_p)]


class Gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("anchor", C.c_void_p), ("mean_in", C.c_void_p), ("cov_in", C.c_void_p),
                ("mean_out", C.c_void_p), ("cov_out", C.c_void_p)]


EXPORTS = ["vi_ctx_create", "vi_ctx_destroy", "vi_ctx_set_stream", "vi_last_error", "vi_version",
           "imu_preintegrate", "vi_workspace_size", "vi_ba_step", "vi_ba_solve", "vi_workspace_size_batched",
           "vi_ba_solve_batched", "vi_ctx_set_autotune", "vi_ctx_set_tolerance", "vi_warm_param_count", "vi_warm_workspace_size",
           "vi_warm_features", "vi_warm_forward", "vi_warm_gradients", "vi_warm_adamw", "vi_warm_apply",
           "vi_warm_start_workspace_size", "vi_warm_start", "vi_ba_solve_warm", "vi_reanchor_workspace_size",
           "vi_gaussian_reanchor", "vi_gaussian_reanchor_noalloc", "vi_pgba_workspace_size", "vi_pgba_solve",
           "vi_predict_keyframe", "vi_inertial_init_workspace_size",
           "vi_inertial_init_solve"]

_lib = None


def load(path: str = LIB_PATH):
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    lib = C.CDLL(path)
    lib.vi_ctx_create.argtypes = [C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]
    lib.vi_ctx_create.restype = C.c_int
    lib.vi_ctx_destroy.argtypes = [C.c_void_p]
    lib.vi_ctx_destroy.restype = None
    lib.vi_ctx_set_stream.argtypes = [C.c_void_p, C.c_void_p]
    lib.vi_ctx_set_stream.restype = C.c_int
    lib.vi_last_error.argtypes = [C.c_void_p]
    lib.vi_last_error.restype = C.c_char_p
    lib.vi_version.argtypes = []
    lib.vi_version.restype = C.c_char_p
    lib.imu_preintegrate.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.POINTER(ImuNoise), C.c_void_p]
    lib.imu_preintegrate.restype = C.c_int
    lib.vi_workspace_size.argtypes = [C.POINTER(Camera), C.c_int32, C.POINTER(Edges), C.POINTER(Opts)]
    lib.vi_workspace_size.restype = C.c_size_t
    lib.vi_ba_step.argtypes = [C.c_void_p, C.POINTER(Camera), C.POINTER(State), C.POINTER(Edges), C.c_void_p,
                               C.POINTER(Opts), C.c_void_p, C.c_size_t, C.POINTER(Report)]
    lib.vi_ba_step.restype = C.c_int
    lib.vi_ba_solve.argtypes = [C.c_void_p, C.POINTER(Camera), C.POINTER(State), C.POINTER(Edges), C.c_void_p,
                                C.POINTER(Opts), C.c_int32, C.c_void_p, C.c_size_t, C.POINTER(Report)]
    lib.vi_ba_solve.restype = C.c_int
    lib.vi_workspace_size_batched.argtypes = [C.c_int32, C.POINTER(Window), C.POINTER(Opts)]
    lib.vi_workspace_size_batched.restype = C.c_size_t
    lib.vi_ba_solve_batched.argtypes = [C.c_void_p, C.c_int32, C.POINTER(Window), C.POINTER(Opts), C.c_int32,
                                        C.c_void_p, C.c_size_t]
    lib.vi_ba_solve_batched.restype = C.c_int
    lib.vi_ctx_set_autotune.argtypes = [C.c_void_p, C.c_int32]
    lib.vi_ctx_set_autotune.restype = C.c_int
    lib.vi_ctx_set_tolerance.argtypes = [C.c_void_p, C.c_double]
    lib.vi_ctx_set_tolerance.restype = C.c_int
    vp, i32, f32 = C.c_void_p, C.c_int32, C.c_float
    lib.vi_warm_param_count.argtypes = []
    lib.vi_warm_param_count.restype = i32
    lib.vi_warm_workspace_size.argtypes = [i32, i32, i32]
    lib.vi_warm_workspace_size.restype = C.c_size_t
    lib.vi_warm_features.argtypes = [vp, i32, C.POINTER(Window), C.POINTER(Opts), i32, i32, vp, vp]
    lib.vi_warm_features.restype = C.c_int
    lib.vi_warm_forward.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp]
    lib.vi_warm_forward.restype = C.c_int
    lib.vi_warm_gradients.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp, f32, vp, C.c_size_t, vp,
                                      C.POINTER(C.c_float)]
    lib.vi_warm_gradients.restype = C.c_int
    lib.vi_warm_adamw.argtypes = [vp, vp, vp, vp, vp, i32, f32, f32, f32, f32, f32]
    lib.vi_warm_adamw.restype = C.c_int
    lib.vi_warm_apply.argtypes = [vp, i32, C.POINTER(Window), C.POINTER(Opts), i32, i32, vp, vp]
    lib.vi_warm_apply.restype = C.c_int
    lib.vi_warm_start_workspace_size.argtypes = [i32, C.POINTER(Window), C.POINTER(Opts)]
    lib.vi_warm_start_workspace_size.restype = C.c_size_t
    lib.vi_warm_start.argtypes = [vp, i32, C.POINTER(Window), C.POINTER(Opts), vp, vp, C.c_size_t, vp]
    lib.vi_warm_start.restype = C.c_int
    lib.vi_reanchor_workspace_size.argtypes = [i32]
    lib.vi_reanchor_workspace_size.restype = C.c_size_t
    lib.vi_gaussian_reanchor.argtypes = [vp, i32, vp, vp, vp, C.POINTER(Gaussians), vp, C.c_size_t, vp]
    lib.vi_gaussian_reanchor.restype = C.c_int
    lib.vi_gaussian_reanchor_noalloc.argtypes = [vp, i32, vp, vp, vp, C.POINTER(Gaussians), vp]
    lib.vi_gaussian_reanchor_noalloc.restype = C.c_int
    lib.vi_pgba_workspace_size.argtypes = [C.POINTER(Camera), i32, C.POINTER(Edges), C.POINTER(RelPoses),
                                           C.POINTER(Opts)]
    lib.vi_pgba_workspace_size.restype = C.c_size_t
    lib.vi_pgba_solve.argtypes = [vp, C.POINTER(Camera), i32, vp, vp, vp, C.POINTER(Edges), C.POINTER(RelPoses),
                                  C.POINTER(Opts), i32, vp, C.c_size_t, C.POINTER(Report)]
    lib.vi_pgba_solve.restype = C.c_int
    lib.vi_predict_keyframe.argtypes = [vp, i32, vp, vp, vp, vp, C.POINTER(C.c_double * 3), C.c_double, vp, vp, vp,
                                        vp]
    lib.vi_predict_keyframe.restype = C.c_int
    lib.vi_inertial_init_workspace_size.argtypes = [i32, C.POINTER(InertialInit)]
    lib.vi_inertial_init_workspace_size.restype = C.c_size_t
    lib.vi_inertial_init_solve.argtypes = [vp, i32, C.POINTER(InertialInit), C.c_double, C.c_double, i32, vp,
                                           C.c_size_t]
    lib.vi_inertial_init_solve.restype = C.c_int
    lib.vi_ba_solve_warm.argtypes = [vp, i32, C.POINTER(Window), C.POINTER(Opts), vp, i32, vp, C.c_size_t, vp]
    lib.vi_ba_solve_warm.restype = C.c_int
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check_dev(t, shape, dtype, name, min_rows=None):
    """Device tensor of the given dtype, contiguous, with the given shape
    (None = any extent)."""
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name}: expected a contiguous {dtype} GPU tensor")
    if len(t.shape) != len(shape) or any(s is not None and int(a) != s for a, s in zip(t.shape, shape)):
        raise ValueError(f"{name}: shape {tuple(t.shape)} does not match {shape}")
    if min_rows is not None and int(t.shape[0]) < min_rows:
        raise ValueError(f"{name}: {int(t.shape[0])} rows, {min_rows} needed")


def make_camera(fx, fy, cx, cy, H, W, gravity=(0.0, 0.0, -9.81), T_bc=None) -> Camera:
    """T_bc: body-from-camera (t, q xyzw), None for the identity."""
    tb = (0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0) if T_bc is None else tuple(float(v) for v in T_bc)
    return Camera(fx, fy, cx, cy, H, W, (C.c_double * 3)(*gravity), (C.c_double * 7)(*tb))


VI_BIAS_PER_KF, VI_BIAS_FIXED, VI_BIAS_GLOBAL = 0, 1, 2


def make_opts(n_fixed=1, use_imu=True, bias_fixed=False, lm_lambda=1e-4, depth_eta=1e-8, z_min=0.1,
              d_min=1e-3, precision=0, bias_mode=None, invdepth_f32=False) -> Opts:
    """precision: VI_PREC_FP64 (0) or VI_PREC_MIXED (1); bias_mode: VI_BIAS_* (bias_fixed=True is
    VI_BIAS_FIXED); invdepth_f32: the states' inverse depths are float32 (mixed precision only)."""
    mode = (VI_BIAS_FIXED if bias_fixed else VI_BIAS_PER_KF) if bias_mode is None else int(bias_mode)
    return Opts(n_fixed, int(bool(use_imu)), mode, int(precision), int(bool(invdepth_f32)), 0, lm_lambda, depth_eta,
                z_min, d_min)


class Context:
    """A library context bound to one device and torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = load()
        self.torch = torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        h = C.c_void_p()
        rc = self.lib.vi_ctx_create(device, C.c_void_p(stream.cuda_stream), C.byref(h))
        if rc != VI_OK:
            raise ViError(rc, "vi_ctx_create failed")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            self.lib.vi_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != VI_OK:
            raise ViError(rc, self.lib.vi_last_error(self.h).decode())

    def last_error(self) -> str:
        return self.lib.vi_last_error(self.h).decode()

    # -- preintegration ------------------------------------------------------
    def imu_preintegrate(self, off: np.ndarray, gyro, accel, dt, bias_hat, noise, out=None):
        """Returns a (F, 154) float64 device tensor of vi_preint records."""
        torch = self.torch
        off = np.ascontiguousarray(off, dtype=np.int32)
        F = off.shape[0] - 1
        S = int(off[-1]) if F >= 0 else 0
        _check_dev(gyro, (None, 3), torch.float64, "gyro", min_rows=S)
        _check_dev(accel, (None, 3), torch.float64, "accel", min_rows=S)
        _check_dev(dt, (None,), torch.float64, "dt", min_rows=S)
        _check_dev(bias_hat, (max(F, 0), 6), torch.float64, "bias_hat")
        if out is None:
            out = torch.empty((F, PREINT_DOUBLES), dtype=torch.float64, device=gyro.device)
        nz = ImuNoise(*[float(x) for x in noise])
        rc = self.lib.imu_preintegrate(self.h, F, off.ctypes.data_as(C.c_void_p), _ptr(gyro), _ptr(accel),
                                       _ptr(dt), _ptr(bias_hat), C.byref(nz), _ptr(out))
        self._check(rc)
        return out

    # -- BA ------------------------------------------------------------------
    def workspace_size(self, cam: Camera, n_kf: int, ii: np.ndarray, jj: np.ndarray, opts: Opts) -> int:
        ed = Edges(int(ii.shape[0]), ii.ctypes.data_as(C.c_void_p), jj.ctypes.data_as(C.c_void_p), None, None)
        return int(self.lib.vi_workspace_size(C.byref(cam), n_kf, C.byref(ed), C.byref(opts)))

    def solve(self, cam: Camera, pose, vel, bias, invdepth, ii: np.ndarray, jj: np.ndarray, target, weight,
              imu, opts: Opts, iters: int, workspace, dxi=None, dd=None, costs: bool = False,
              stage_ms: bool = False):
        """Run ``iters`` steps in place.  Returns a dict report."""
        torch = self.torch
        ii = np.ascontiguousarray(ii, dtype=np.int32)
        jj = np.ascontiguousarray(jj, dtype=np.int32)
        N, E, H, W = int(pose.shape[0]), int(ii.shape[0]), int(cam.H), int(cam.W)
        if jj.shape != ii.shape:
            raise ValueError("ii and jj differ in length")
        _check_dev(pose, (N, 7), torch.float64, "pose")
        _check_dev(vel, (N, 3), torch.float64, "vel")
        _check_dev(bias, (N, 6), torch.float64, "bias")
        _check_dev(invdepth, (N, H, W), torch.float32 if opts.invdepth_f32 else torch.float64, "invdepth")
        _check_dev(target, (E, 2, H, W), torch.float32, "target")
        _check_dev(weight, (E, 2, H, W), torch.float32, "weight")
        if imu is not None:
            _check_dev(imu, (N - 1, PREINT_DOUBLES), torch.float64, "imu")
        if dxi is not None:
            _check_dev(dxi, (N, 15), torch.float64, "dxi")
        if dd is not None:
            _check_dev(dd, (N, H, W), torch.float64, "dd")
        _check_dev(workspace, (None,), torch.uint8, "workspace")
        st = State(int(pose.shape[0]), _ptr(pose), _ptr(vel), _ptr(bias), _ptr(invdepth))
        ed = Edges(int(ii.shape[0]), ii.ctypes.data_as(C.c_void_p), jj.ctypes.data_as(C.c_void_p),
                   _ptr(target), _ptr(weight))
        cost_arr = np.zeros(iters + 1) if costs else None
        stage_arr = np.zeros(NUM_STAGES, dtype=np.float32) if stage_ms else None
        rep = Report(0.0, 0.0, 0, 0, 0, _ptr(dxi), _ptr(dd),
                     cost_arr.ctypes.data_as(C.c_void_p) if costs else None,
                     stage_arr.ctypes.data_as(C.c_void_p) if stage_ms else None)
        nbytes = workspace.numel() * workspace.element_size()
        if iters == 1 and not costs and not stage_ms:
            rc = self.lib.vi_ba_step(self.h, C.byref(cam), C.byref(st), C.byref(ed), _ptr(imu), C.byref(opts),
                                     _ptr(workspace), nbytes, C.byref(rep))
        else:
            rc = self.lib.vi_ba_solve(self.h, C.byref(cam), C.byref(st), C.byref(ed), _ptr(imu), C.byref(opts),
                                      iters, _ptr(workspace), nbytes, C.byref(rep))
        out = dict(cost_before=rep.cost_before, cost_after=rep.cost_after, n_valid=int(rep.n_valid),
                   iters_done=int(rep.iters_done), tile_px=int(rep.tile_px), status=rc)
        if costs:
            out["costs"] = cost_arr
        if stage_ms:
            out["stage_ms"] = dict(zip(STAGE_NAMES, stage_arr.tolist()))
        self._check(rc)
        return out


    def set_autotune(self, enable: bool):
        self._check(self.lib.vi_ctx_set_autotune(self.h, int(bool(enable))))

    def set_tolerance(self, rel_tol: float):
        """Tolerance stop of later solves on this context (vi_ctx_set_tolerance); 0 turns it off."""
        self._check(self.lib.vi_ctx_set_tolerance(self.h, float(rel_tol)))

    # -- batches of independent windows ---------------------------------------
    def _windows(self, opts, probs, imus, with_reports, costs, iters, stage_ms=False):
        torch = self.torch
        n = len(probs)
        wins = (Window * n)()
        keep = []
        reps = []
        for w, (dp, imu) in enumerate(zip(probs, imus)):
            N, E, H, W = int(dp.pose.shape[0]), int(dp.ii.shape[0]), int(dp.cam.H), int(dp.cam.W)
            for t, shape, dt, name in ((dp.pose, (N, 7), torch.float64, "pose"), (dp.vel, (N, 3), torch.float64, "vel"),
                                       (dp.bias, (N, 6), torch.float64, "bias"),
                                       (dp.invdepth, (N, H, W),
                                        torch.float32 if opts.invdepth_f32 else torch.float64, "invdepth"),
                                       (dp.target, (E, 2, H, W), torch.float32, "target"),
                                       (dp.weight, (E, 2, H, W), torch.float32, "weight")):
                _check_dev(t, shape, dt, f"window {w} {name}")
            if imu is not None:
                _check_dev(imu, (N - 1, PREINT_DOUBLES), torch.float64, f"window {w} imu")
            wins[w].cam = dp.cam
            wins[w].state = State(N, _ptr(dp.pose), _ptr(dp.vel), _ptr(dp.bias), _ptr(dp.invdepth))
            wins[w].edges = Edges(E, dp.ii.ctypes.data_as(C.c_void_p), dp.jj.ctypes.data_as(C.c_void_p),
                                  _ptr(dp.target), _ptr(dp.weight))
            wins[w].imu = _ptr(imu)
            if with_reports:
                cost_arr = np.zeros(iters + 1) if costs else None
                stage_arr = np.zeros(NUM_STAGES, dtype=np.float32) if (stage_ms and w == 0) else None
                r = Report(0.0, 0.0, 0, 0, 0, None, None,
                           cost_arr.ctypes.data_as(C.c_void_p) if costs else None,
                           stage_arr.ctypes.data_as(C.c_void_p) if stage_arr is not None else None)
                keep.append((r, cost_arr, stage_arr))
                wins[w].report = C.pointer(r)
                reps.append((r, cost_arr, stage_arr))
        return wins, reps, keep

    def workspace_size_batched(self, probs, opts: Opts) -> int:
        wins, _, _ = self._windows(opts, probs, [None] * len(probs), False, False, 1)
        return int(self.lib.vi_workspace_size_batched(len(probs), wins, C.byref(opts)))

    def solve_batched(self, probs, imus, opts: Opts, iters: int, workspace, costs=False, stage_ms=False):
        """Solve every window of a batch in the same launches; returns per-window reports."""
        _check_dev(workspace, (None,), self.torch.uint8, "workspace")
        wins, reps, keep = self._windows(opts, probs, imus, True, costs, iters, stage_ms)
        rc = self.lib.vi_ba_solve_batched(self.h, len(probs), wins, C.byref(opts), iters, _ptr(workspace),
                                          workspace.numel())
        out = []
        for r, cost_arr, stage_arr in reps:
            d = dict(cost_before=r.cost_before, cost_after=r.cost_after, n_valid=int(r.n_valid),
                     iters_done=int(r.iters_done), tile_px=int(r.tile_px))
            if costs:
                d["costs"] = cost_arr
            if stage_arr is not None:
                d["stage_ms"] = dict(zip(STAGE_NAMES, stage_arr.tolist()))
            out.append(d)
        self._check(rc)
        return out


    # -- learned warm start ---------------------------------------------------
    def warm_features(self, probs, imus, opts: Opts, hq: int, wq: int):
        """Input planes of every keyframe of the windows: (feat [n][15][hq][wq], dims [n][2])."""
        torch = self.torch
        wins, _, _ = self._windows(opts, probs, imus, False, False, 1)
        n = sum(int(d.pose.shape[0]) for d in probs)
        feat = torch.empty((n, 15, hq, wq), dtype=torch.float32, device=probs[0].pose.device)
        dims = torch.empty((n, 2), dtype=torch.int32, device=probs[0].pose.device)
        self._check(self.lib.vi_warm_features(self.h, len(probs), wins, C.byref(opts), hq, wq, _ptr(feat), _ptr(dims)))
        return feat, dims

    def warm_forward(self, params, feat, dims):
        torch = self.torch
        n, _, hq, wq = feat.shape
        dd = torch.empty((n, hq, wq), dtype=torch.float32, device=feat.device)
        db = torch.empty((n, 6), dtype=torch.float32, device=feat.device)
        self._check(self.lib.vi_warm_forward(self.h, n, hq, wq, _ptr(dims), _ptr(params), _ptr(feat), _ptr(dd),
                                             _ptr(db)))
        return dd, db

    def warm_gradients(self, params, feat, dims, label_dd, label_db, n_valid, workspace=None):
        """(loss, grads) of the training loss; workspace is allocated when not given."""
        torch = self.torch
        n, _, hq, wq = feat.shape
        nb = int(self.lib.vi_warm_workspace_size(n, hq, wq))
        if workspace is None or workspace.numel() < nb:
            workspace = torch.empty(nb, dtype=torch.uint8, device=feat.device)
        grads = torch.empty_like(params)
        loss = C.c_float(0.0)
        self._check(self.lib.vi_warm_gradients(self.h, n, hq, wq, _ptr(dims), _ptr(params), _ptr(feat),
                                               _ptr(label_dd), _ptr(label_db), float(n_valid), _ptr(workspace),
                                               workspace.numel(), _ptr(grads), C.byref(loss)))
        return float(loss.value), grads

    def reanchor_workspace_size(self, n_kf: int) -> int:
        return int(self.lib.vi_reanchor_workspace_size(int(n_kf)))

    def gaussian_reanchor(self, pose_pre, pose_post, scale_change, anchor, mean_in, cov_in=None, mean_out=None,
                          cov_out=None, ws=None, n_rejected=None):
        """Loop-closure update of a Gaussian map (vi_gaussian_reanchor, Eq. 7-8).
        Device tensors: poses float64 [N][7], scale_change float64 [N], anchor
        int32 [K], means float32 [K][3], covariances float32 [K][6] (optional).
        Outputs default to the inputs (in place).  Asynchronous on the context's
        stream; n_rejected (device int32 [1], optional) receives the count of
        Gaussians left unchanged.  ws="noalloc" calls the allocation-free entry
        point (vi_gaussian_reanchor_noalloc) instead."""
        import torch
        N = int(pose_pre.shape[0])
        K = int(anchor.shape[0])
        _check_dev(pose_pre, (N, 7), torch.float64, "pose_pre")
        _check_dev(pose_post, (N, 7), torch.float64, "pose_post")
        _check_dev(scale_change, (N,), torch.float64, "scale_change")
        _check_dev(anchor, (K,), torch.int32, "anchor")
        _check_dev(mean_in, (K, 3), torch.float32, "mean_in")
        mean_out = mean_in if mean_out is None else mean_out
        _check_dev(mean_out, (K, 3), torch.float32, "mean_out")
        if cov_in is not None:
            _check_dev(cov_in, (K, 6), torch.float32, "cov_in")
            cov_out = cov_in if cov_out is None else cov_out
            _check_dev(cov_out, (K, 6), torch.float32, "cov_out")
        elif cov_out is not None:
            raise ValueError("cov_out given without cov_in")
        g = Gaussians(K, _ptr(anchor), _ptr(mean_in), _ptr(cov_in), _ptr(mean_out), _ptr(cov_out))
        if ws == "noalloc":
            # vi_gaussian_reanchor_noalloc: the library's fixed keyframe table, no workspace
            self._check(self.lib.vi_gaussian_reanchor_noalloc(self.h, N, _ptr(pose_pre), _ptr(pose_post),
                                                              _ptr(scale_change), C.byref(g), _ptr(n_rejected)))
            return
        if ws is None:
            ws = torch.empty(max(self.reanchor_workspace_size(N), 256), dtype=torch.uint8, device=mean_in.device)
        self._check(self.lib.vi_gaussian_reanchor(self.h, N, _ptr(pose_pre), _ptr(pose_post), _ptr(scale_change),
                                                  C.byref(g), _ptr(ws), ws.numel(), _ptr(n_rejected)))

    # -- loop closure: pose-graph bundle adjustment in Sim(3) ----------------------
    def _pgba_args(self, pg):
        torch = self.torch
        N, E, H, W = int(pg.pose.shape[0]), int(pg.ii.shape[0]), int(pg.cam.H), int(pg.cam.W)
        _check_dev(pg.pose, (N, 7), torch.float64, "pose")
        _check_dev(pg.scale, (N,), torch.float64, "scale")
        _check_dev(pg.invdepth, (N, H, W), torch.float64, "invdepth")
        _check_dev(pg.target, (E, 2, H, W), torch.float32, "target")
        _check_dev(pg.weight, (E, 2, H, W), torch.float32, "weight")
        R = int(pg.rel_ii.shape[0])
        _check_dev(pg.rel_meas, (R, 8), torch.float64, "rel_meas")
        _check_dev(pg.rel_info, (R, 7, 7), torch.float64, "rel_info")
        ed = Edges(E, pg.ii.ctypes.data_as(C.c_void_p), pg.jj.ctypes.data_as(C.c_void_p), _ptr(pg.target),
                   _ptr(pg.weight))
        rel = RelPoses(R, pg.rel_ii.ctypes.data_as(C.c_void_p), pg.rel_jj.ctypes.data_as(C.c_void_p),
                       _ptr(pg.rel_meas), _ptr(pg.rel_info))
        return N, ed, rel

    def pgba_workspace_size(self, pg, opts: Opts) -> int:
        N, ed, rel = self._pgba_args(pg)
        return int(self.lib.vi_pgba_workspace_size(C.byref(pg.cam), N, C.byref(ed), C.byref(rel), C.byref(opts)))

    def pgba_solve(self, pg, opts: Opts, iters: int, workspace, dxi=None, dd=None):
        """vi_pgba_solve on a DevicePGBA problem (state updated in place); returns the report."""
        N, ed, rel = self._pgba_args(pg)
        if dxi is not None:
            _check_dev(dxi, (N, 7), self.torch.float64, "dxi")
        if dd is not None:
            _check_dev(dd, tuple(pg.invdepth.shape), self.torch.float64, "dd")
        _check_dev(workspace, (None,), self.torch.uint8, "workspace")
        costs = np.zeros(iters + 1)
        rep = Report(0.0, 0.0, 0, 0, 0, _ptr(dxi), _ptr(dd), costs.ctypes.data_as(C.c_void_p), None)
        rc = self.lib.vi_pgba_solve(self.h, C.byref(pg.cam), N, _ptr(pg.pose), _ptr(pg.scale), _ptr(pg.invdepth),
                                    C.byref(ed), C.byref(rel), C.byref(opts), iters, _ptr(workspace),
                                    workspace.numel(), C.byref(rep))
        self._check(rc)
        return dict(cost_before=rep.cost_before, cost_after=rep.cost_after, n_valid=int(rep.n_valid),
                    iters_done=int(rep.iters_done), tile_px=int(rep.tile_px), costs=costs)

    def predict_keyframe(self, pose_prev, vel_prev, bias_prev, imu, gravity, tau=1e-4, pose_new=None,
                         vel_new=None, bias_new=None, used_imu=None):
        """Initial state of new keyframes from preintegration (vi_predict_keyframe).
        Device tensors float64 [n][7], [n][3], [n][6]; imu = float64 [n][154]
        factors (as returned by imu_preintegrate); gravity = 3 host floats.
        Returns (pose_new, vel_new, bias_new, used_imu), allocating what is not
        given.  Asynchronous on the context's stream."""
        import torch
        n = int(pose_prev.shape[0])
        _check_dev(pose_prev, (n, 7), torch.float64, "pose_prev")
        _check_dev(vel_prev, (n, 3), torch.float64, "vel_prev")
        _check_dev(bias_prev, (n, 6), torch.float64, "bias_prev")
        _check_dev(imu, (n, PREINT_DOUBLES), torch.float64, "imu")
        pose_new = torch.empty_like(pose_prev) if pose_new is None else pose_new
        vel_new = torch.empty_like(vel_prev) if vel_new is None else vel_new
        bias_new = torch.empty_like(bias_prev) if bias_new is None else bias_new
        used_imu = torch.empty(n, dtype=torch.int32, device=pose_prev.device) if used_imu is None else used_imu
        _check_dev(pose_new, (n, 7), torch.float64, "pose_new")
        _check_dev(vel_new, (n, 3), torch.float64, "vel_new")
        _check_dev(bias_new, (n, 6), torch.float64, "bias_new")
        _check_dev(used_imu, (n,), torch.int32, "used_imu")
        g = (C.c_double * 3)(*[float(x) for x in gravity])
        self._check(self.lib.vi_predict_keyframe(self.h, n, _ptr(pose_prev), _ptr(vel_prev), _ptr(bias_prev),
                                                 _ptr(imu), C.byref(g), float(tau), _ptr(pose_new), _ptr(vel_new),
                                                 _ptr(bias_new), _ptr(used_imu)))
        return pose_new, vel_new, bias_new, used_imu

    def inertial_init_solve(self, problems, gravity_z=-9.81, lm_lambda=0.0, iters=10, ws=None):
        """IMU initialisation stage 2 (vi_inertial_init_solve) on a batch.
        problems: list of dicts of device float64 tensors: pose_vis [N][7],
        imu [N-1][154], vel_vis [N][3], bias [N][6], rot_wg [4], log_scale [1],
        optional cost [iters + 1]; the state tensors are updated in place.
        Synchronous."""
        import torch
        descs = (InertialInit * len(problems))()
        for k, q in enumerate(problems):
            N = int(q["pose_vis"].shape[0])
            _check_dev(q["pose_vis"], (N, 7), torch.float64, "pose_vis")
            _check_dev(q["imu"], (N - 1, PREINT_DOUBLES), torch.float64, "imu")
            _check_dev(q["vel_vis"], (N, 3), torch.float64, "vel_vis")
            _check_dev(q["bias"], (N, 6), torch.float64, "bias")
            _check_dev(q["rot_wg"], (4,), torch.float64, "rot_wg")
            _check_dev(q["log_scale"], (1,), torch.float64, "log_scale")
            if q.get("cost") is not None:
                _check_dev(q["cost"], (iters + 1,), torch.float64, "cost")
            descs[k] = InertialInit(N, _ptr(q["pose_vis"]), _ptr(q["imu"]), _ptr(q["vel_vis"]), _ptr(q["bias"]),
                                    _ptr(q["rot_wg"]), _ptr(q["log_scale"]), _ptr(q.get("cost")))
        nb = int(self.lib.vi_inertial_init_workspace_size(len(problems), descs))
        if ws is None:
            ws = torch.empty(max(nb, 256), dtype=torch.uint8, device="cuda:%d" % self.device)
        self._check(self.lib.vi_inertial_init_solve(self.h, len(problems), descs, float(gravity_z), float(lm_lambda),
                                                    int(iters), _ptr(ws), ws.numel()))

    def warm_adamw(self, params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=1e-4):
        self._check(self.lib.vi_warm_adamw(self.h, _ptr(params), _ptr(grads), _ptr(m), _ptr(v), int(t), float(lr),
                                           float(beta1), float(beta2), float(eps), float(weight_decay)))

    def warm_apply(self, probs, imus, opts: Opts, dd, db):
        n, hq, wq = dd.shape
        wins, _, _ = self._windows(opts, probs, imus, False, False, 1)
        self._check(self.lib.vi_warm_apply(self.h, len(probs), wins, C.byref(opts), hq, wq, _ptr(dd), _ptr(db)))

    def warm_start_workspace_size(self, probs, opts: Opts) -> int:
        wins, _, _ = self._windows(opts, probs, [None] * len(probs), False, False, 1)
        return int(self.lib.vi_warm_start_workspace_size(len(probs), wins, C.byref(opts)))

    def warm_start(self, probs, imus, opts: Opts, params, workspace):
        """Warm start of every window with the plain cost as the arbiter; returns
        per-window dicts (accepted, cost_init, cost_warm, cost_after)."""
        _check_dev(workspace, (None,), self.torch.uint8, "workspace")
        _check_dev(params, (int(self.lib.vi_warm_param_count()),), self.torch.float32, "params")
        wins, reps, keep = self._windows(opts, probs, imus, True, True, 1)
        acc = np.zeros(len(probs), dtype=np.int32)
        self._check(self.lib.vi_warm_start(self.h, len(probs), wins, C.byref(opts), _ptr(params), _ptr(workspace),
                                           workspace.numel(), acc.ctypes.data_as(C.c_void_p)))
        return [dict(accepted=bool(a), cost_init=float(c[0]), cost_warm=float(c[1]), cost_after=r.cost_after)
                for a, (r, c, _) in zip(acc, reps)]

    def solve_warm(self, probs, imus, opts: Opts, params, iters: int, workspace, costs=False):
        """Warm start then iters GN steps in one graph; per-window reports with 'accepted'."""
        _check_dev(workspace, (None,), self.torch.uint8, "workspace")
        _check_dev(params, (int(self.lib.vi_warm_param_count()),), self.torch.float32, "params")
        wins, reps, keep = self._windows(opts, probs, imus, True, costs, max(iters, 1))
        acc = np.zeros(len(probs), dtype=np.int32)
        self._check(self.lib.vi_ba_solve_warm(self.h, len(probs), wins, C.byref(opts), _ptr(params), iters,
                                              _ptr(workspace), workspace.numel(), acc.ctypes.data_as(C.c_void_p)))
        out = []
        for a, (r, cost_arr, _) in zip(acc, reps):
            d = dict(accepted=bool(a), cost_before=r.cost_before, cost_after=r.cost_after, n_valid=int(r.n_valid),
                     iters_done=int(r.iters_done))
            if costs:
                d["costs"] = cost_arr[: iters + 1]
            out.append(d)
        return out


class DeviceProblem:
    """A synthetic problem's arrays moved to the GPU (inputs resident in HBM)."""

    def __init__(self, prob, device="cuda:0", invdepth_f32=False):
        import torch
        self.prob = prob
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=device)
        self.pose = t(prob.pose, torch.float64)
        self.vel = t(prob.vel, torch.float64)
        self.bias = t(prob.bias, torch.float64)
        self.invdepth = t(prob.invdepth, torch.float32 if invdepth_f32 else torch.float64)
        self.target = t(prob.target, torch.float32)
        self.weight = t(prob.weight, torch.float32)
        self.gyro = t(prob.gyro, torch.float64)
        self.accel = t(prob.accel, torch.float64)
        self.imu_dt = t(prob.imu_dt, torch.float64)
        self.bias_hat = t(prob.bias_hat, torch.float64)
        self.ii = np.ascontiguousarray(prob.ii, dtype=np.int32)
        self.jj = np.ascontiguousarray(prob.jj, dtype=np.int32)
        self.off = np.ascontiguousarray(prob.imu_off, dtype=np.int32)
        self.cam = make_camera(prob.fx, prob.fy, prob.cx, prob.cy, prob.H, prob.W, tuple(prob.gravity),
                               getattr(prob, "T_bc", None))
        self.noise = tuple(float(x) for x in prob.noise)

    def reset_state(self):
        import torch
        p = self.prob
        self.pose.copy_(torch.as_tensor(p.pose))
        self.vel.copy_(torch.as_tensor(p.vel))
        self.bias.copy_(torch.as_tensor(p.bias))
        self.invdepth.copy_(torch.as_tensor(p.invdepth).to(self.invdepth.dtype))


class DevicePGBA:
    """A synthetic pose-graph problem's arrays on the GPU."""

    def __init__(self, prob, device="cuda:0"):
        import torch
        self.prob = prob
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=device)
        self.pose = t(prob.pose, torch.float64)
        self.scale = t(prob.scale, torch.float64)
        self.invdepth = t(prob.invdepth, torch.float64)
        self.target = t(prob.target, torch.float32)
        self.weight = t(prob.weight, torch.float32)
        self.rel_meas = t(prob.rel_meas, torch.float64)
        self.rel_info = t(prob.rel_info, torch.float64)
        self.ii = np.ascontiguousarray(prob.ii, dtype=np.int32)
        self.jj = np.ascontiguousarray(prob.jj, dtype=np.int32)
        self.rel_ii = np.ascontiguousarray(prob.rel_ii, dtype=np.int32)
        self.rel_jj = np.ascontiguousarray(prob.rel_jj, dtype=np.int32)
        self.cam = make_camera(prob.fx, prob.fy, prob.cx, prob.cy, prob.H, prob.W)

    def reset_state(self):
        import torch
        self.pose.copy_(torch.as_tensor(self.prob.pose))
        self.scale.copy_(torch.as_tensor(self.prob.scale))
        self.invdepth.copy_(torch.as_tensor(self.prob.invdepth))

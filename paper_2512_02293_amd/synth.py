"""Seeded synthetic workloads for the visual-inertial bundle-adjustment step.

This module only *simulates sensors*.  It draws a smooth, periodic rig
trajectory, samples an ideal IMU along it, gives every keyframe its own smooth
inverse-depth field and projects each keyframe's pixels into its neighbours to
make correspondence targets.  It holds none of the solver's arithmetic: no
residual linearisation, no preintegration, no normal equations.  Both the CPU
oracle and the HIP path consume the arrays it returns, and nothing else is
shared between them.

Ground truth is *discrete-consistent*: the rig state at every IMU tick is
defined by integrating the sampled angular rate and specific force with a
zero-order hold (rotation by the exact exponential of ``omega*dt``, velocity and
position with the exact constant-acceleration update).  With zero noise and a
bias linearisation point equal to the true bias, a preintegrated IMU factor is
therefore exactly satisfied by the ground truth, up to rounding.

Conventions (the paper leaves them open; Sec. 3.1, Eq. 1-3):
  * world frame is z-up, gravity ``(0, 0, -9.81)``;
  * the camera frame equals the body frame (identity camera-IMU extrinsics);
  * a pose is world-from-body, stored ``(px, py, pz, qx, qy, qz, qw)``;
  * pixel ``(x, y)`` = (column, row) at integer coordinates;
  * ``fx = fy = 60 * W / 64``, ``cx = W / 2``, ``cy = H / 2`` (60/60/32/24 at
    48x64 and 75/75/40/30 at 60x80, i.e. the same field of view).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Tuple

import numpy as np

GRAVITY = np.array([0.0, 0.0, -9.81])
TRAJ_PERIOD_S = 6.4          # trajectory period: 64 keyframes at 10 Hz


# --------------------------------------------------------------------------
# small quaternion helpers (Hamilton product, xyzw storage)
# --------------------------------------------------------------------------
def _qmul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    ax, ay, az, aw = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    bx, by, bz, bw = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([
        aw * bx + ax * bw + ay * bz - az * by,
        aw * by - ax * bz + ay * bw + az * bx,
        aw * bz + ax * by - ay * bx + az * bw,
        aw * bw - ax * bx - ay * by - az * bz,
    ], axis=-1)


def _quat_from_rotvec(v: np.ndarray) -> np.ndarray:
    """Unit quaternion of the rotation by angle |v| about v/|v| (half-angle form)."""
    v = np.asarray(v, dtype=np.float64)
    ang = np.linalg.norm(v, axis=-1, keepdims=True)
    half = 0.5 * ang
    # sin(half)/ang with its series near zero
    with np.errstate(invalid="ignore", divide="ignore"):
        k = np.where(ang > 1e-8, np.sin(half) / np.where(ang > 0, ang, 1.0),
                     0.5 - ang * ang / 48.0)
    return np.concatenate([v * k, np.cos(half)], axis=-1)


def _quat_to_mat(q: np.ndarray) -> np.ndarray:
    x, y, z, w = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    n = x * x + y * y + z * z + w * w
    s = 2.0 / n
    return np.stack([
        np.stack([1 - s * (y * y + z * z), s * (x * y - z * w), s * (x * z + y * w)], -1),
        np.stack([s * (x * y + z * w), 1 - s * (x * x + z * z), s * (y * z - x * w)], -1),
        np.stack([s * (x * z - y * w), s * (y * z + x * w), 1 - s * (x * x + y * y)], -1),
    ], -2)


def _unit(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


# --------------------------------------------------------------------------
# configuration
# --------------------------------------------------------------------------
@dataclass
class SceneConfig:
    """Shape and noise of one synthetic window (one keyframe graph)."""
    n_kf: int = 8
    H: int = 48
    W: int = 64
    k_out: int = 3                      # outgoing edges per keyframe, nearest by index
    n_loop: int = 0                     # extra long-range edges (|i-j| >= loop_gap)
    loop_gap: int = 55
    out_degrees: Optional[List[int]] = None   # per-KF out-degree (overrides k_out)
    imu_rate: float = 200.0
    kf_gap: int = 20                    # IMU samples between keyframes
    gap_range: Optional[Tuple[int, int]] = None   # uniform integer gaps instead
    gaps: Optional[List[int]] = None    # explicit IMU samples per keyframe gap (n_kf - 1 of them)
    sigma_px: float = 0.5
    w_lo: float = 0.1
    w_hi: float = 1.0
    sigma_g: float = 1.7e-4             # rad/s/sqrt(Hz)
    sigma_a: float = 2e-3               # m/s^2/sqrt(Hz)
    sigma_bgw: float = 2e-5             # rad/s^2/sqrt(Hz)
    sigma_baw: float = 3e-3             # m/s^3/sqrt(Hz)
    bg0_std: float = 0.005
    ba0_std: float = 0.05
    init_dp: float = 0.05               # m
    init_dtheta_deg: float = 2.0
    init_depth_rel: float = 0.1
    init_depth_smooth: bool = False     # relative depth error: smooth field (True) or per-pixel white
    init_dv_std: float = 0.05
    z_min: float = 0.1
    noiseless: bool = False             # no pixel/IMU noise, no bias random walk
    zero_bias: bool = False             # true bias identically zero
    # body-from-camera extrinsic (t (3), q xyzw (4)); None: the camera is the body
    T_bc: Optional[Tuple[float, ...]] = None

    @property
    def fx(self) -> float:
        return 60.0 * self.W / 64.0

    @property
    def fy(self) -> float:
        return 60.0 * self.W / 64.0

    @property
    def cx(self) -> float:
        return self.W / 2.0

    @property
    def cy(self) -> float:
        return self.H / 2.0


def config_small() -> SceneConfig:
    """8 keyframes, 48x64 maps, 3 outgoing edges each (24 edges), 4 GN iterations."""
    return SceneConfig(n_kf=8, H=48, W=64, k_out=3)


def config_window() -> SceneConfig:
    """24-keyframe sliding window, 60x80 maps, 12 outgoing edges each (288 edges)."""
    return SceneConfig(n_kf=24, H=60, W=80, k_out=12)


def config_global() -> SceneConfig:
    """512 keyframes, 60x80 maps, 11 outgoing edges each + 200 loop edges."""
    return SceneConfig(n_kf=512, H=60, W=80, k_out=11, n_loop=200)


def config_batched_window(w: int) -> SceneConfig:
    """Window ``w`` of the 64-window batch: N ~ U{8..32}, out-degree ~ U{3..8},
    map 48x64 or 60x80, IMU gaps ~ U{5..40} samples."""
    return config_random_window(4000 + w)


def config_random_window(seed: int, smooth_depth_init: bool = False) -> SceneConfig:
    """A window drawn from the batched-window distribution with its own seed
    (training windows of the warm start use seeds 100000 and up, with a smooth
    initial depth error: ``smooth_depth_init``)."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(8, 33))
    degs = [int(rng.integers(3, min(8, n - 1) + 1)) for _ in range(n)]
    if rng.random() < 0.5:
        H, W = 48, 64
    else:
        H, W = 60, 80
    return SceneConfig(n_kf=n, H=H, W=W, out_degrees=degs, gap_range=(5, 40), init_depth_smooth=smooth_depth_init)


# --------------------------------------------------------------------------
# problem container
# --------------------------------------------------------------------------
@dataclass
class Problem:
    """All arrays of one window.  Estimate arrays are the solver's initial state."""
    cfg: SceneConfig
    seed: int
    # camera
    fx: float
    fy: float
    cx: float
    cy: float
    H: int
    W: int
    gravity: np.ndarray
    # initial estimate
    pose: np.ndarray         # (N,7) float64
    vel: np.ndarray          # (N,3) float64
    bias: np.ndarray         # (N,6) float64 (bg, ba)
    invdepth: np.ndarray     # (N,H,W) float64
    # frame graph
    ii: np.ndarray           # (E,) int32 source keyframe (owns the depth)
    jj: np.ndarray           # (E,) int32 target keyframe
    target: np.ndarray       # (E,2,H,W) float32 pixel coordinates (x, y)
    weight: np.ndarray       # (E,2,H,W) float32 information weights
    target64: np.ndarray     # (E,2,H,W) float64 (exact values, for noiseless pins)
    # IMU stream, CSR over the N-1 consecutive pairs
    imu_off: np.ndarray      # (N,) int32
    gyro: np.ndarray         # (S,3) float64
    accel: np.ndarray        # (S,3) float64
    imu_dt: np.ndarray       # (S,) float64
    bias_hat: np.ndarray     # (N-1,6) float64 bias linearisation point per factor
    noise: np.ndarray        # (4,) sigma_g, sigma_a, sigma_bgw, sigma_baw
    # ground truth
    pose_gt: np.ndarray
    vel_gt: np.ndarray
    bias_gt: np.ndarray
    invdepth_gt: np.ndarray
    kf_tick: np.ndarray      # (N,) IMU tick index of each keyframe
    z_min: float = 0.1
    T_bc: Optional[np.ndarray] = None   # (7,) body-from-camera t, q xyzw; None = identity

    @property
    def n_kf(self) -> int:
        return self.pose.shape[0]

    @property
    def n_edges(self) -> int:
        return int(self.ii.shape[0])

    def copy_state(self):
        return (self.pose.copy(), self.vel.copy(), self.bias.copy(), self.invdepth.copy())


# --------------------------------------------------------------------------
# generator pieces
# --------------------------------------------------------------------------
class _Trajectory:
    """Smooth periodic motion: sinusoidal position, sinusoidal body rate."""

    def __init__(self, rng: np.random.Generator):
        T = TRAJ_PERIOD_S
        self.fp = np.array([1.0, 2.0, 3.0]) / T                    # Hz
        self.Ap = rng.uniform(0.06, 0.12, size=(3, 3))              # axis x harmonic
        self.Ap[:, 0] *= 1.6                                        # more lateral motion
        self.php = rng.uniform(0, 2 * np.pi, size=(3, 3))
        self.fw = np.array([1.0, 2.0, 3.0]) / T
        self.Aw = rng.uniform(0.08, 0.18, size=(3, 3))              # rad/s
        self.phw = rng.uniform(0, 2 * np.pi, size=(3, 3))

    def pos(self, t):
        t = np.atleast_1d(t)[:, None, None]
        return (self.Ap[None] * np.sin(2 * np.pi * self.fp[None, None] * t + self.php[None])).sum(-1)

    def vel(self, t):
        t = np.atleast_1d(t)[:, None, None]
        w = 2 * np.pi * self.fp[None, None]
        return (self.Ap[None] * w * np.cos(w * t + self.php[None])).sum(-1)

    def acc(self, t):
        t = np.atleast_1d(t)[:, None, None]
        w = 2 * np.pi * self.fp[None, None]
        return (-self.Ap[None] * w * w * np.sin(w * t + self.php[None])).sum(-1)

    def omega(self, t):
        t = np.atleast_1d(t)[:, None, None]
        return (self.Aw[None] * np.cos(2 * np.pi * self.fw[None, None] * t + self.phw[None])).sum(-1)


# camera looking along world +y, image-down along world -z
_Q0 = np.array([-np.sqrt(0.5), 0.0, 0.0, np.sqrt(0.5)])


def _edge_list(cfg: SceneConfig, rng: np.random.Generator):
    N = cfg.n_kf
    ii, jj = [], []
    for i in range(N):
        k = cfg.out_degrees[i] if cfg.out_degrees is not None else cfg.k_out
        k = min(k, N - 1)
        cand = []
        for s in range(1, N):
            for j in (i + s, i - s):          # forward neighbour first on ties
                if 0 <= j < N:
                    cand.append(j)
        for j in cand[:k]:
            ii.append(i)
            jj.append(j)
    have = set(zip(ii, jj))
    n_loop = 0
    period_kf = int(round(TRAJ_PERIOD_S * cfg.imu_rate / cfg.kf_gap)) if (cfg.gap_range is None and cfg.gaps is None) else 0
    tries = 0
    while n_loop < cfg.n_loop and tries < 100000:
        tries += 1
        i = int(rng.integers(0, N))
        if period_kf > 0:
            # near-revisits of the periodic trajectory
            m = int(rng.integers(1, max(2, N // period_kf + 1)))
            j = i + (m if rng.random() < 0.5 else -m) * period_kf + int(rng.integers(-1, 2))
        else:
            j = int(rng.integers(0, N))
        if not (0 <= j < N) or abs(i - j) < cfg.loop_gap or (i, j) in have:
            continue
        have.add((i, j))
        ii.append(i)
        jj.append(j)
        n_loop += 1
    return np.array(ii, dtype=np.int32), np.array(jj, dtype=np.int32)


def _depth_field(cfg: SceneConfig, rng: np.random.Generator) -> np.ndarray:
    H, W = cfg.H, cfg.W
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    u = np.stack([xs / W, ys / H], 0)
    acc = np.zeros((H, W))
    for _ in range(4):
        f = rng.uniform(-2.0, 2.0, size=2)
        f *= min(1.0, 2.0 / max(np.linalg.norm(f), 1e-12))
        a = rng.uniform(0.6, 1.4)
        ph = rng.uniform(0, 2 * np.pi)
        acc += a * np.cos(2 * np.pi * (f[0] * u[0] + f[1] * u[1]) + ph)
    return 0.2 + 1.8 / (1.0 + np.exp(-acc))


def _smooth_unit_field(cfg: SceneConfig, rng: np.random.Generator) -> np.ndarray:
    """Zero-mean, unit-variance smooth random field (four plane waves of at
    most two cycles per image, as the depth fields), clipped to +-3."""
    H, W = cfg.H, cfg.W
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    acc = np.zeros((H, W))
    for _ in range(4):
        f = rng.uniform(-2.0, 2.0, size=2)
        f *= min(1.0, 2.0 / max(np.linalg.norm(f), 1e-12))
        acc += rng.uniform(0.6, 1.4) * np.cos(2 * np.pi * (f[0] * xs / W + f[1] * ys / H) + rng.uniform(0, 2 * np.pi))
    acc = acc - acc.mean()
    return np.clip(acc / max(acc.std(), 1e-12), -3.0, 3.0)


def _project(cfg: SceneConfig, R_i, p_i, R_j, p_j, invdepth_i):
    """Pixel coordinates in camera j of camera i's pixels back-projected at their
    inverse depth; also the depth seen from j."""
    H, W = cfg.H, cfg.W
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    ray = np.stack([(xs - cfg.cx) / cfg.fx, (ys - cfg.cy) / cfg.fy, np.ones_like(xs)], 0)
    X_ci = ray / invdepth_i[None]
    X_w = np.einsum("ab,bhw->ahw", R_i, X_ci) + p_i[:, None, None]
    X_cj = np.einsum("ba,bhw->ahw", R_j, X_w - p_j[:, None, None])
    z = X_cj[2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = cfg.fx * X_cj[0] / z + cfg.cx
        v = cfg.fy * X_cj[1] / z + cfg.cy
    return np.stack([u, v], 0), z


def make_problem(cfg: SceneConfig, seed: int, bias_hat_mode: str = "zero") -> Problem:
    """Build one seeded window.

    ``bias_hat_mode``: ``"zero"`` linearises every IMU factor at zero bias (the
    solver's initial bias estimate), ``"gt"`` at the true bias.
    """
    rng = np.random.default_rng(seed)
    N = cfg.n_kf
    dt_imu = 1.0 / cfg.imu_rate
    if cfg.gaps is not None:
        assert len(cfg.gaps) == N - 1
        gaps = np.asarray(cfg.gaps, dtype=np.int64)
    elif cfg.gap_range is None:
        gaps = np.full(N - 1, cfg.kf_gap, dtype=np.int64)
    else:
        gaps = rng.integers(cfg.gap_range[0], cfg.gap_range[1] + 1, size=N - 1)
    kf_tick = np.concatenate([[0], np.cumsum(gaps)]).astype(np.int64)
    n_ticks = int(kf_tick[-1])

    traj = _Trajectory(rng)
    t = np.arange(n_ticks + 1) * dt_imu
    omega = traj.omega(t)                                   # body rate at ticks
    acc_w = traj.acc(t)                                     # world acceleration

    # biases: constant per keyframe interval, random walk between intervals
    bias_gt = np.zeros((N, 6))
    b0 = np.r_[rng.normal(0, cfg.bg0_std, 3), rng.normal(0, cfg.ba0_std, 3)]
    rw = np.r_[np.full(3, cfg.sigma_bgw), np.full(3, cfg.sigma_baw)]
    steps = rng.normal(size=(N, 6))
    if not cfg.zero_bias:
        bias_gt[0] = b0
        for i in range(1, N):
            Dt = gaps[i - 1] * dt_imu
            bias_gt[i] = bias_gt[i - 1] + (0.0 if cfg.noiseless else 1.0) * rw * np.sqrt(Dt) * steps[i]

    # discrete-consistent ground truth along the IMU ticks
    q = np.empty((n_ticks + 1, 4))
    v = np.empty((n_ticks + 1, 3))
    p = np.empty((n_ticks + 1, 3))
    f_body = np.empty((n_ticks, 3))                         # true specific force
    q[0] = _Q0
    v[0] = traj.vel(0.0)[0]
    p[0] = traj.pos(0.0)[0]
    dq = _quat_from_rotvec(omega[:-1] * dt_imu)
    for k in range(n_ticks):
        R = _quat_to_mat(q[k])
        f_body[k] = R.T @ (acc_w[k] - GRAVITY)
        Rf = R @ f_body[k]
        v[k + 1] = v[k] + GRAVITY * dt_imu + Rf * dt_imu
        p[k + 1] = p[k] + v[k] * dt_imu + 0.5 * GRAVITY * dt_imu ** 2 + 0.5 * Rf * dt_imu ** 2
        qn = _qmul(q[k], dq[k])
        q[k + 1] = qn / np.linalg.norm(qn)

    # IMU measurements: truth + interval bias + white noise
    interval = np.searchsorted(kf_tick, np.arange(n_ticks), side="right") - 1
    gyro = omega[:-1] + bias_gt[interval, :3]
    accel = f_body + bias_gt[interval, 3:]
    if not cfg.noiseless:
        gyro = gyro + rng.normal(0, cfg.sigma_g / np.sqrt(dt_imu), size=gyro.shape)
        accel = accel + rng.normal(0, cfg.sigma_a / np.sqrt(dt_imu), size=accel.shape)
    imu_dt = np.full(n_ticks, dt_imu)

    pose_gt = np.concatenate([p[kf_tick], q[kf_tick]], axis=1)
    vel_gt = v[kf_tick].copy()
    R_gt = _quat_to_mat(q[kf_tick])

    invdepth_gt = np.stack([_depth_field(cfg, rng) for _ in range(N)], 0)
    ii, jj = _edge_list(cfg, rng)
    E = ii.shape[0]
    H, W = cfg.H, cfg.W
    target64 = np.empty((E, 2, H, W))
    weight = np.empty((E, 2, H, W), dtype=np.float32)
    # cameras of the keyframes: T_wc = T_wb T_bc (the IMU trajectory is the body's)
    Rc_gt, pc_gt = R_gt, pose_gt[:, :3]
    if cfg.T_bc is not None:
        tb = np.asarray(cfg.T_bc, dtype=np.float64)
        R_bc = _quat_to_mat(tb[3:7] / np.linalg.norm(tb[3:7]))
        Rc_gt = R_gt @ R_bc
        pc_gt = pose_gt[:, :3] + np.einsum("nab,b->na", R_gt, tb[:3])
    for e in range(E):
        i, j = int(ii[e]), int(jj[e])
        uv, z = _project(cfg, Rc_gt[i], pc_gt[i], Rc_gt[j], pc_gt[j], invdepth_gt[i])
        ok = z > cfg.z_min
        uv = np.where(ok[None], uv, 0.0)
        target64[e] = uv
        w = rng.uniform(cfg.w_lo, cfg.w_hi, size=(2, H, W))
        weight[e] = np.where(ok[None], w, 0.0)
    if not cfg.noiseless:
        target64 = target64 + rng.normal(0, cfg.sigma_px, size=target64.shape)
    target = target64.astype(np.float32)

    # perturbed initial estimate (keyframe 0 keeps its true pose: it is the gauge)
    pose0 = pose_gt.copy()
    vel0 = vel_gt.copy()
    if N > 1:
        dth = np.deg2rad(cfg.init_dtheta_deg) * _unit(rng, N - 1)
        pose0[1:, :3] += cfg.init_dp * _unit(rng, N - 1)
        qp = _qmul(pose_gt[1:, 3:], _quat_from_rotvec(dth))
        pose0[1:, 3:] = qp / np.linalg.norm(qp, axis=1, keepdims=True)
        vel0 += rng.normal(0, cfg.init_dv_std, size=vel0.shape)
    eps = np.clip(rng.normal(size=invdepth_gt.shape), -3.0, 3.0)
    if cfg.init_depth_smooth:
        eps = np.stack([_smooth_unit_field(cfg, rng) for _ in range(N)], 0)
    invdepth0 = invdepth_gt * (1.0 + cfg.init_depth_rel * eps)
    bias0 = np.zeros((N, 6))
    if bias_hat_mode == "gt":
        bias_hat = bias_gt[:-1].copy()
    else:
        bias_hat = np.zeros((N - 1, 6))

    return Problem(
        cfg=cfg, seed=seed, fx=cfg.fx, fy=cfg.fy, cx=cfg.cx, cy=cfg.cy, H=H, W=W,
        gravity=GRAVITY.copy(),
        pose=pose0, vel=vel0, bias=bias0, invdepth=invdepth0,
        ii=ii, jj=jj, target=target, weight=weight, target64=target64,
        imu_off=kf_tick.astype(np.int32), gyro=gyro, accel=accel, imu_dt=imu_dt,
        bias_hat=bias_hat,
        noise=np.array([cfg.sigma_g, cfg.sigma_a, cfg.sigma_bgw, cfg.sigma_baw]),
        pose_gt=pose_gt, vel_gt=vel_gt, bias_gt=bias_gt, invdepth_gt=invdepth_gt,
        kf_tick=kf_tick, z_min=cfg.z_min,
        T_bc=None if cfg.T_bc is None else np.asarray(cfg.T_bc, dtype=np.float64),
    )


def tiny_config(n_kf: int = 3, H: int = 4, W: int = 5, k_out: int = 2,
                noiseless: bool = False, zero_bias: bool = False, kf_gap: int = 20) -> SceneConfig:
    """Tiny windows used for brute-force checks (finite differences, dense solves)."""
    return SceneConfig(n_kf=n_kf, H=H, W=W, k_out=k_out, noiseless=noiseless,
                       zero_bias=zero_bias, kf_gap=kf_gap)


def add_degenerate_pixels(prob: Problem, seed: int, frac_near: float = 0.06, frac_nonpos: float = 0.02,
                          frac_zero_w: float = 0.03, frac_zero_wx: float = 0.01, frac_no_info: float = 0.01) -> Problem:
    """Plant the degenerate cases of the vision term in a problem's initial
    state and weights (in place; returns the problem):
      * frac_near of every keyframe's pixels get an inverse depth in [6, 25]
        (points 4-17 cm from camera i, so most of their pixel-residuals lie
        within z_min of camera j and are not valid, some just beyond it);
      * frac_nonpos get an inverse depth of 0 or a negative one (not valid);
      * frac_zero_w of the (edge, pixel) pairs get zero weight in both
        coordinates, frac_zero_wx only in x;
      * frac_no_info of every keyframe's pixels get zero weight on all of its
        outgoing edges (no information: C = 0 before damping)."""
    rng = np.random.default_rng(seed)
    N, H, W = prob.invdepth.shape
    HW = H * W
    d = prob.invdepth.reshape(N, HW)
    for i in range(N):
        perm = rng.permutation(HW)
        n1, n2, n3 = int(frac_near * HW), int(frac_nonpos * HW), int(frac_no_info * HW)
        near, nonpos, noinfo = perm[:n1], perm[n1:n1 + n2], perm[n1 + n2:n1 + n2 + n3]
        d[i, near] = rng.uniform(6.0, 25.0, size=n1)
        d[i, nonpos] = np.where(rng.random(n2) < 0.5, 0.0, -rng.uniform(0.01, 1.0, size=n2))
        w = prob.weight[prob.ii == i].reshape(-1, 2, HW)
        w[:, :, noinfo] = 0.0
        prob.weight[prob.ii == i] = w.reshape(-1, 2, H, W)
    E = prob.n_edges
    wt = prob.weight.reshape(E, 2, HW)
    m0 = rng.random((E, HW)) < frac_zero_w
    wt[:, 0][m0] = 0.0
    wt[:, 1][m0] = 0.0
    mx = rng.random((E, HW)) < frac_zero_wx
    wt[:, 0][mx] = 0.0
    return prob


# --------------------------------------------------------------------------
# pose-graph bundle adjustment in Sim(3) (loop closure)
# --------------------------------------------------------------------------
@dataclass
class PGBAProblem:
    """Keyframes with Sim(3) poses (camera-to-world s R x + p), loop pairs with
    dense targets and weights, and relative Sim(3) measurements of the pose
    graph.  Estimate arrays are the solver's initial state."""
    fx: float
    fy: float
    cx: float
    cy: float
    H: int
    W: int
    pose: np.ndarray         # (N, 7) p, q (x, y, z, w)
    scale: np.ndarray        # (N,)
    invdepth: np.ndarray     # (N, H, W)
    ii: np.ndarray           # (E*,) int32 loop-pair sources
    jj: np.ndarray           # (E*,) int32
    target: np.ndarray       # (E*, 2, H, W) float32
    weight: np.ndarray       # (E*, 2, H, W) float32
    target64: np.ndarray     # (E*, 2, H, W) float64 (exact values, for noiseless pins)
    rel_ii: np.ndarray       # (E+,) int32
    rel_jj: np.ndarray       # (E+,) int32
    rel_meas: np.ndarray     # (E+, 8) measured relative similarity E_ij = T_j^-1 T_i: t (3), q (4), s
    rel_info: np.ndarray     # (E+, 7, 7) information in the (rotation, translation, log-scale) order
    pose_gt: np.ndarray
    scale_gt: np.ndarray
    invdepth_gt: np.ndarray

    @property
    def n_kf(self) -> int:
        return self.pose.shape[0]

    @property
    def n_edges(self) -> int:
        return int(self.ii.shape[0])


def _quat_to_mat_np(q):
    return _quat_to_mat(np.asarray(q, dtype=np.float64)[None])[0]


def _mat_to_quat(R):
    tr = np.trace(R)
    if tr > 0:
        s = 2.0 * np.sqrt(tr + 1.0)
        q = np.array([(R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s, (R[1, 0] - R[0, 1]) / s, 0.25 * s])
    else:
        k = int(np.argmax(np.diag(R)))
        i, j, m = k, (k + 1) % 3, (k + 2) % 3
        s = 2.0 * np.sqrt(1.0 + R[i, i] - R[j, j] - R[m, m])
        q = np.zeros(4)
        q[i] = 0.25 * s
        q[j] = (R[j, i] + R[i, j]) / s
        q[m] = (R[m, i] + R[i, m]) / s
        q[3] = (R[m, j] - R[j, m]) / s
    return q / np.linalg.norm(q) * (1.0 if q[3] >= 0 else -1.0)


def make_pgba_problem(cfg: SceneConfig, seed: int, loops, rel_pairs, log_scale_drift: float = 0.1,
                      noiseless: bool = False, rel_sigma=(0.005, 0.01, 0.005), init_dlogs: float = 0.05) -> PGBAProblem:
    """A loop-closure problem on the trajectory of ``make_problem(cfg, seed)``:
    the true keyframe scales drift as exp(log_scale_drift i / (N - 1)) (the
    scale drift the pose graph corrects); ``loops`` lists the loop pairs (i, j)
    whose dense targets are the true projections (+ N(0, sigma_px^2) unless
    noiseless) with weights U[w_lo, w_hi] (0 where the point is behind camera
    j); ``rel_pairs`` lists the pose-graph edges, measured as the true E_ij
    times Exp(n), n ~ N(0, diag(rel_sigma^2)) per (rotation, translation,
    log-scale) axis (none if noiseless), with information diag(rel_sigma^-2).
    Initial estimate: the true state with the rotation, position and
    inverse-depth perturbations of ``make_problem`` and log-scale errors
    U[-init_dlogs, init_dlogs], keyframe 0 held at the truth (gauge)."""
    base = make_problem(cfg, seed)
    rng = np.random.default_rng(seed + 7919)
    N, H, W = cfg.n_kf, cfg.H, cfg.W
    s_gt = np.exp(log_scale_drift * np.arange(N) / max(N - 1, 1))
    R_gt = np.stack([_quat_to_mat_np(q) for q in base.pose_gt[:, 3:]])
    p_gt = base.pose_gt[:, :3]
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    ray = np.stack([(xs - cfg.cx) / cfg.fx, (ys - cfg.cy) / cfg.fy, np.ones_like(xs)], 0)
    ii = np.array([a for a, b in loops], dtype=np.int32)
    jj = np.array([b for a, b in loops], dtype=np.int32)
    E = len(loops)
    target = np.zeros((E, 2, H, W))
    weight = np.zeros((E, 2, H, W), dtype=np.float32)
    for e, (i, j) in enumerate(loops):
        Xw = s_gt[i] * np.einsum("ab,bhw->ahw", R_gt[i], ray / base.invdepth_gt[i][None]) + p_gt[i][:, None, None]
        Xj = np.einsum("ba,bhw->ahw", R_gt[j], Xw - p_gt[j][:, None, None]) / s_gt[j]
        z = Xj[2]
        ok = z > cfg.z_min
        with np.errstate(divide="ignore", invalid="ignore"):
            uv = np.stack([cfg.fx * Xj[0] / z + cfg.cx, cfg.fy * Xj[1] / z + cfg.cy])
        target[e] = np.where(ok[None], uv, 0.0)
        weight[e] = np.where(ok[None], rng.uniform(cfg.w_lo, cfg.w_hi, size=(2, H, W)), 0.0)
    if not noiseless:
        target = target + rng.normal(0, cfg.sigma_px, size=target.shape)
    rel_ii = np.array([a for a, b in rel_pairs], dtype=np.int32)
    rel_jj = np.array([b for a, b in rel_pairs], dtype=np.int32)
    sig = np.array([rel_sigma[0]] * 3 + [rel_sigma[1]] * 3 + [rel_sigma[2]])
    rel_meas = np.zeros((len(rel_pairs), 8))
    for f, (i, j) in enumerate(rel_pairs):
        # E_ij = T_j^-1 T_i: scale s_i / s_j, rotation R_j^T R_i, translation R_j^T (p_i - p_j) / s_j
        s = s_gt[i] / s_gt[j]
        R = R_gt[j].T @ R_gt[i]
        t = R_gt[j].T @ (p_gt[i] - p_gt[j]) / s_gt[j]
        if not noiseless:
            n = rng.normal(size=7) * sig
            # right-multiply by a small similarity: rotation Exp(n_rot), translation n_t, scale e^n_s
            dR = _quat_to_mat_np(_quat_from_rotvec(n[0:3]))
            t = t + s * R @ n[3:6]
            R = R @ dR
            s = s * np.exp(n[6])
        rel_meas[f] = np.r_[t, _mat_to_quat(R), s]
    rel_info = np.tile(np.diag(1.0 / sig ** 2), (len(rel_pairs), 1, 1))
    pose0 = base.pose.copy()
    pose0[0] = base.pose_gt[0]
    s0 = s_gt * np.exp(rng.uniform(-init_dlogs, init_dlogs, size=N))
    s0[0] = s_gt[0]
    pose_gt = base.pose_gt.copy()
    return PGBAProblem(fx=cfg.fx, fy=cfg.fy, cx=cfg.cx, cy=cfg.cy, H=H, W=W, pose=pose0, scale=s0,
                       invdepth=base.invdepth.copy(), ii=ii, jj=jj, target=target.astype(np.float32),
                       weight=weight, target64=target, rel_ii=rel_ii, rel_jj=rel_jj, rel_meas=rel_meas, rel_info=rel_info,
                       pose_gt=pose_gt, scale_gt=s_gt, invdepth_gt=base.invdepth_gt.copy())


def pgba_loop_closure_problem(seed: int = 3) -> PGBAProblem:
    """Loop closure on the 512-keyframe trajectory of config_global(): 200
    near-revisit loop edges drawn by that configuration's edge generator
    (|i - j| >= loop_gap, at most 3 per source for seed 3) are the loop
    pairs E*, the relative poses
    E+ link every keyframe to its next three (1530), and the keyframe scales
    drift by 10 % along the trajectory."""
    cfg = config_global()
    ii, jj = _edge_list(cfg, np.random.default_rng(seed))
    ii, jj = np.array(ii), np.array(jj)
    far = np.abs(ii - jj) >= cfg.loop_gap
    loops = list(zip(ii[far].tolist(), jj[far].tolist()))
    rel = [(i, i + s) for s in range(1, 4) for i in range(cfg.n_kf - s)]
    return make_pgba_problem(cfg, seed, loops, rel)


# --------------------------------------------------------------------------
# Gaussian map and a loop-closure pose correction (input of the map update)
# --------------------------------------------------------------------------
@dataclass
class GaussianMap:
    """A map of K Gaussians anchored to N keyframes, with the keyframe poses
    before and after a loop-closure correction.  Means are world-frame FP32
    [K][3]; covariances are the 6 upper-triangle entries (xx, xy, xz, yy, yz,
    zz) in FP32 [K][6]; anchors are int32 [K]; poses are camera-to-world FP64
    [N][7] (t, q xyzw); scale_change is FP64 [N]."""
    mean: np.ndarray
    cov: np.ndarray
    anchor: np.ndarray
    pose_pre: np.ndarray
    pose_post: np.ndarray
    scale_change: np.ndarray


def make_gaussian_map(n_kf: int, per_kf: int, seed: int, H: int = 480, W: int = 640,
                      reorder_frac: float = 0.05, chunk: int = 1 << 20) -> GaussianMap:
    """Seeded map: keyframes on a loop of radius 2 m looking outwards; each
    keyframe unprojects ``per_kf`` pixels at inverse depths in [0.2, 2] into
    Gaussians whose axes follow the pixel footprint (a random orientation, scales
    0.5..2 pixel footprints).  Gaussians are stored in keyframe order (as they
    are created) with a fraction ``reorder_frac`` of positions permuted, as
    pruning and densification leave them.  The loop-closure correction grows
    along the trajectory: up to 3 degrees of rotation, 0.3 m of translation and a
    scale change of up to 5 %, plus small per-keyframe noise."""
    rng = np.random.default_rng(seed)
    fx = fy = 0.8 * W
    cx, cy = 0.5 * W, 0.5 * H
    ang = 2 * np.pi * np.arange(n_kf) / max(n_kf, 1)
    t_pre = np.stack([2.0 * np.cos(ang), 2.0 * np.sin(ang), 0.1 * np.sin(3 * ang)], 1)
    # camera z axis points outwards (yaw ang), small roll/pitch wobble
    yaw = _quat_from_rotvec(np.stack([np.zeros(n_kf), np.zeros(n_kf), ang], 1))
    tilt = _quat_from_rotvec(np.stack([0.5 * np.pi + 0.05 * rng.normal(size=n_kf),
                                       0.05 * rng.normal(size=n_kf), np.zeros(n_kf)], 1))
    q_pre = _qmul(yaw, _qmul(_quat_from_rotvec(np.tile([0.0, 0.5 * np.pi, 0.0], (n_kf, 1))), tilt))
    frac = np.arange(n_kf) / max(n_kf - 1, 1)
    corr_axis = _unit(rng, 1)[0]
    dq = _quat_from_rotvec(np.deg2rad(3.0) * frac[:, None] * corr_axis + 1e-3 * rng.normal(size=(n_kf, 3)))
    q_post = _qmul(dq, q_pre)
    t_post = t_pre + 0.3 * frac[:, None] * _unit(rng, 1)[0] + 0.005 * rng.normal(size=(n_kf, 3))
    scale_change = np.exp(np.log(1.05) * frac + 0.002 * rng.normal(size=n_kf))
    pose_pre = np.concatenate([t_pre, q_pre], 1)
    pose_post = np.concatenate([t_post, q_post], 1)

    K = n_kf * per_kf
    anchor = np.repeat(np.arange(n_kf, dtype=np.int32), per_kf)
    if reorder_frac > 0 and K > 1:
        pos = rng.choice(K, size=int(reorder_frac * K), replace=False)
        anchor[pos] = anchor[rng.permutation(pos)]
    mean = np.empty((K, 3), np.float32)
    cov = np.empty((K, 6), np.float32)
    Rk = _quat_to_mat(q_pre)
    for s in range(0, K, chunk):
        e = min(K, s + chunk)
        n = e - s
        a = anchor[s:e]
        u = rng.uniform(0, W, n)
        v = rng.uniform(0, H, n)
        z = 1.0 / rng.uniform(0.2, 2.0, n)
        xc = np.stack([(u - cx) / fx * z, (v - cy) / fy * z, z], 1)
        foot = z / fx
        Ra = Rk.reshape(n_kf, 9)[a]
        for r in range(3):
            mean[s:e, r] = Ra[:, 3 * r] * xc[:, 0] + Ra[:, 3 * r + 1] * xc[:, 1] + Ra[:, 3 * r + 2] * xc[:, 2] + t_pre[a, r]
        # Sigma = Q diag(sc^2) Q^T with Q the rotation of a random unit quaternion
        qv = rng.normal(size=(4, n))
        qv /= np.sqrt(np.sum(qv * qv, axis=0))
        x, y, zq, w = qv
        Q = [[1 - 2 * (y * y + zq * zq), 2 * (x * y - zq * w), 2 * (x * zq + y * w)],
             [2 * (x * y + zq * w), 1 - 2 * (x * x + zq * zq), 2 * (y * zq - x * w)],
             [2 * (x * zq - y * w), 2 * (y * zq + x * w), 1 - 2 * (x * x + y * y)]]
        var = (foot[:, None] * rng.uniform(0.5, 2.0, (n, 3))) ** 2
        for e6, (r, c) in enumerate(((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))):
            cov[s:e, e6] = Q[r][0] * Q[c][0] * var[:, 0] + Q[r][1] * Q[c][1] * var[:, 1] + Q[r][2] * Q[c][2] * var[:, 2]
    return GaussianMap(mean, cov, anchor, pose_pre, pose_post, scale_change)


# --------------------------------------------------------------------------
# inertial-only initialisation: the window as a monocular visual front end
# would see it (input of the IMU initialisation, stage 2)
# --------------------------------------------------------------------------
@dataclass
class InertialInitProblem:
    """Keyframe poses in an arbitrary visual frame at an unknown scale, the IMU
    stream between the keyframes, and the truth the initialisation should
    recover.  The visual frame w' is the gravity-aligned world frame rotated by
    R_wg (true) and shrunk by e^-s (true): p^vis = e^-s R_wg p, R^vis = R_wg R,
    v^vis = e^-s R_wg v; gravity in w' is R_wg (0, 0, -9.81)."""
    pose_vis: np.ndarray      # (N, 7) (p^vis, q xyzw)
    imu_off: np.ndarray
    gyro: np.ndarray
    accel: np.ndarray
    imu_dt: np.ndarray
    bias_hat: np.ndarray
    noise: np.ndarray
    R_wg: np.ndarray          # (3, 3) truth
    s: float                  # truth
    v_vis: np.ndarray         # (N, 3) truth
    b: np.ndarray             # (N, 6) truth


def make_inertial_init_problem(cfg: SceneConfig, seed: int, tilt_deg: float = 25.0, log_scale: float = 0.9,
                               pose_noise: Tuple[float, float] = (0.0, 0.0),
                               bias_hat_mode: str = "zero") -> InertialInitProblem:
    """Window ``cfg`` (seed ``seed``) seen by a visual front end: its frame is
    tilted by ``tilt_deg`` about a random horizontal axis (and turned by a random
    yaw), its scale is e^-log_scale; ``pose_noise`` = (position std in m,
    rotation std in degrees) of the visual poses' errors (metric, before the
    scale change)."""
    p = make_problem(cfg, seed, bias_hat_mode=bias_hat_mode)
    rng = np.random.default_rng(seed + 7919)
    axis = rng.normal(size=3)
    axis[2] = 0.0
    axis /= np.linalg.norm(axis)
    q_tilt = _quat_from_rotvec(np.deg2rad(tilt_deg) * axis)
    q_yaw = _quat_from_rotvec(np.array([0.0, 0.0, rng.uniform(-np.pi, np.pi)]))
    q_vw = _qmul(q_tilt, q_yaw)
    R_vw = _quat_to_mat(q_vw)
    N = p.pose_gt.shape[0]
    src = p.pose_gt.copy()
    src[:, :3] += pose_noise[0] * rng.normal(size=(N, 3))
    src[:, 3:7] = _qmul(src[:, 3:7], _quat_from_rotvec(np.deg2rad(pose_noise[1]) * rng.normal(size=(N, 3))))
    shrink = np.exp(-log_scale)
    pos = shrink * src[:, :3] @ R_vw.T
    quat = _qmul(np.broadcast_to(q_vw, src[:, 3:7].shape), src[:, 3:7])
    return InertialInitProblem(
        pose_vis=np.concatenate([pos, quat], 1), imu_off=p.imu_off, gyro=p.gyro, accel=p.accel,
        imu_dt=p.imu_dt, bias_hat=p.bias_hat, noise=p.noise, R_wg=R_vw, s=float(log_scale),
        v_vis=shrink * p.vel_gt @ R_vw.T, b=p.bias_gt.copy())

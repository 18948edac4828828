"""Pins of the inertial-only initialisation oracle (IMU initialisation stage 2):
finite differences, exact recovery of gravity direction, scale, velocities and
biases on noiseless data seen from a tilted and rescaled visual frame,
stationarity on noisy data, and the invariance of the cost to a rotation about
gravity."""
import numpy as np
import pytest

from oracle import inertial_init as oi
from oracle import preint
from oracle.so3 import Exp, quat_to_R
from paper_2512_02293_amd import synth

G_I = np.array([0.0, 0.0, -9.81])


def _setup(n_kf=12, seed=3, noiseless=False, mode="zero", pose_noise=(0.0, 0.0)):
    ip = synth.make_inertial_init_problem(synth.tiny_config(n_kf=n_kf, noiseless=noiseless), seed,
                                          bias_hat_mode=mode, pose_noise=pose_noise)
    fs = preint.preintegrate_all(ip.imu_off, ip.gyro, ip.accel, ip.imu_dt, ip.bias_hat, ip.noise)
    R = np.stack([quat_to_R(q) for q in ip.pose_vis[:, 3:7]])
    return ip, fs, R


def _zero_state(N):
    return oi.InitState(np.eye(3), 0.0, np.zeros((N, 3)), np.zeros((N, 6)))


def test_jacobian_matches_finite_differences():
    ip, fs, R = _setup()
    rng = np.random.default_rng(0)
    N = len(R)
    st = oi.InitState(ip.R_wg @ Exp(rng.normal(0, 0.05, 3)), ip.s + 0.1, ip.v_vis + rng.normal(0, 0.02, (N, 3)),
                      ip.b + rng.normal(0, [0.002] * 3 + [0.05] * 3, (N, 6)))
    r0, J, _ = oi.linearize(R, ip.pose_vis[:, :3], st, fs, G_I)
    h = 1e-6
    for c in range(J.shape[1]):
        d = np.zeros(J.shape[1])
        d[c] = h
        rp, _, _ = oi.linearize(R, ip.pose_vis[:, :3], oi.retract(st, d), fs, G_I)
        rm, _, _ = oi.linearize(R, ip.pose_vis[:, :3], oi.retract(st, -d), fs, G_I)
        fd = (rp - rm) / (2 * h)
        assert np.allclose(J[:, c], fd, rtol=1e-5, atol=1e-5 * max(1.0, np.abs(fd).max())), c


def test_noiseless_recovery_of_gravity_scale_velocity_and_bias():
    """Noiseless IMU, bias linearised at the truth, exact visual poses in a frame
    tilted by 25 degrees and shrunk by e^-0.9: from R_wg = I, s = 0, v = b = 0
    the iteration reaches the truth."""
    ip, fs, R = _setup(n_kf=16, noiseless=True, mode="gt")
    assert np.abs(ip.b).max() > 1e-3
    st, costs = oi.solve(R, ip.pose_vis[:, :3], _zero_state(len(R)), fs, G_I, iters=10)
    g_err = np.linalg.norm(np.cross(st.R_wg @ G_I, ip.R_wg @ G_I)) / (G_I @ G_I)   # sine of the angle
    assert g_err < 1e-10
    assert abs(st.s - ip.s) < 1e-10
    np.testing.assert_allclose(st.v_vis, ip.v_vis, atol=1e-10)
    np.testing.assert_allclose(st.b, ip.b, atol=1e-10)
    assert costs[-1] < 1e-18 * costs[0]


def test_noisy_problem_reaches_a_stationary_point():
    ip, fs, R = _setup(n_kf=16, seed=5, pose_noise=(2e-4, 0.01))
    st, costs = oi.solve(R, ip.pose_vis[:, :3], _zero_state(len(R)), fs, G_I, iters=15)
    _, rep0 = oi.step(R, ip.pose_vis[:, :3], _zero_state(len(R)), fs, G_I)
    _, rep = oi.step(R, ip.pose_vis[:, :3], st, fs, G_I)
    assert np.abs(rep["grad"]).max() < 1e-9 * np.abs(rep0["grad"]).max()
    assert costs[-1] < costs[0]


def test_cost_is_invariant_to_a_rotation_about_gravity():
    ip, fs, R = _setup()
    st = oi.InitState(ip.R_wg @ Exp([0.02, -0.01, 0.0]), 0.5, ip.v_vis * 1.1, ip.b * 0.9)
    c0 = oi.cost(R, ip.pose_vis[:, :3], st, fs, G_I)
    turned = st.copy()
    turned.R_wg = st.R_wg @ Exp([0.0, 0.0, 0.7])
    assert oi.cost(R, ip.pose_vis[:, :3], turned, fs, G_I) == pytest.approx(c0, rel=1e-12)
    tilted = st.copy()
    tilted.R_wg = st.R_wg @ Exp([0.01, 0.0, 0.0])
    assert abs(oi.cost(R, ip.pose_vis[:, :3], tilted, fs, G_I) - c0) > 1e-6 * c0

"""Pins of the new-keyframe prediction oracle (preintegration-based pose
initialisation with the covariance-trace fallback): the simulator's ground
truth, the Eq. 3 residual of oracle.imu, re-preintegration at a moved bias, and
the fallback rule."""
import dataclasses

import numpy as np
import pytest

from oracle import imu, predict, preint
from oracle.so3 import Log, quat_to_R
from paper_2512_02293_amd import synth


def _noiseless(gap_range=None, n_kf=6, seed=1):
    cfg = dataclasses.replace(synth.tiny_config(n_kf=n_kf, noiseless=True), gap_range=gap_range)
    return synth.make_problem(cfg, seed, bias_hat_mode="gt")


def _factors(p):
    return preint.preintegrate_all(p.imu_off, p.gyro, p.accel, p.imu_dt, p.bias_hat, p.noise)


def test_prediction_reproduces_ground_truth_on_noiseless_data():
    """The simulator integrates the true rates exactly as the preintegration
    does, so predicting keyframe f+1 from the true state of f returns its true
    state (an independent route: the generator's own integration)."""
    p = _noiseless()
    assert np.abs(p.bias_gt).max() > 1e-3
    for f, P in enumerate(_factors(p)):
        pose, v, b, used = predict.predict_pose7(p.pose_gt[f], p.vel_gt[f], p.bias_gt[f], P, p.gravity, tau=np.inf)
        assert used
        R_err = np.linalg.norm(Log(quat_to_R(pose[3:7]).T @ quat_to_R(p.pose_gt[f + 1, 3:7])))
        assert R_err < 1e-12
        np.testing.assert_allclose(pose[:3], p.pose_gt[f + 1, :3], atol=1e-12)
        np.testing.assert_allclose(v, p.vel_gt[f + 1], atol=1e-12)
        np.testing.assert_array_equal(b, p.bias_gt[f])


def test_prediction_zeroes_the_inertial_residual():
    """On noisy data with the bias linearised at zero and the previous state
    off the truth, the predicted state still zeroes Eq. 3's residual."""
    p = synth.make_problem(synth.config_small(), 5)
    for f, P in enumerate(_factors(p)):
        Ri = quat_to_R(p.pose[f, 3:7])
        bi = p.bias[f] + np.array([0.003, -0.002, 0.001, 0.03, -0.02, 0.04])
        Rj, pj, vj, bj, used = predict.predict(Ri, p.pose[f, :3], p.vel[f], bi, P, p.gravity, tau=np.inf)
        r = imu.residual(Ri, p.pose[f, :3], p.vel[f], bi, Rj, pj, vj, bj, P, p.gravity)
        assert np.abs(r).max() < 1e-12, np.abs(r).max()


def test_bias_correction_converges_to_re_preintegration():
    """Predicting with b_i = b_hat + delta equals, to second order in delta,
    predicting with the factor preintegrated at b_hat + delta."""
    p = synth.make_problem(synth.config_small(), 7)
    s0, s1 = int(p.imu_off[0]), int(p.imu_off[1])
    sg, sa, sbg, sba = p.noise
    P = preint.preintegrate(p.gyro[s0:s1], p.accel[s0:s1], p.imu_dt[s0:s1], p.bias_hat[0], sg, sa, sbg, sba)
    Ri, pi, vi = quat_to_R(p.pose[0, 3:7]), p.pose[0, :3], p.vel[0]
    d0 = np.array([0.01, -0.02, 0.015, 0.2, -0.1, 0.15])
    errs = []
    for s in (1.0, 0.5, 0.25):
        b = p.bias_hat[0] + s * d0
        lin = predict.predict(Ri, pi, vi, b, P, p.gravity, tau=np.inf)
        Pb = preint.preintegrate(p.gyro[s0:s1], p.accel[s0:s1], p.imu_dt[s0:s1], b, sg, sa, sbg, sba)
        ref = predict.predict(Ri, pi, vi, b, Pb, p.gravity, tau=np.inf)
        errs.append(max(np.linalg.norm(Log(lin[0].T @ ref[0])), np.linalg.norm(lin[1] - ref[1]),
                        np.linalg.norm(lin[2] - ref[2])))
    assert errs[0] > 1e-9
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0, errs


def test_fallback_copies_the_previous_state_and_the_threshold_is_strict():
    """Long gaps (paper-like: up to 3 s at 200 Hz) push tr(Sigma^iner) past
    1e-4; the new keyframe then takes the previous keyframe's state."""
    cfg = dataclasses.replace(synth.tiny_config(n_kf=8), gap_range=(20, 600))
    p = synth.make_problem(cfg, 3)
    fs = _factors(p)
    traces = np.array([predict.inertial_cov_trace(P) for P in fs])
    gaps = np.diff(p.imu_off)
    used = []
    for f, P in enumerate(fs):
        pose, v, b, u = predict.predict_pose7(p.pose[f], p.vel[f], p.bias[f], P, p.gravity)
        used.append(u)
        if not u:
            np.testing.assert_array_equal(pose, p.pose[f])
            np.testing.assert_array_equal(v, p.vel[f])
            np.testing.assert_array_equal(b, p.bias[f])
    used = np.array(used)
    assert used.any() and (~used).any(), (traces, gaps)
    np.testing.assert_array_equal(used, traces <= predict.TAU_INIT)
    # the trace grows with the gap
    order = np.argsort(gaps)
    assert np.all(np.diff(traces[order]) > 0)
    # strict: a trace equal to tau still uses the IMU
    f = int(np.flatnonzero(used)[0])
    assert predict.predict_pose7(p.pose[f], p.vel[f], p.bias[f], fs[f], p.gravity, tau=traces[f])[3]
    assert not predict.predict_pose7(p.pose[f], p.vel[f], p.bias[f], fs[f], p.gravity,
                                     tau=np.nextafter(traces[f], 0))[3]


def test_trace_is_the_sum_of_the_variances():
    p = _noiseless(n_kf=3)
    P = _factors(p)[0]
    full = np.zeros((15, 15))
    full[:9, :9] = P.cov
    full[9:, 9:] = np.diag(P.cov_bias)
    assert predict.inertial_cov_trace(P) == pytest.approx(np.trace(full), rel=1e-15)
    # and equals the sum of the eigenvalues of the inverse of the factor's information
    lam = imu.information(P)
    assert predict.inertial_cov_trace(P) == pytest.approx(np.sum(1.0 / np.linalg.eigvalsh(lam)), rel=1e-8)

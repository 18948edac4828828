"""Initial state of a new keyframe from IMU preintegration, with the
covariance-trace fallback (Sec. 3.1, "Frontend Tracking: Local Bundle
Adjustment", and the implementation details of the experiments section:
tau = 1e-4).

TEST INFRASTRUCTURE ONLY (see the package header).

Given the state (R_i, p_i, v_i, b_i) of the last keyframe and the factor
preintegrated from it to the new keyframe j, the prediction is the state that
makes the inertial residual of Eq. 3 vanish: the deltas are first corrected to
the bias b_i to first order (as in Eq. 3), then
    R_j = R_i dR~,  v_j = v_i + g dt + R_i dv~,  p_j = p_i + v_i dt + g dt^2 / 2 + R_i dp~,
    b_j = b_i.
When the trace of the factor's covariance Sigma^iner (the 9x9 preintegration
covariance and the 6 bias random-walk variances, blkdiag as in Eq. 3's
information) exceeds tau, the new keyframe takes the previous keyframe's state
instead; a trace that is not a number counts as exceeding it.

Pinned by (tests/test_oracle_predict.py): on noiseless, discrete-consistent
data it reproduces the simulator's ground-truth state of keyframe j; the
predicted state zeroes the Eq. 3 residual of oracle.imu; the first-order bias
correction converges quadratically to re-preintegration at the new bias; the
fallback copies the previous state exactly, with the threshold strict.
"""
import numpy as np

from .so3 import Exp, R_to_quat, quat_to_R

TAU_INIT = 1e-4


def inertial_cov_trace(P):
    """tr(Sigma^iner) of one preintegrated factor."""
    return float(np.trace(P.cov) + np.sum(P.cov_bias))


def predict(Ri, pi, vi, bi, P, g, tau=TAU_INIT):
    """-> (R_j, p_j, v_j, b_j, used_imu)."""
    Ri, pi, vi, bi = (np.asarray(a, dtype=np.float64) for a in (Ri, pi, vi, bi))
    if not inertial_cov_trace(P) <= tau:
        return Ri.copy(), pi.copy(), vi.copy(), bi.copy(), False
    db = bi - P.bias_hat
    dR = P.dR @ Exp(P.J_rot @ db[:3])
    dv = P.dv + P.J_vel @ db
    dp = P.dp + P.J_pos @ db
    dt = P.dt
    Rj = Ri @ dR
    vj = vi + g * dt + Ri @ dv
    pj = pi + vi * dt + 0.5 * g * dt * dt + Ri @ dp
    return Rj, pj, vj, bi.copy(), True


def predict_pose7(pose_i, vel_i, bias_i, P, g, tau=TAU_INIT):
    """The same with poses stored as (p, q xyzw): -> (pose_j, vel_j, bias_j, used_imu)."""
    pose_i = np.asarray(pose_i, dtype=np.float64)
    Rj, pj, vj, bj, used = predict(quat_to_R(pose_i[3:7]), pose_i[:3], vel_i, bias_i, P, g, tau)
    if not used:
        return pose_i.copy(), np.asarray(vel_i, np.float64).copy(), np.asarray(bias_i, np.float64).copy(), False
    return np.concatenate([pj, R_to_quat(Rj)]), vj, bj, True

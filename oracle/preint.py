"""IMU preintegration between two keyframes (Sec. 3.1, "Inertial Residual").

The paper preintegrates following Forster et al. and lists the outputs: the
relative rotation, velocity and position, their bias Jacobians (J^rot, J^vel,
J^pos) and the covariance Sigma^iner.  It gives no discretisation, so this
oracle takes Forster's zero-order-hold (Euler) recursion, one step per IMU
sample, with white-noise covariance sigma^2/dt per sample; see the reading list
in the design notes.

Test infrastructure (see the package header).  Pinned by: constant-acceleration
and constant-rate closed forms (exact), the discrete geometric-series closed
form for constant rate and acceleration, first-order convergence to the
continuous closed form, bias Jacobians against finite differences of
re-preintegration, and the covariance against a Monte-Carlo sample covariance.
"""
from dataclasses import dataclass

import numpy as np

from .so3 import Exp, Jr, hat

I3 = np.eye(3)


@dataclass
class Preintegrated:
    dt: float                 # total time Delta t_ij
    dR: np.ndarray            # (3,3)
    dv: np.ndarray            # (3,)
    dp: np.ndarray            # (3,)
    J_rot: np.ndarray         # (3,3)  d(dR)/d(b_g), right-perturbation form
    J_vel: np.ndarray         # (3,6)  d(dv)/d(b_g, b_a)
    J_pos: np.ndarray         # (3,6)  d(dp)/d(b_g, b_a)
    cov: np.ndarray           # (9,9)  residual order (rot, pos, vel)
    bias_hat: np.ndarray      # (6,)   linearisation point (b_g, b_a)
    cov_bias: np.ndarray      # (6,)   bias random-walk variance over Delta t_ij


def preintegrate(gyro, accel, dt, bias_hat, sigma_g, sigma_a, sigma_bgw, sigma_baw):
    """Preintegrate samples ``gyro[k], accel[k]`` held for ``dt[k]`` seconds.

    Recursion per sample, with w = gyro - b_g, a = accel - b_a, h = dt and
    dRk = Exp(w h); every right-hand side uses the values before this sample:
        dp    += dv h + 1/2 dR a h^2
        dv    += dR a h
        Jp_a  += Jv_a h - 1/2 dR h^2        Jp_g += Jv_g h - 1/2 dR [a]x J^rot h^2
        Jv_a  -= dR h                       Jv_g -= dR [a]x J^rot h
        Sigma  = A Sigma A^T + Bg (sg^2/h) Bg^T + Ba (sa^2/h) Ba^T
        J^rot  = dRk^T J^rot - Jr(w h) h
        dR     = dR dRk
    The covariance is propagated in (rot, vel, pos) order and permuted to the
    residual order (rot, pos, vel) of Eq. 3 on output.
    """
    gyro = np.asarray(gyro, dtype=np.float64)
    accel = np.asarray(accel, dtype=np.float64)
    dt = np.asarray(dt, dtype=np.float64)
    bias_hat = np.asarray(bias_hat, dtype=np.float64)
    bg, ba = bias_hat[:3], bias_hat[3:]
    dR = I3.copy()
    dv = np.zeros(3)
    dp = np.zeros(3)
    JR = np.zeros((3, 3))
    Jv_g = np.zeros((3, 3))
    Jv_a = np.zeros((3, 3))
    Jp_g = np.zeros((3, 3))
    Jp_a = np.zeros((3, 3))
    cov = np.zeros((9, 9))          # (rot, vel, pos)
    for k in range(gyro.shape[0]):
        h = dt[k]
        w = gyro[k] - bg
        a = accel[k] - ba
        dRk = Exp(w * h)
        ax = hat(a)
        # covariance transition, built from the values before the update
        A = np.eye(9)
        A[0:3, 0:3] = dRk.T
        A[3:6, 0:3] = -dR @ ax * h
        A[6:9, 0:3] = -0.5 * dR @ ax * h * h
        A[6:9, 3:6] = I3 * h
        Bg = np.zeros((9, 3))
        Bg[0:3] = Jr(w * h) * h
        Ba = np.zeros((9, 3))
        Ba[3:6] = dR * h
        Ba[6:9] = 0.5 * dR * h * h
        cov = A @ cov @ A.T + (sigma_g ** 2 / h) * (Bg @ Bg.T) + (sigma_a ** 2 / h) * (Ba @ Ba.T)
        # bias Jacobians (old dv-Jacobians feed the position ones)
        Jp_a = Jp_a + Jv_a * h - 0.5 * dR * h * h
        Jp_g = Jp_g + Jv_g * h - 0.5 * dR @ ax @ JR * h * h
        Jv_a = Jv_a - dR * h
        Jv_g = Jv_g - dR @ ax @ JR * h
        # mean
        dp = dp + dv * h + 0.5 * dR @ a * h * h
        dv = dv + dR @ a * h
        JR = dRk.T @ JR - Jr(w * h) * h
        dR = dR @ dRk
    Dt = float(dt.sum())
    perm = np.r_[0:3, 6:9, 3:6]        # (rot, vel, pos) -> (rot, pos, vel)
    cov_out = cov[np.ix_(perm, perm)]
    cov_bias = np.r_[np.full(3, sigma_bgw ** 2 * Dt), np.full(3, sigma_baw ** 2 * Dt)]
    return Preintegrated(dt=Dt, dR=dR, dv=dv, dp=dp, J_rot=JR,
                         J_vel=np.hstack([Jv_g, Jv_a]), J_pos=np.hstack([Jp_g, Jp_a]),
                         cov=cov_out, bias_hat=bias_hat.copy(), cov_bias=cov_bias)


def preintegrate_all(off, gyro, accel, dt, bias_hat, noise):
    """One factor per consecutive keyframe pair; samples of factor f are
    ``off[f] : off[f+1]`` (CSR)."""
    sg, sa, sbg, sba = (float(x) for x in noise)
    out = []
    for f in range(len(off) - 1):
        s0, s1 = int(off[f]), int(off[f + 1])
        out.append(preintegrate(gyro[s0:s1], accel[s0:s1], dt[s0:s1], bias_hat[f], sg, sa, sbg, sba))
    return out

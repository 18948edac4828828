"""Inertial residual of Eq. 3 (Sec. 3.1) and its Jacobian.

For a consecutive keyframe pair (i, j=i+1) with preintegrated factor P and
b = (b_g, b_a):
    r_rot  = Log( (dR Exp(J^rot (b_g,i - bh_g)))^T R_i^T R_j )
    r_pos  = R_i^T (p_j - p_i - v_i dt - 1/2 g dt^2) - (dp + J^pos (b_i - bh))
    r_vel  = R_i^T (v_j - v_i - g dt)                - (dv + J^vel (b_i - bh))
    r_bias = b_j - b_i
Readings (the paper is loose here): the velocity term uses the full 6-vector
bias like the position term (the printed form shows only b_g, but dv depends on
b_a); the factor uses the bias of the earlier keyframe i; the information is
the inverse of blkdiag(Sigma_preint, diag(cov_bias)).

The tangent of one keyframe is (dtheta, dp, dv, db_g, db_a) with the
right-perturbation R <- R Exp(dtheta) and additive world-frame p, v, b.

Test infrastructure (see the package header).  Pinned by: zero residual at
discrete-consistent ground truth, and the Jacobian against central finite
differences through the same retraction.
"""
import numpy as np

from .so3 import Exp, Log, Jr, Jr_inv, hat

I3 = np.eye(3)


def residual(Ri, pi, vi, bi, Rj, pj, vj, bj, P, g):
    """15-vector (rot, pos, vel, bias)."""
    dbg = bi[:3] - P.bias_hat[:3]
    db = bi - P.bias_hat
    dt = P.dt
    dR_corr = P.dR @ Exp(P.J_rot @ dbg)
    r_rot = Log(dR_corr.T @ Ri.T @ Rj)
    r_pos = Ri.T @ (pj - pi - vi * dt - 0.5 * g * dt * dt) - (P.dp + P.J_pos @ db)
    r_vel = Ri.T @ (vj - vi - g * dt) - (P.dv + P.J_vel @ db)
    r_bias = bj - bi
    return np.concatenate([r_rot, r_pos, r_vel, r_bias])


def jacobian(Ri, pi, vi, bi, Rj, pj, vj, bj, P, g):
    """15x30 Jacobian of ``residual`` with respect to (tangent_i, tangent_j)."""
    dt = P.dt
    dbg = bi[:3] - P.bias_hat[:3]
    r = residual(Ri, pi, vi, bi, Rj, pj, vj, bj, P, g)
    r_rot = r[0:3]
    Jri = Jr_inv(r_rot)
    J = np.zeros((15, 30))
    # rows 0:3 rotation
    J[0:3, 0:3] = -Jri @ Rj.T @ Ri
    J[0:3, 9:12] = -Jri @ Exp(r_rot).T @ Jr(P.J_rot @ dbg) @ P.J_rot
    J[0:3, 15:18] = Jri
    # rows 3:6 position
    y_p = pj - pi - vi * dt - 0.5 * g * dt * dt
    J[3:6, 0:3] = hat(Ri.T @ y_p)
    J[3:6, 3:6] = -Ri.T
    J[3:6, 6:9] = -Ri.T * dt
    J[3:6, 9:15] = -P.J_pos
    J[3:6, 18:21] = Ri.T
    # rows 6:9 velocity
    y_v = vj - vi - g * dt
    J[6:9, 0:3] = hat(Ri.T @ y_v)
    J[6:9, 6:9] = -Ri.T
    J[6:9, 9:15] = -P.J_vel
    J[6:9, 21:24] = Ri.T
    # rows 9:15 bias random walk
    J[9:15, 9:15] = -np.eye(6)
    J[9:15, 24:30] = np.eye(6)
    return J


def information(P):
    """Lambda = (Sigma^iner)^-1 with Sigma^iner = blkdiag(cov (9x9), diag(cov_bias))."""
    S = np.zeros((15, 15))
    S[0:9, 0:9] = P.cov
    S[9:15, 9:15] = np.diag(P.cov_bias)
    return np.linalg.inv(S)

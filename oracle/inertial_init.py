"""IMU initialisation, stage 2: inertial-only optimisation (Sec. 3.2, "Stage 2:
Inertial-Only Optimization", and the IMU-initialisation paragraph of the
implementation details).

TEST INFRASTRUCTURE ONLY (see the package header).

The visual poses T_i^vis = (R_i, p_i^vis) of the first keyframes are known up
to one global scale and are held fixed.  Positions and velocities are written
as p_i = e^s p_i^vis and v_i = e^s v_i^vis with a global log-scale s; gravity is
g = R_wg g_I with g_I = (0, 0, G).  The unknowns are the gravity direction
R_wg, s, every v_i^vis and every bias b_i; the objective is the inertial energy
of Eq. 2 (the residual of Eq. 3 with the substitutions above, weighted by the
factor information).  R_wg is perturbed on the right about the first two axes
of the gravity frame only (a rotation about g_I leaves g unchanged).

The step is the damped Gauss-Newton step of that objective, written out in
full: the stacked Jacobian J (15 rows per factor, 3 + 9 N columns ordered
(phi_x, phi_y, s, then (v^vis_i, b_i) per keyframe)), H = J^T Lambda J with
the Marquardt damping H_rr += lambda H_rr, and Delta = solve(H, -J^T Lambda r)
by numpy.linalg.solve; then R_wg <- R_wg Exp((Delta_phi, 0)), s, v^vis, b +=.
The Jacobian is the chain rule through Eq. 3's own Jacobian (oracle.imu) and
the substitutions.

Pinned by (tests/test_oracle_inertial_init.py): the Jacobian against central
finite differences through the same retraction; on noiseless,
discrete-consistent data seen from a tilted, rescaled visual frame, the
iteration recovers the gravity direction, the scale, the velocities and the
biases; on noisy data it reaches a stationary point (gradient -> 0).
"""
from dataclasses import dataclass

import numpy as np

from . import imu
from .so3 import Exp, hat


@dataclass
class InitState:
    R_wg: np.ndarray    # (3, 3)
    s: float            # log-scale
    v_vis: np.ndarray   # (N, 3) velocities in the visual scale
    b: np.ndarray       # (N, 6) (b_g, b_a)

    def copy(self):
        return InitState(self.R_wg.copy(), float(self.s), self.v_vis.copy(), self.b.copy())


def n_unknowns(N):
    return 3 + 9 * N


def _factor(R, p_vis, st, f, P, g_I):
    """Residual (15) and its Jacobian (15 x (3 + 18): globals, keyframe f, keyframe f+1)."""
    i, j = f, f + 1
    es = np.exp(st.s)
    g = st.R_wg @ g_I
    args = (R[i], es * p_vis[i], es * st.v_vis[i], st.b[i], R[j], es * p_vis[j], es * st.v_vis[j], st.b[j], P, g)
    r = imu.residual(*args)
    Jm = imu.jacobian(*args)        # 15 x 30 w.r.t. (dtheta, dp, dv, db) of keyframes i and j (metric)
    J = np.zeros((15, 21))
    # gravity: r_p holds -R_i^T g dt^2 / 2 and r_v holds -R_i^T g dt; dg/dphi = -R_wg [g_I]x (first two columns)
    dg_dphi = -(st.R_wg @ hat(g_I))[:, :2]
    dr_dg = np.zeros((15, 3))
    dr_dg[3:6] = -0.5 * P.dt ** 2 * R[i].T
    dr_dg[6:9] = -P.dt * R[i].T
    J[:, 0:2] = dr_dg @ dg_dphi
    # log-scale: d(e^s x)/ds = e^s x for the positions and velocities of both keyframes
    J[:, 2] = (Jm[:, 3:6] @ (es * p_vis[i]) + Jm[:, 6:9] @ (es * st.v_vis[i])
               + Jm[:, 18:21] @ (es * p_vis[j]) + Jm[:, 21:24] @ (es * st.v_vis[j]))
    J[:, 3:6] = es * Jm[:, 6:9]          # v^vis_i
    J[:, 6:12] = Jm[:, 9:15]             # b_i
    J[:, 12:15] = es * Jm[:, 21:24]      # v^vis_j
    J[:, 15:21] = Jm[:, 24:30]           # b_j
    return r, J


def linearize(R, p_vis, st, factors, g_I):
    """Stacked residual (15 F), Jacobian (15 F x (3 + 9 N)) and block-diagonal information."""
    N = len(R)
    F = len(factors)
    r = np.zeros(15 * F)
    J = np.zeros((15 * F, n_unknowns(N)))
    L = np.zeros((15 * F, 15 * F))
    for f, P in enumerate(factors):
        rf, Jf = _factor(R, p_vis, st, f, P, g_I)
        rows = slice(15 * f, 15 * f + 15)
        r[rows] = rf
        J[rows, 0:3] = Jf[:, 0:3]
        J[rows, 3 + 9 * f:3 + 9 * f + 9] = Jf[:, 3:12]
        J[rows, 3 + 9 * (f + 1):3 + 9 * (f + 1) + 9] = Jf[:, 12:21]
        L[rows, rows] = imu.information(P)
    return r, J, L


def cost(R, p_vis, st, factors, g_I):
    r, _, L = linearize(R, p_vis, st, factors, g_I)
    return float(r @ L @ r)


def retract(st, delta):
    N = len(st.v_vis)
    out = st.copy()
    out.R_wg = st.R_wg @ Exp(np.array([delta[0], delta[1], 0.0]))
    out.s = st.s + delta[2]
    blk = delta[3:].reshape(N, 9)
    out.v_vis = st.v_vis + blk[:, 0:3]
    out.b = st.b + blk[:, 3:9]
    return out


def step(R, p_vis, st, factors, g_I, lm_lambda=0.0):
    """One damped Gauss-Newton step -> (new state, report)."""
    r, J, L = linearize(R, p_vis, st, factors, g_I)
    H = J.T @ L @ J
    g = -J.T @ L @ r
    H[np.diag_indices_from(H)] *= 1.0 + lm_lambda
    delta = np.linalg.solve(H, g)
    return retract(st, delta), {"delta": delta, "cost_before": float(r @ L @ r), "grad": g}


def solve(R, p_vis, st, factors, g_I, iters, lm_lambda=0.0):
    """`iters` steps; returns the final state and the cost before each step and
    at the end (iters + 1 values)."""
    costs = []
    for _ in range(iters):
        st, rep = step(R, p_vis, st, factors, g_I, lm_lambda)
        costs.append(rep["cost_before"])
    costs.append(cost(R, p_vis, st, factors, g_I))
    return st, costs

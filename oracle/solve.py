"""One damped Gauss-Newton step of the joint visual-inertial problem and its
iteration (Sec. 3.1, Eq. 1-4).

A step linearises every residual at the current state, assembles and
eliminates the normal equations (Eq. 4), solves the reduced system by
Cholesky and retracts:
    R <- R Exp(dtheta),  p, v, b <- p, v, b + (dp, dv, db),
    d <- max(d + dd, d_min)          (keeps inverse depth positive).
The cost reported before and after a step is
    F = sum_vision w r^2 + sum_imu r^T Lambda r     (no 1/2 factor).

Test infrastructure (see the package header).  Pinned by: convergence to the
ground truth (F -> 0) on noiseless problems with pure Gauss-Newton, the dense
full solve, and a gauge-invariance check (a global yaw and translation of the
problem transforms the increments accordingly).
"""
import numpy as np

from . import imu as imu_mod
from . import preint, vision
from .normal_eq import (Camera, Graph, Options, State, fold_global_bias, linearize, schur_solve,
                        active_mask, NotPositiveDefinite)  # noqa: F401
from .so3 import Exp, quat_to_R, R_to_quat


def state_from_arrays(pose, vel, bias, invdepth):
    R = np.stack([quat_to_R(q) for q in np.asarray(pose)[:, 3:7]])
    return State(R=R, p=np.array(pose[:, 0:3], dtype=np.float64),
                 v=np.array(vel, dtype=np.float64), b=np.array(bias, dtype=np.float64),
                 d=np.array(invdepth, dtype=np.float64))


def pose_array(state):
    return np.concatenate([state.p, np.stack([R_to_quat(R) for R in state.R])], axis=1)


def from_problem(prob, exact_targets=False):
    """Camera, state, graph and options from a synthetic problem's arrays.
    ``exact_targets`` uses the float64 targets (noiseless pins) instead of the
    float32 ones every solver receives."""
    T_bc = None
    if getattr(prob, "T_bc", None) is not None:
        t = np.asarray(prob.T_bc, dtype=np.float64)
        T_bc = (quat_to_R(t[3:7] / np.linalg.norm(t[3:7])), t[:3].copy())
    cam = Camera(prob.fx, prob.fy, prob.cx, prob.cy, prob.H, prob.W,
                 np.asarray(prob.gravity, dtype=np.float64), T_bc)
    st = state_from_arrays(prob.pose, prob.vel, prob.bias, prob.invdepth)
    tgt = prob.target64 if exact_targets else prob.target.astype(np.float64)
    factors = preint.preintegrate_all(prob.imu_off, prob.gyro, prob.accel, prob.imu_dt,
                                      prob.bias_hat, prob.noise)
    gr = Graph(ii=np.asarray(prob.ii), jj=np.asarray(prob.jj), target=tgt,
               weight=prob.weight.astype(np.float64), factors=factors)
    return cam, st, gr


def cost(cam, state, graph, opts):
    """F at ``state`` and the number of valid pixel-residuals."""
    F = 0.0
    n_valid = 0
    for e in range(len(graph.ii)):
        i, j = int(graph.ii[e]), int(graph.jj[e])
        r, valid = vision.edge_residual_body(cam.intr, cam.T_bc, state.R[i], state.p[i], state.R[j], state.p[j],
                                             state.d[i], graph.target[e], opts.z_min)
        w = np.asarray(graph.weight[e], np.float64).reshape(2, -1)
        F += float((np.where(valid[None], w, 0.0) * r * r).sum())
        n_valid += int(valid.sum())
    if opts.use_imu:
        for f, P in enumerate(graph.factors):
            i, j = f, f + 1
            r = imu_mod.residual(state.R[i], state.p[i], state.v[i], state.b[i],
                                 state.R[j], state.p[j], state.v[j], state.b[j], P, cam.gravity)
            F += float(r @ imu_mod.information(P) @ r)
    return F, n_valid


def retract(state, dxi, dd, d_min):
    N = state.R.shape[0]
    R = np.stack([state.R[k] @ Exp(dxi[k, 0:3]) for k in range(N)])
    d = np.maximum(state.d + dd.reshape(state.d.shape), d_min)
    return State(R=R, p=state.p + dxi[:, 3:6], v=state.v + dxi[:, 6:9],
                 b=state.b + dxi[:, 9:15], d=d)


def step(cam, state, graph, opts):
    """One damped Gauss-Newton step.  Returns (new_state, report)."""
    neq = linearize(cam, state, graph, opts)
    N = state.R.shape[0]
    if opts.bias_global and opts.use_imu and not opts.bias_fixed:
        neq = fold_global_bias(neq, N)
    dxi, dd = schur_solve(neq, opts, N)
    if opts.bias_global and opts.use_imu and not opts.bias_fixed:
        dxi[:, 9:15] = dxi[N - 1, 9:15]
    new = retract(state, dxi, dd, opts.d_min)
    F1, _ = cost(cam, new, graph, opts)
    return new, dict(dxi=dxi, dd=dd.reshape(state.d.shape), cost_before=neq.cost,
                     cost_after=F1, n_valid=neq.n_valid)


def solve(cam, state, graph, opts, iters):
    """``iters`` steps; returns the final state and the per-step reports."""
    reports = []
    for _ in range(iters):
        state, rep = step(cam, state, graph, opts)
        reports.append(rep)
    return state, reports

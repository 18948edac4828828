"""Full stacked-Jacobian normal equations for tiny problems.

The damped Gauss-Newton step is by definition the solution of
    (J^T W J + D) delta = -J^T W rho
over all unknowns at once: (xi, d) with xi the 15 per-keyframe coordinates and
d every source pixel's inverse depth.  This module writes that definition out
with an explicit dense J (one row per scalar residual) and solves it with
numpy.linalg.solve, so that Eq. 4's Schur route can be checked against a
textbook routine.  Only usable on tiny problems (a few keyframes, a few
pixels).

Test infrastructure (see the package header).
"""
import numpy as np

from . import imu as imu_mod
from . import vision
from .normal_eq import active_mask


def full_system(cam, state, graph, opts, global_bias=False):
    """Dense (H, g) over [xi (15N), d (N*HW)] with g = -J^T W rho.  global_bias:
    each inertial factor's bias columns are added into the last keyframe's."""
    N = state.R.shape[0]
    HW = cam.H * cam.W
    n = 15 * N + N * HW
    rows_J, rows_r, rows_w = [], [], []
    for e in range(len(graph.ii)):
        i, j = int(graph.ii[e]), int(graph.jj[e])
        r, valid, Jp, Jd = vision.edge_linearize_body(cam.intr, cam.T_bc, state.R[i], state.p[i], state.R[j],
                                                      state.p[j], state.d[i], graph.target[e], opts.z_min)
        w = np.where(valid[None], np.asarray(graph.weight[e], np.float64).reshape(2, -1), 0.0)
        for c in range(2):
            for p in range(HW):
                row = np.zeros(n)
                row[15 * i:15 * i + 6] = Jp[c, p, 0:6]
                row[15 * j:15 * j + 6] += Jp[c, p, 6:12]
                row[15 * N + i * HW + p] = Jd[c, p]
                rows_J.append(row)
                rows_r.append(r[c, p])
                rows_w.append(w[c, p])
    Jv = np.array(rows_J)
    rv = np.array(rows_r)
    Wv = np.array(rows_w)
    H = Jv.T @ (Wv[:, None] * Jv)
    g = -Jv.T @ (Wv * rv)
    if opts.use_imu:
        for f, P in enumerate(graph.factors):
            i, j = f, f + 1
            args = (state.R[i], state.p[i], state.v[i], state.b[i],
                    state.R[j], state.p[j], state.v[j], state.b[j], P, cam.gravity)
            r = imu_mod.residual(*args)
            Jf = np.zeros((15, n))
            Jij = imu_mod.jacobian(*args)
            Jf[:, 15 * i:15 * i + 15] = Jij[:, 0:15]
            Jf[:, 15 * j:15 * j + 15] = Jij[:, 15:30]
            if global_bias:
                last = 15 * (N - 1) + 9
                for k in (i, j):
                    if k != N - 1:
                        Jf[:, last:last + 6] += Jf[:, 15 * k + 9:15 * k + 15]
                        Jf[:, 15 * k + 9:15 * k + 15] = 0.0
            L = imu_mod.information(P)
            H += Jf.T @ L @ Jf
            g -= Jf.T @ L @ r
    return H, g


def dense_step(cam, state, graph, opts):
    """Increments (dxi (N,15), dd (N,HW)) from the damped full system.  With
    one global bias the stacked Jacobian's bias columns of all keyframes are
    summed into the last keyframe's (the column of the shared unknown) before
    forming the normal equations."""
    N = state.R.shape[0]
    HW = cam.H * cam.W
    glob = opts.bias_global and opts.use_imu and not opts.bias_fixed
    H, g = full_system(cam, state, graph, opts, glob)
    nx = 15 * N
    Hd = H.copy()
    k = np.arange(nx)
    Hd[k, k] += opts.lm_lambda * H[k, k]
    k = np.arange(nx, H.shape[0])
    Hd[k, k] += opts.depth_eta
    act = np.concatenate([active_mask(N, opts).ravel(), np.ones(N * HW, dtype=bool)])
    x = np.zeros(H.shape[0])
    x[act] = np.linalg.solve(Hd[np.ix_(act, act)], g[act])
    dxi = x[:nx].reshape(N, 15)
    if glob:
        dxi[:, 9:15] = dxi[N - 1, 9:15]
    return dxi, x[nx:].reshape(N, HW)

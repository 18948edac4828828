"""Loop closure by pose-graph bundle adjustment in Sim(3) (Sec. 3.1, "Loop
Closure: Pose Graph Bundle Adjustment", Eq. 5): one damped Gauss-Newton step,
in FP64.

The energy is the vision energy of Eq. 1 restricted to the loop-closure pairs
E* plus relative-pose terms over the pose graph E+:
    E = sum_{(i,j) in E*} sum_u w_x r_x^2 + w_y r_y^2
      + sum_{(i,j) in E+} r_ij^T Lambda_ij r_ij,
    r_ij = log(T~_ij E_ij^-1),   E_ij = T_j^-1 T_i,
optimised over Sim(3) keyframe poses and the inverse depths of the loop
pairs' source keyframes.  Conventions (as for the visual-inertial step):
  * a keyframe pose is the camera-to-world similarity T_i = (s_i, R_i, p_i),
    X_w = s_i R_i X_c + p_i; E_ij = T_j^-1 T_i takes camera i coordinates to
    camera j coordinates, so the vision term reads X_j = E_ij (K^-1 [u; 1] / d);
    T~_ij is the measured E_ij (the paper writes the same residual with
    world-to-camera poses, log(T~_ij T_i T_j^-1));
  * sim(3) tangent ordered (phi, rho, sigma): the Lie-algebra matrix is
    [[sigma I + [phi]x, rho], [0, 0]];
  * keyframe update (dtheta, dp, dsigma): R <- R Exp(dtheta), p <- p + dp,
    s <- s exp(dsigma); inverse depths d <- max(d + dd, d_min);
  * Lambda_ij = (Sigma^rel_ij)^-1 is an input (7 x 7, in the sim(3) order);
  * damping and gauge as in the step: B_rr += lambda B_rr on every solved
    pose coordinate, C += eta; the first n_fixed keyframes are held (all
    seven coordinates).
The step is the exact solution of the damped normal equations, computed by
eliminating the inverse depths (Eq. 4) and solving the reduced 7N system.
Group operations use their definitions: the exponential and logarithm are
scipy's matrix exp / log of the 4 x 4 matrices; ad and Ad are built column by
column from the commutator and the conjugation; the right Jacobian is its
power series in ad, inverted numerically.

Test infrastructure (see the package header).  Pinned by: Exp / Log against
each other and against closed forms for pure rotation, translation and scale;
the Jacobians of both residuals against central finite differences through
the retraction; the Schur-reduced step against the dense stacked-Jacobian
solve; noiseless recovery of a planted scale drift (tests/test_oracle_pgba.py).
"""
from dataclasses import dataclass

import numpy as np
from scipy.linalg import expm, logm

from .so3 import Exp, hat

I3 = np.eye(3)


# --------------------------------------------------------------------------
# Sim(3)
# --------------------------------------------------------------------------
def mat(s, R, t):
    """4 x 4 matrix of the similarity x -> s R x + t."""
    T = np.eye(4)
    T[:3, :3] = s * np.asarray(R)
    T[:3, 3] = t
    return T


def parts(T):
    """(s, R, t) of a 4 x 4 similarity matrix."""
    A = T[:3, :3]
    s = np.cbrt(np.linalg.det(A))
    return s, A / s, T[:3, 3].copy()


def hat7(x):
    """sim(3) vector (phi, rho, sigma) -> 4 x 4 Lie-algebra matrix."""
    x = np.asarray(x, dtype=np.float64)
    M = np.zeros((4, 4))
    M[:3, :3] = x[6] * I3 + hat(x[0:3])
    M[:3, 3] = x[3:6]
    return M


def vee7(M):
    A = M[:3, :3]
    sigma = np.trace(A) / 3.0
    W = A - sigma * I3
    return np.array([W[2, 1], W[0, 2], W[1, 0], M[0, 3], M[1, 3], M[2, 3], sigma])


def Exp7(x):
    return expm(hat7(x))


def Log7(T):
    return vee7(np.real(logm(T)))


def ad7(x):
    """7 x 7 matrix of y -> vee([hat(x), hat(y)])."""
    X = hat7(x)
    A = np.zeros((7, 7))
    for k in range(7):
        Y = hat7(np.eye(7)[k])
        A[:, k] = vee7(X @ Y - Y @ X)
    return A


def Ad7(T):
    """7 x 7 matrix of y -> vee(T hat(y) T^-1)."""
    Ti = np.linalg.inv(T)
    A = np.zeros((7, 7))
    for k in range(7):
        A[:, k] = vee7(T @ hat7(np.eye(7)[k]) @ Ti)
    return A


def Jr7(x, terms=40):
    """Right Jacobian sum_n (-ad_x)^n / (n + 1)!: Exp(x + dx) ~= Exp(x) Exp(Jr dx)."""
    a = -ad7(x)
    J = np.eye(7)
    P = np.eye(7)
    f = 1.0
    for n in range(1, terms):
        P = P @ a
        f /= (n + 1)
        J = J + f * P
    return J


# --------------------------------------------------------------------------
# problem
# --------------------------------------------------------------------------
@dataclass
class PGState:
    R: np.ndarray     # (N, 3, 3)
    p: np.ndarray     # (N, 3)
    s: np.ndarray     # (N,)
    d: np.ndarray     # (N, H, W) inverse depths


@dataclass
class PGGraph:
    ii: np.ndarray         # (E*,) loop-pair sources
    jj: np.ndarray         # (E*,) loop-pair targets
    target: np.ndarray     # (E*, 2, H, W)
    weight: np.ndarray     # (E*, 2, H, W)
    rel_ii: np.ndarray     # (E+,)
    rel_jj: np.ndarray     # (E+,)
    rel_T: np.ndarray      # (E+, 4, 4) measured E_ij
    rel_info: np.ndarray   # (E+, 7, 7) Lambda_ij


@dataclass
class PGOptions:
    n_fixed: int = 1
    lm_lambda: float = 1e-4
    depth_eta: float = 1e-8
    z_min: float = 0.1
    d_min: float = 1e-3


def pose_mat(st, i):
    return mat(st.s[i], st.R[i], st.p[i])


def retract(st, dxi, dd, d_min):
    """Keyframe and inverse-depth update of a step."""
    R = np.stack([st.R[i] @ Exp(dxi[i, 0:3]) for i in range(len(st.s))])
    return PGState(R=R, p=st.p + dxi[:, 3:6], s=st.s * np.exp(dxi[:, 6]), d=np.maximum(st.d + dd, d_min))


# --------------------------------------------------------------------------
# residuals and Jacobians
# --------------------------------------------------------------------------
def rel_residual(st, i, j, Tm):
    """r_ij = Log(T~_ij E_ij^-1), E_ij = T_j^-1 T_i."""
    Eij = np.linalg.inv(pose_mat(st, j)) @ pose_mat(st, i)
    return Log7(Tm @ np.linalg.inv(Eij))


def rel_jacobian(st, i, j, Tm):
    """(7, 7) blocks dr/d(dtheta, dp, dsigma) of keyframes i and j.

    A right perturbation T <- T Exp(xi) moves r by -Jr^-1(r) Ad(E_ij) xi_i
    (keyframe i) and by Jr^-1(r) xi_j (keyframe j); the keyframe update maps
    into xi = (dtheta, R^T dp / s, dsigma) to first order."""
    Eij = np.linalg.inv(pose_mat(st, j)) @ pose_mat(st, i)
    r = Log7(Tm @ np.linalg.inv(Eij))
    Ji = np.linalg.inv(Jr7(r))

    def K(k):
        M = np.eye(7)
        M[3:6, 3:6] = st.R[k].T / st.s[k]
        return M
    return -Ji @ Ad7(Eij) @ K(i), Ji @ K(j)


def vision_edge(cam, st, i, j, target, z_min):
    """Residual r (2, HW), validity (HW,), pose Jacobian (2, HW, 14) with
    respect to (dtheta_i, dp_i, dsigma_i, dtheta_j, dp_j, dsigma_j) and the
    inverse-depth Jacobian (2, HW) of one loop pair:
        X_i = K^-1 [u; 1] / d,  X_j = (s_i R_ij X_i + R_j^T (p_i - p_j)) / s_j,
        r = target - (f X_j,xy / X_j,z + c), valid iff d > 0 and X_j,z > z_min."""
    fx, fy, cx, cy, H, W = cam
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    q = np.stack([((xs - cx) / fx).ravel(), ((ys - cy) / fy).ravel(), np.ones(H * W)], 0)
    d = np.asarray(st.d[i], np.float64).ravel()
    Ri, Rj = st.R[i], st.R[j]
    si, sj = st.s[i], st.s[j]
    Rji = Rj.T @ Ri
    dsafe = np.where(d > 0, d, 1.0)
    Xi = q / dsafe[None]
    Xj = (si * (Rji @ Xi) + (Rj.T @ (st.p[i] - st.p[j]))[:, None]) / sj
    valid = (d > 0) & (Xj[2] > z_min)
    Z = np.where(valid, Xj[2], 1.0)
    u = fx * Xj[0] / Z + cx
    v = fy * Xj[1] / Z + cy
    tg = np.asarray(target, np.float64).reshape(2, -1)
    r = np.where(valid[None], tg - np.stack([u, v]), 0.0)
    # dPi/dX (2, 3, HW)
    dPi = np.zeros((2, 3, H * W))
    dPi[0, 0] = fx / Z
    dPi[0, 2] = -fx * Xj[0] / Z ** 2
    dPi[1, 1] = fy / Z
    dPi[1, 2] = -fy * Xj[1] / Z ** 2
    # dX_j / d(parameters) (3, 14, HW)
    dX = np.zeros((3, 14, H * W))
    A = (si / sj) * Rji
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        dX[:, k] = A @ np.cross(e[:, None], Xi, axis=0)            # R_i <- R_i Exp(dtheta): R_i X_i + R_i (dtheta x X_i)
        dX[:, 3 + k] = (Rj.T[:, k] / sj)[:, None]
        dX[:, 7 + k] = -np.cross(e[:, None], Xj, axis=0)           # R_j^T <- Exp(-dtheta) R_j^T
        dX[:, 10 + k] = -(Rj.T[:, k] / sj)[:, None]
    dX[:, 6] = A @ Xi                                              # s_i <- s_i e^dsigma
    dX[:, 13] = -Xj                                                # 1 / s_j <- e^-dsigma / s_j
    Jp = -np.einsum("cxp,xkp->cpk", dPi, dX)
    Jp = np.where(valid[None, :, None], Jp, 0.0)
    dXd = -(A @ q) / dsafe[None] ** 2
    Jd = np.where(valid[None], -np.einsum("cxp,xp->cp", dPi, dXd), 0.0)
    return r, valid, Jp, Jd


# --------------------------------------------------------------------------
# normal equations, Schur step, dense pin
# --------------------------------------------------------------------------
def linearize(cam, st, gr, opts):
    N = len(st.s)
    fx, fy, cx, cy, H, W = cam
    HW = H * W
    B = np.zeros((7 * N, 7 * N))
    g = np.zeros(7 * N)
    C = np.zeros((N, HW))
    wd = np.zeros((N, HW))
    E = {}
    cost = 0.0
    n_valid = 0
    for e in range(len(gr.ii)):
        i, j = int(gr.ii[e]), int(gr.jj[e])
        r, valid, Jp, Jd = vision_edge(cam, st, i, j, gr.target[e], opts.z_min)
        w = np.where(valid[None], np.asarray(gr.weight[e], np.float64).reshape(2, -1), 0.0)
        n_valid += int(valid.sum())
        cost += float((w * r * r).sum())
        H14 = np.einsum("cp,cpa,cpb->ab", w, Jp, Jp)
        g14 = np.einsum("cp,cpa,cp->a", w, Jp, r)
        idx = np.r_[7 * i:7 * i + 7, 7 * j:7 * j + 7]
        B[np.ix_(idx, idx)] += H14
        g[idx] -= g14
        C[i] += (w * Jd * Jd).sum(0)
        wd[i] -= (w * Jd * r).sum(0)
        Ecol = np.einsum("cp,cpa,cp->ap", w, Jp, Jd)     # (14, HW)
        E.setdefault(i, {})
        for k, blk in ((i, Ecol[0:7]), (j, Ecol[7:14])):
            E[i][k] = E[i].get(k, 0.0) + blk
    for f in range(len(gr.rel_ii)):
        i, j = int(gr.rel_ii[f]), int(gr.rel_jj[f])
        r = rel_residual(st, i, j, gr.rel_T[f])
        Ji, Jj = rel_jacobian(st, i, j, gr.rel_T[f])
        J = np.concatenate([Ji, Jj], axis=1)
        L = gr.rel_info[f]
        cost += float(r @ L @ r)
        idx = np.r_[7 * i:7 * i + 7, 7 * j:7 * j + 7]
        B[np.ix_(idx, idx)] += J.T @ L @ J
        g[idx] -= J.T @ L @ r
    return B, g, C, wd, E, cost, n_valid


def active(N, opts):
    a = np.ones((N, 7), dtype=bool)
    a[:opts.n_fixed] = False
    return a.ravel()


def step(cam, st, gr, opts):
    """One damped Gauss-Newton step by Schur elimination of the inverse
    depths (Eq. 4); returns the new state and a report."""
    N = len(st.s)
    B, g, C, wd, E, cost, n_valid = linearize(cam, st, gr, opts)
    k = np.arange(7 * N)
    Bd = B.copy()
    Bd[k, k] += opts.lm_lambda * B[k, k]
    Cd = C + opts.depth_eta
    inv = np.where(Cd > 0, 1.0 / np.where(Cd > 0, Cd, 1.0), 0.0)
    S = Bd.copy()
    s = g.copy()
    for i, blocks in E.items():
        keys = sorted(blocks)
        rows = np.concatenate([np.arange(7 * t, 7 * t + 7) for t in keys])
        Em = np.concatenate([blocks[t] for t in keys], axis=0)
        S[np.ix_(rows, rows)] -= (Em * inv[i][None]) @ Em.T
        s[rows] -= Em @ (inv[i] * wd[i])
    act = active(N, opts)
    x = np.zeros(7 * N)
    x[act] = np.linalg.solve(S[np.ix_(act, act)], s[act])
    dd = np.zeros_like(wd)
    for i in range(N):
        if i in E:
            keys = sorted(E[i])
            rows = np.concatenate([np.arange(7 * t, 7 * t + 7) for t in keys])
            Em = np.concatenate([E[i][t] for t in keys], axis=0)
            dd[i] = inv[i] * (wd[i] - Em.T @ x[rows])
        else:
            dd[i] = inv[i] * wd[i]
    dxi = x.reshape(N, 7)
    new = retract(st, dxi, dd.reshape(st.d.shape), opts.d_min)
    return new, {"dxi": dxi, "dd": dd.reshape(st.d.shape), "cost_before": cost, "n_valid": n_valid,
                 "cost_after": energy(cam, new, gr, opts)[0]}


def energy(cam, st, gr, opts):
    cost = 0.0
    n_valid = 0
    for e in range(len(gr.ii)):
        i, j = int(gr.ii[e]), int(gr.jj[e])
        r, valid, _, _ = vision_edge(cam, st, i, j, gr.target[e], opts.z_min)
        w = np.where(valid[None], np.asarray(gr.weight[e], np.float64).reshape(2, -1), 0.0)
        cost += float((w * r * r).sum())
        n_valid += int(valid.sum())
    for f in range(len(gr.rel_ii)):
        r = rel_residual(st, int(gr.rel_ii[f]), int(gr.rel_jj[f]), gr.rel_T[f])
        cost += float(r @ gr.rel_info[f] @ r)
    return cost, n_valid


def dense_step(cam, st, gr, opts):
    """The same damped step from the full stacked Jacobian (tiny problems)."""
    N = len(st.s)
    fx, fy, cx, cy, H, W = cam
    HW = H * W
    nd = N * HW
    rows, res, wts = [], [], []
    for e in range(len(gr.ii)):
        i, j = int(gr.ii[e]), int(gr.jj[e])
        r, valid, Jp, Jd = vision_edge(cam, st, i, j, gr.target[e], opts.z_min)
        w = np.where(valid[None], np.asarray(gr.weight[e], np.float64).reshape(2, -1), 0.0)
        for c in range(2):
            for p in range(HW):
                row = np.zeros(7 * N + nd)
                row[7 * i:7 * i + 7] = Jp[c, p, 0:7]
                row[7 * j:7 * j + 7] += Jp[c, p, 7:14]
                row[7 * N + i * HW + p] = Jd[c, p]
                rows.append(row)
                res.append(r[c, p])
                wts.append(w[c, p])
    for f in range(len(gr.rel_ii)):
        i, j = int(gr.rel_ii[f]), int(gr.rel_jj[f])
        r = rel_residual(st, i, j, gr.rel_T[f])
        Ji, Jj = rel_jacobian(st, i, j, gr.rel_T[f])
        Lc = np.linalg.cholesky(gr.rel_info[f])          # Lambda = Lc Lc^T: whitened rows Lc^T J
        for a in range(7):
            row = np.zeros(7 * N + nd)
            row[7 * i:7 * i + 7] = Lc[:, a] @ Ji
            row[7 * j:7 * j + 7] += Lc[:, a] @ Jj
            rows.append(row)
            res.append(Lc[:, a] @ r)
            wts.append(1.0)
    J = np.array(rows)
    rv = np.array(res)
    Wv = np.array(wts)
    Hm = J.T @ (Wv[:, None] * J)
    gv = -J.T @ (Wv * rv)
    k = np.arange(7 * N)
    Hd = Hm.copy()
    Hd[k, k] += opts.lm_lambda * Hm[k, k]
    kd = np.arange(7 * N, 7 * N + nd)
    Hd[kd, kd] += opts.depth_eta
    act = np.concatenate([active(N, opts), np.ones(nd, dtype=bool)])
    x = np.zeros(7 * N + nd)
    x[act] = np.linalg.solve(Hd[np.ix_(act, act)], gv[act])
    return x[:7 * N].reshape(N, 7), x[7 * N:].reshape(st.d.shape)


def solve(cam, st, gr, opts, iters):
    reps = []
    for _ in range(iters):
        st, rep = step(cam, st, gr, opts)
        reps.append(rep)
    return st, reps

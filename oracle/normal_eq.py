"""Normal equations of the joint visual-inertial step and their Schur
elimination (Sec. 3.1, "Frontend Tracking: Local Bundle Adjustment", Eq. 4).

Unknowns: per keyframe the 15-vector (dtheta, dp, dv, db_g, db_a) stacked as
xi (length 15N), and one inverse-depth increment per source pixel, d.  The
system is
    [[B, E], [E^T, C]] [dxi; dd] = [w_xi; w_d]
with H = sum J^T W J over all residuals and w = -sum J^T W r (so the solution
is the descent step).  C is diagonal because each vision term touches one
depth, and is inverted elementwise.  Eq. 4 then gives
    dxi = (B - E C^-1 E^T)^-1 (w_xi - E C^-1 w_d),   dd = C^-1 (w_d - E^T dxi).

Readings: damping is Levenberg-Marquardt with fixed factors applied to the
full system before elimination, B_rr += lambda * B_rr on active pose/velocity/
bias coordinates and C += eta, so the Schur solution equals the damped full
solve exactly; lambda = eta = 0 is pure Gauss-Newton.  The gauge is fixed by
removing the pose coordinates of the first ``n_fixed`` keyframes; with the IMU
off, velocity and bias are removed; with the bias fixed, bias is removed; with
one global bias the biases of all keyframes are the one unknown held in the
last keyframe's slot (fold_global_bias) and the step moves every keyframe's
bias by its increment.
Pixels whose C is zero carry no information (their E column is zero too) and
get dd = 0.

Test infrastructure (see the package header).  Pinned by: equality with the
dense full solve of the stacked Jacobian on tiny problems, symmetry and
positive semi-definiteness of H, and the Cholesky factor against
numpy.linalg.cholesky.
"""
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import imu as imu_mod
from . import vision


class NotPositiveDefinite(Exception):
    """The reduced system is not positive definite."""


@dataclass
class Options:
    n_fixed: int = 1
    use_imu: bool = True
    bias_fixed: bool = False
    bias_global: bool = False      # one bias shared by every keyframe (Table 6 (f))
    lm_lambda: float = 1e-4
    depth_eta: float = 1e-8
    z_min: float = 0.1
    d_min: float = 1e-3


@dataclass
class State:
    R: np.ndarray     # (N,3,3) world-from-body rotation
    p: np.ndarray     # (N,3)
    v: np.ndarray     # (N,3)
    b: np.ndarray     # (N,6)
    d: np.ndarray     # (N,H,W) inverse depth

    def copy(self):
        return State(self.R.copy(), self.p.copy(), self.v.copy(), self.b.copy(), self.d.copy())


@dataclass
class Camera:
    fx: float
    fy: float
    cx: float
    cy: float
    H: int
    W: int
    gravity: np.ndarray
    T_bc: Optional[Tuple[np.ndarray, np.ndarray]] = None   # body-from-camera (R_bc, t_bc); None = identity

    @property
    def intr(self):
        return (self.fx, self.fy, self.cx, self.cy, self.H, self.W)


@dataclass
class Graph:
    ii: np.ndarray                 # (E,) source keyframe
    jj: np.ndarray                 # (E,) target keyframe
    target: np.ndarray             # (E,2,H,W)
    weight: np.ndarray             # (E,2,H,W)
    factors: list                  # preintegrated factor per pair (i, i+1)


@dataclass
class NormalEquations:
    B: np.ndarray                              # (15N, 15N)
    w_xi: np.ndarray                           # (15N,)
    C: np.ndarray                              # (N, HW)
    w_d: np.ndarray                            # (N, HW)
    E: Dict[int, Tuple[np.ndarray, np.ndarray]]  # source i -> (touched KFs, (nt, 6, HW))
    cost: float
    n_valid: int


def active_mask(N, opts):
    """(N, 15) boolean mask of the coordinates that are solved for."""
    a = np.ones((N, 15), dtype=bool)
    a[: opts.n_fixed, 0:6] = False
    if not opts.use_imu:
        a[:, 6:15] = False
    if opts.bias_fixed:
        a[:, 9:15] = False
    elif opts.bias_global:
        a[:-1, 9:15] = False          # the shared bias sits in the last keyframe's slot
    return a


def fold_global_bias(neq, N):
    """One bias for the whole window (Table 6 (f)): every keyframe's bias is
    the single unknown b, held in the last keyframe's bias slot.  With G the
    15N x 15N map that copies that slot into every keyframe's bias (and is the
    identity on poses and velocities), the normal equations become G^T B G and
    G^T w_xi; E couples depths to poses only and is unchanged.  The random-walk
    term b_j - b_i is then constant and drops out of the step."""
    G = np.zeros((15 * N, 15 * N))
    for a in range(N):
        for c in range(9):
            G[15 * a + c, 15 * a + c] = 1.0
        for c in range(9, 15):
            G[15 * a + c, 15 * (N - 1) + c] = 1.0
    return NormalEquations(B=G.T @ neq.B @ G, w_xi=G.T @ neq.w_xi, C=neq.C, w_d=neq.w_d, E=neq.E, cost=neq.cost,
                           n_valid=neq.n_valid)


def linearize(cam, state, graph, opts):
    """Assemble B, w_xi, E, C, w_d and the cost at ``state``."""
    N = state.R.shape[0]
    HW = cam.H * cam.W
    B = np.zeros((15 * N, 15 * N))
    w_xi = np.zeros(15 * N)
    C = np.zeros((N, HW))
    w_d = np.zeros((N, HW))
    E: Dict[int, Tuple[np.ndarray, np.ndarray]] = {}
    cost = 0.0
    n_valid = 0
    for i in range(N):
        T = [i] + [int(j) for j in graph.jj[graph.ii == i]]
        E[i] = (np.array(T), np.zeros((len(T), 6, HW)))
    for e in range(len(graph.ii)):
        i, j = int(graph.ii[e]), int(graph.jj[e])
        r, valid, Jp, Jd = vision.edge_linearize_body(
            cam.intr, cam.T_bc, state.R[i], state.p[i], state.R[j], state.p[j],
            state.d[i], graph.target[e], opts.z_min)
        w = np.where(valid[None], np.asarray(graph.weight[e], np.float64).reshape(2, -1), 0.0)
        n_valid += int(valid.sum())
        cost += float((w * r * r).sum())
        H12 = np.einsum("cp,cpa,cpb->ab", w, Jp, Jp)
        g12 = np.einsum("cp,cpa,cp->a", w, Jp, r)
        blocks = [15 * i, 15 * j]
        for a in range(2):
            for b in range(2):
                B[blocks[a]:blocks[a] + 6, blocks[b]:blocks[b] + 6] += H12[6 * a:6 * a + 6, 6 * b:6 * b + 6]
            w_xi[blocks[a]:blocks[a] + 6] -= g12[6 * a:6 * a + 6]
        C[i] += (w * Jd * Jd).sum(0)
        w_d[i] -= (w * Jd * r).sum(0)
        T, Ei = E[i]
        Ecol = np.einsum("cp,cpa,cp->ap", w, Jp, Jd)     # (12, HW)
        Ei[0] += Ecol[0:6]
        Ei[int(np.nonzero(T == j)[0][0])] += Ecol[6:12]
    if opts.use_imu:
        g = cam.gravity
        for f, P in enumerate(graph.factors):
            i, j = f, f + 1
            args = (state.R[i], state.p[i], state.v[i], state.b[i],
                    state.R[j], state.p[j], state.v[j], state.b[j], P, g)
            r = imu_mod.residual(*args)
            J = imu_mod.jacobian(*args)
            L = imu_mod.information(P)
            cost += float(r @ L @ r)
            Hf = J.T @ L @ J
            gf = J.T @ L @ r
            idx = np.r_[15 * i:15 * i + 15, 15 * j:15 * j + 15]
            B[np.ix_(idx, idx)] += Hf
            w_xi[idx] -= gf
    return NormalEquations(B=B, w_xi=w_xi, C=C, w_d=w_d, E=E, cost=cost, n_valid=n_valid)


def damped(neq, opts):
    """B with lambda * diag(B) added on its diagonal, and C + eta."""
    B = neq.B.copy()
    k = np.arange(B.shape[0])
    B[k, k] += opts.lm_lambda * neq.B[k, k]
    return B, neq.C + opts.depth_eta


def reduced_system(neq, opts):
    """Eq. 4's reduced matrix S = B - E C^-1 E^T and vector s = w_xi - E C^-1 w_d
    (damped, over all 15N coordinates)."""
    B, Cd = damped(neq, opts)
    S = B.copy()
    s = neq.w_xi.copy()
    for i, (T, Ei) in neq.E.items():
        rows = np.concatenate([np.arange(15 * t, 15 * t + 6) for t in T])
        Em = Ei.reshape(len(T) * 6, -1)
        inv = np.where(Cd[i] > 0, 1.0 / np.where(Cd[i] > 0, Cd[i], 1.0), 0.0)
        S[np.ix_(rows, rows)] -= (Em * inv[None]) @ Em.T
        s[rows] -= Em @ (inv * neq.w_d[i])
    return S, s, Cd


def cholesky(S):
    """Lower-triangular L with S = L L^T (plain column algorithm)."""
    n = S.shape[0]
    L = np.zeros_like(S)
    for k in range(n):
        piv = S[k, k] - L[k, :k] @ L[k, :k]
        if not piv > 0.0:
            raise NotPositiveDefinite(f"pivot {k} = {piv}")
        L[k, k] = np.sqrt(piv)
        L[k + 1:, k] = (S[k + 1:, k] - L[k + 1:, :k] @ L[k, :k]) / L[k, k]
    return L


def solve_spd(S, s):
    """Solve S x = s by Cholesky, forward and back substitution."""
    L = cholesky(S)
    n = S.shape[0]
    y = np.zeros(n)
    for k in range(n):
        y[k] = (s[k] - L[k, :k] @ y[:k]) / L[k, k]
    x = np.zeros(n)
    for k in range(n - 1, -1, -1):
        x[k] = (y[k] - L[k + 1:, k] @ x[k + 1:]) / L[k, k]
    return x


def schur_solve(neq, opts, N):
    """Eq. 4: returns dxi (N, 15) and dd (N, HW)."""
    S, s, Cd = reduced_system(neq, opts)
    act = active_mask(N, opts).ravel()
    x = solve_spd(S[np.ix_(act, act)], s[act])
    dxi = np.zeros(15 * N)
    dxi[act] = x
    dd = np.zeros_like(neq.w_d)
    for i, (T, Ei) in neq.E.items():
        rows = np.concatenate([np.arange(15 * t, 15 * t + 6) for t in T])
        Em = Ei.reshape(len(T) * 6, -1)
        inv = np.where(Cd[i] > 0, 1.0 / np.where(Cd[i] > 0, Cd[i], 1.0), 0.0)
        dd[i] = inv * (neq.w_d[i] - Em.T @ dxi[rows])
    return dxi.reshape(N, 15), dd

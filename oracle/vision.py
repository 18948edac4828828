"""Vision residual of Eq. 1 (Sec. 3.1) for one edge (i, j) of the frame graph.

For every pixel u of keyframe i with inverse depth d:
    X_i = Pi^-1(u, d) = K^-1 [u; 1] / d          (point in camera i)
    X_j = T_ij X_i = R_ij X_i + t_ij               (T_ij takes frame i to frame j)
    r   = u*_ij(u) - Pi(X_j)
with world-from-body poses (R, p): R_ij = R_j^T R_i, t_ij = R_j^T (p_i - p_j).
The energy weights each coordinate by the confidence w (read as information):
    E_vis = sum_u  w_x r_x^2 + w_y r_y^2.
A pixel-residual is used only when d > 0 and the point lies in front of
camera j by more than z_min (X_j.z > z_min); otherwise its residual and
Jacobian are zero and it is excluded from the cost.  Projections that land
outside the image remain valid: the target is only a coordinate.

Analytic Jacobians with respect to (dtheta_i, dp_i, dtheta_j, dp_j, d), from
R <- R Exp(dtheta) and additive world-frame p:
    dX_j/dtheta_i = -R_ij [X_i]x      dX_j/dp_i =  R_j^T
    dX_j/dtheta_j =  [X_j]x           dX_j/dp_j = -R_j^T
    dX_j/dd       = -R_ij K^-1[u;1] / d^2
and r's Jacobian is -dPi/dX times these.

Camera-IMU extrinsics (Sec. 3.1, inertial residual: left out of the
printed equations, used by the implementation): the state holds world-from-
body poses (R_b, p_b); the camera of a keyframe is T_wc = T_wb T_bc with the
constant body-from-camera T_bc = (R_bc, t_bc), i.e. R_c = R_b R_bc and
p_c = p_b + R_b t_bc, and the residual above is taken between camera poses.
A body increment (dtheta, dp) moves the camera by
    dtheta_c = R_bc^T dtheta,   dp_c = dp - R_b [t_bc]x dtheta
to first order, so the Jacobian with respect to the body increments is the
camera Jacobian times K = [[R_bc^T, 0], [-R_b [t_bc]x, I]] per keyframe
(edge_linearize_body).  With T_bc = identity both coincide.

Test infrastructure (see the package header).  Pinned by: zero residual at
noiseless ground truth, hand closed forms for identity rotation, and the
Jacobians against central finite differences (also through the body
retraction with a non-identity T_bc).
"""
import numpy as np


def pixel_rays(fx, fy, cx, cy, H, W):
    """K^-1 [x; y; 1] for x = column, y = row; shape (3, H*W)."""
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    return np.stack([((xs - cx) / fx).ravel(), ((ys - cy) / fy).ravel(), np.ones(H * W)], 0)


def _skew_batch(v):
    """[v]x for each column of v (3, n) -> (n, 3, 3)."""
    n = v.shape[1]
    S = np.zeros((n, 3, 3))
    S[:, 0, 1] = -v[2]
    S[:, 0, 2] = v[1]
    S[:, 1, 0] = v[2]
    S[:, 1, 2] = -v[0]
    S[:, 2, 0] = -v[1]
    S[:, 2, 1] = v[0]
    return S


def edge_residual(cam, Ri, pi, Rj, pj, d, target, z_min):
    """Residual r (2, HW) and validity (HW,) of one edge; r is zero where invalid."""
    fx, fy, cx, cy, H, W = cam
    R_ij = Rj.T @ Ri
    t_ij = Rj.T @ (pi - pj)
    q = pixel_rays(fx, fy, cx, cy, H, W)
    d = np.asarray(d, dtype=np.float64).ravel()
    pos = d > 0
    ds = np.where(pos, d, 1.0)
    X_i = q / ds[None]
    X_j = R_ij @ X_i + t_ij[:, None]
    valid = pos & (X_j[2] > z_min)
    zs = np.where(valid, X_j[2], 1.0)
    proj = np.stack([fx * X_j[0] / zs + cx, fy * X_j[1] / zs + cy], 0)
    tgt = np.asarray(target, dtype=np.float64).reshape(2, -1)
    r = np.where(valid[None], tgt - proj, 0.0)
    return r, valid


def edge_linearize(cam, Ri, pi, Rj, pj, d, target, z_min):
    """Residual, validity and Jacobians of one edge.

    Returns r (2, HW), valid (HW,), J_pose (2, HW, 12) in the order
    (dtheta_i, dp_i, dtheta_j, dp_j), and J_d (2, HW); all zero where invalid.
    """
    fx, fy, cx, cy, H, W = cam
    R_ij = Rj.T @ Ri
    t_ij = Rj.T @ (pi - pj)
    q = pixel_rays(fx, fy, cx, cy, H, W)
    d = np.asarray(d, dtype=np.float64).ravel()
    pos = d > 0
    ds = np.where(pos, d, 1.0)
    X_i = q / ds[None]
    X_j = R_ij @ X_i + t_ij[:, None]
    valid = pos & (X_j[2] > z_min)
    Z = np.where(valid, X_j[2], 1.0)
    proj = np.stack([fx * X_j[0] / Z + cx, fy * X_j[1] / Z + cy], 0)
    tgt = np.asarray(target, dtype=np.float64).reshape(2, -1)
    r = np.where(valid[None], tgt - proj, 0.0)

    n = q.shape[1]
    # dPi/dX, (n, 2, 3)
    dPi = np.zeros((n, 2, 3))
    dPi[:, 0, 0] = fx / Z
    dPi[:, 0, 2] = -fx * X_j[0] / (Z * Z)
    dPi[:, 1, 1] = fy / Z
    dPi[:, 1, 2] = -fy * X_j[1] / (Z * Z)
    dX = np.zeros((n, 3, 13))
    dX[:, :, 0:3] = -R_ij[None] @ _skew_batch(X_i)
    dX[:, :, 3:6] = Rj.T[None]
    dX[:, :, 6:9] = _skew_batch(X_j)
    dX[:, :, 9:12] = -Rj.T[None]
    dX[:, :, 12] = -(R_ij @ q).T / (ds * ds)[:, None]
    J = -(dPi @ dX)                                   # (n, 2, 13)
    J = np.where(valid[:, None, None], J, 0.0)
    J_pose = np.transpose(J[:, :, 0:12], (1, 0, 2))  # (2, n, 12)
    J_d = J[:, :, 12].T                               # (2, n)
    return r, valid, J_pose, J_d


def skew(v):
    v = np.asarray(v, dtype=np.float64)
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def camera_pose(R_b, p_b, T_bc):
    """World-from-camera rotation and position of a keyframe with world-from-
    body pose (R_b, p_b); T_bc = (R_bc, t_bc) or None for the identity."""
    if T_bc is None:
        return R_b, p_b
    R_bc, t_bc = T_bc
    return R_b @ R_bc, p_b + R_b @ t_bc


def body_map(R_b, T_bc):
    """6x6 K with (dtheta_c, dp_c) = K (dtheta, dp) for a body increment."""
    K = np.eye(6)
    if T_bc is not None:
        R_bc, t_bc = T_bc
        K[0:3, 0:3] = R_bc.T
        K[3:6, 0:3] = -R_b @ skew(t_bc)
    return K


def edge_residual_body(cam, T_bc, Ri, pi, Rj, pj, d, target, z_min):
    """edge_residual between the cameras of body poses i and j."""
    Rci, pci = camera_pose(Ri, pi, T_bc)
    Rcj, pcj = camera_pose(Rj, pj, T_bc)
    return edge_residual(cam, Rci, pci, Rcj, pcj, d, target, z_min)


def edge_linearize_body(cam, T_bc, Ri, pi, Rj, pj, d, target, z_min):
    """edge_linearize between the cameras of body poses i and j, with the
    pose Jacobian taken with respect to the body increments
    (dtheta_i, dp_i, dtheta_j, dp_j)."""
    Rci, pci = camera_pose(Ri, pi, T_bc)
    Rcj, pcj = camera_pose(Rj, pj, T_bc)
    r, valid, Jp, Jd = edge_linearize(cam, Rci, pci, Rcj, pcj, d, target, z_min)
    if T_bc is not None:
        Jp = np.concatenate([Jp[..., 0:6] @ body_map(Ri, T_bc), Jp[..., 6:12] @ body_map(Rj, T_bc)], axis=-1)
    return r, valid, Jp, Jd

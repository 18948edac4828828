"""Loop-closure update of a Gaussian map (Sec. 3.3, "Loop Closure Gaussian
Update", Eq. 7 and Eq. 8).

TEST INFRASTRUCTURE ONLY (see the package header).

After pose-graph bundle adjustment every keyframe k has a pre-update pose
(R_k^-, t_k^-), a post-update pose (R_k^+, t_k^+) and a scale change ds_k.  A
Gaussian initialised from keyframe k moves with it: its mean is taken into the
old camera frame, scaled by ds_k and mapped out of the new one (Eq. 7); its
covariance is rotated the same way and scaled by ds_k^2 (Eq. 8).  Opacity and
colour do not change, so they are not inputs here.

Poses are camera-to-world, stored as 7 doubles (t, q xyzw); the quaternion is
normalised before use.  Covariances are stored as their 6 upper-triangle
entries (xx, xy, xz, yy, yz, zz).

Pinned by (tests/test_oracle_gauss.py): the identity update returns its input;
the means agree with a 4x4 homogeneous similarity built from the two poses and
inverted by numpy.linalg.inv; the covariance update agrees with the image of
sigma points mu + L e_c (L = Cholesky factor of Sigma) under the mean map, an
independent route through Eq. 7; local coordinates in the new frame are ds_k
times those in the old frame; eigenvalues scale by ds_k^2; a pure translation
of the keyframe shifts the means and leaves the covariances alone.
"""
import numpy as np

from .so3 import quat_to_R

COV_INDEX = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def cov6_to_mat(c6):
    """[..., 6] upper-triangle entries -> [..., 3, 3] symmetric matrices."""
    c6 = np.asarray(c6, dtype=np.float64)
    S = np.empty(c6.shape[:-1] + (3, 3))
    for e, (r, c) in enumerate(COV_INDEX):
        S[..., r, c] = c6[..., e]
        S[..., c, r] = c6[..., e]
    return S


def mat_to_cov6(S):
    return np.stack([S[..., r, c] for r, c in COV_INDEX], axis=-1)


def pose_Rt(pose):
    """[N][7] (t, q xyzw) -> R [N][3][3], t [N][3]."""
    pose = np.asarray(pose, dtype=np.float64)
    R = np.stack([quat_to_R(q) for q in pose[:, 3:7]]) if len(pose) else np.zeros((0, 3, 3))
    return R, pose[:, 0:3].copy()


def keyframe_valid(pose_pre, pose_post, scale_change):
    """A keyframe's Gaussians are moved only when its scale change is positive and
    finite and both poses are finite with a non-zero quaternion; otherwise they
    are left as they are."""
    pose_pre = np.asarray(pose_pre, dtype=np.float64)
    pose_post = np.asarray(pose_post, dtype=np.float64)
    s = np.asarray(scale_change, dtype=np.float64)
    ok = np.isfinite(s) & (s > 0)
    ok &= np.all(np.isfinite(pose_pre), axis=1) & np.all(np.isfinite(pose_post), axis=1)
    ok &= (np.sum(pose_pre[:, 3:7] ** 2, axis=1) > 0) & (np.sum(pose_post[:, 3:7] ** 2, axis=1) > 0)
    return ok


def reanchor(mean, cov6, anchor, pose_pre, pose_post, scale_change):
    """Eq. 7 and Eq. 8 for every Gaussian, in FP64.

    mean [K][3], cov6 [K][6] or None, anchor [K] (int), poses [N][7],
    scale_change [N].  Returns (mean_new, cov6_new or None, rejected [K] bool):
    a Gaussian whose anchor is outside 0..N-1 or whose keyframe is not valid
    (keyframe_valid) keeps its mean and covariance and is marked rejected.
    """
    mean = np.asarray(mean, dtype=np.float64)
    anchor = np.asarray(anchor, dtype=np.int64)
    N = len(pose_pre)
    K = len(mean)
    kf_ok = keyframe_valid(pose_pre, pose_post, scale_change)
    inside = (anchor >= 0) & (anchor < N)
    ok = np.zeros(K, dtype=bool)
    ok[inside] = kf_ok[anchor[inside]]
    k = np.where(ok, anchor, 0)
    safe_pre = np.where(kf_ok[:, None], pose_pre, [0, 0, 0, 0, 0, 0, 1])
    safe_post = np.where(kf_ok[:, None], pose_post, [0, 0, 0, 0, 0, 0, 1])
    Rm, tm = pose_Rt(safe_pre)
    Rp, tp = pose_Rt(safe_post)
    ds = np.where(kf_ok, scale_change, 1.0)
    if K == 0:
        return mean.copy(), (None if cov6 is None else np.asarray(cov6, np.float64).copy()), ok.copy()
    Rm, tm, Rp, tp, ds = Rm[k], tm[k], Rp[k], tp[k], ds[k]

    # Eq. 7: into the old camera frame, scale, out of the new camera frame
    x_loc_old = np.einsum("kji,kj->ki", Rm, mean - tm)          # (R^-)^T (mu - t^-)
    x_loc_new = ds[:, None] * x_loc_old
    mean_new = np.einsum("kij,kj->ki", Rp, x_loc_new) + tp
    mean_new = np.where(ok[:, None], mean_new, mean)

    cov_new = None
    if cov6 is not None:
        S = cov6_to_mat(cov6)
        # Eq. 8: R^+ (ds^2 (R^-)^T Sigma R^-) (R^+)^T
        inner = (ds ** 2)[:, None, None] * np.einsum("kji,kjl,klm->kim", Rm, S, Rm)
        S_new = np.einsum("kij,kjl,kml->kim", Rp, inner, Rp)
        cov_new = np.where(ok[:, None], mat_to_cov6(S_new), np.asarray(cov6, dtype=np.float64))
    return mean_new, cov_new, ~ok

"""Pins of the Gaussian-map loop-closure update oracle (Sec. 3.3, Eq. 7-8)
against routes that do not go through its own formulas: homogeneous 4x4
similarity matrices inverted by numpy.linalg.inv, sigma points pushed through
the mean map, eigenvalues, and special cases with closed forms."""
import numpy as np
import pytest

from oracle import gauss as og
from oracle.so3 import Exp, quat_to_R, R_to_quat
from paper_2512_02293_amd import synth


def _map(n_kf=6, per_kf=50, seed=3):
    return synth.make_gaussian_map(n_kf, per_kf, seed, H=48, W=64)


def _sim4(pose, s=1.0):
    T = np.eye(4)
    T[:3, :3] = quat_to_R(pose[3:7]) * s
    T[:3, 3] = pose[:3]
    return T


def test_identity_update_returns_input():
    g = _map()
    mean, cov, rej = og.reanchor(g.mean, g.cov, g.anchor, g.pose_pre, g.pose_pre, np.ones(len(g.pose_pre)))
    assert not rej.any()
    np.testing.assert_allclose(mean, g.mean.astype(np.float64), rtol=0, atol=1e-14)
    np.testing.assert_allclose(cov, g.cov.astype(np.float64), rtol=0, atol=1e-13 * np.abs(g.cov).max())


def test_means_match_homogeneous_similarity():
    """mu+ = T+ diag(ds, ds, ds, 1) (T-)^-1 mu with T = [[R, t], [0, 1]]."""
    g = _map()
    mean, _, _ = og.reanchor(g.mean, None, g.anchor, g.pose_pre, g.pose_post, g.scale_change)
    for i in range(0, len(g.mean), 7):
        k = g.anchor[i]
        M = _sim4(g.pose_post[k]) @ np.diag([g.scale_change[k]] * 3 + [1.0]) @ np.linalg.inv(_sim4(g.pose_pre[k]))
        ref = (M @ np.append(g.mean[i].astype(np.float64), 1.0))[:3]
        np.testing.assert_allclose(mean[i], ref, rtol=0, atol=1e-13)


def test_covariance_is_the_image_of_sigma_points_under_the_mean_map():
    """The mean map f is affine, so sum_c (f(mu + L e_c) - f(mu)) (...)^T with
    L L^T = Sigma is the covariance of the mapped Gaussian."""
    g = _map(per_kf=20)
    mean, cov, _ = og.reanchor(g.mean, g.cov, g.anchor, g.pose_pre, g.pose_post, g.scale_change)
    S_new = og.cov6_to_mat(cov)
    for i in range(len(g.mean)):
        S = og.cov6_to_mat(g.cov[i])
        L = np.linalg.cholesky(S)
        pts = g.mean[i].astype(np.float64) + L.T        # rows mu + L e_c
        anc = np.full(3, g.anchor[i])
        fp, _, _ = og.reanchor(pts, None, anc, g.pose_pre, g.pose_post, g.scale_change)
        D = fp - mean[i]
        np.testing.assert_allclose(S_new[i], D.T @ D, rtol=1e-6, atol=1e-8 * np.abs(S).max())


def test_local_coordinates_scale_and_eigenvalues_scale():
    g = _map()
    mean, cov, _ = og.reanchor(g.mean, g.cov, g.anchor, g.pose_pre, g.pose_post, g.scale_change)
    for i in range(0, len(g.mean), 5):
        k = g.anchor[i]
        Rm, Rp = quat_to_R(g.pose_pre[k][3:7]), quat_to_R(g.pose_post[k][3:7])
        loc_old = Rm.T @ (g.mean[i] - g.pose_pre[k][:3])
        loc_new = Rp.T @ (mean[i] - g.pose_post[k][:3])
        np.testing.assert_allclose(loc_new, g.scale_change[k] * loc_old, rtol=1e-12, atol=1e-13)
        ev_old = np.linalg.eigvalsh(og.cov6_to_mat(g.cov[i]))
        ev_new = np.linalg.eigvalsh(og.cov6_to_mat(cov[i]))
        np.testing.assert_allclose(ev_new, g.scale_change[k] ** 2 * ev_old, rtol=1e-9)


def test_pure_translation_and_rotation_about_the_camera_centre():
    g = _map(n_kf=3, per_kf=10)
    post = g.pose_pre.copy()
    post[:, :3] += np.array([0.5, -1.0, 2.0])
    mean, cov, _ = og.reanchor(g.mean, g.cov, g.anchor, g.pose_pre, post, np.ones(3))
    np.testing.assert_allclose(mean, g.mean + np.array([0.5, -1.0, 2.0]), atol=1e-13)
    np.testing.assert_allclose(cov, g.cov.astype(np.float64), rtol=1e-12, atol=1e-20)
    # camera at the origin, rotated by Q: means and covariances rotate by Q
    pre = np.tile([0, 0, 0, 0, 0, 0, 1.0], (3, 1))
    Q = Exp([0.3, -0.2, 0.9])
    post = np.tile(np.concatenate([[0, 0, 0], R_to_quat(Q)]), (3, 1))
    mean, cov, _ = og.reanchor(g.mean, g.cov, g.anchor, pre, post, np.full(3, 2.0))
    np.testing.assert_allclose(mean, 2.0 * g.mean @ Q.T, atol=1e-12)
    S = og.cov6_to_mat(g.cov.astype(np.float64))
    np.testing.assert_allclose(og.cov6_to_mat(cov), 4.0 * Q @ S @ Q.T, rtol=1e-12, atol=1e-20)


def test_rejections_keep_the_gaussian():
    g = _map(n_kf=4, per_kf=5)
    ds = g.scale_change.copy()
    ds[1] = 0.0
    ds[2] = np.nan
    anchor = g.anchor.copy()
    anchor[0] = -1
    anchor[-1] = 4
    mean, cov, rej = og.reanchor(g.mean, g.cov, anchor, g.pose_pre, g.pose_post, ds)
    expect = (anchor < 0) | (anchor >= 4) | (anchor == 1) | (anchor == 2)
    np.testing.assert_array_equal(rej, expect)
    np.testing.assert_array_equal(mean[expect], g.mean[expect].astype(np.float64))
    np.testing.assert_array_equal(cov[expect], g.cov[expect].astype(np.float64))
    assert not np.allclose(mean[~expect], g.mean[~expect])


def test_empty_map():
    g = _map(n_kf=2, per_kf=1)
    mean, cov, rej = og.reanchor(np.zeros((0, 3)), np.zeros((0, 6)), np.zeros(0, np.int32), g.pose_pre,
                                 g.pose_post, g.scale_change)
    assert mean.shape == (0, 3) and cov.shape == (0, 6) and rej.shape == (0,)


@pytest.mark.parametrize("mistake", ["R_pre_not_transposed", "cov_scale_off"])
def test_pins_catch_planted_mistakes(mistake, monkeypatch):
    """A transposed rotation in Eq. 7, or a covariance scaled by a wrong factor
    in Eq. 8, planted in the oracle, fails the pins."""
    real = np.einsum

    def bad(spec, *ops):
        if mistake == "R_pre_not_transposed" and spec == "kji,kj->ki":
            spec = "kij,kj->ki"
        if mistake == "cov_scale_off" and spec == "kji,kjl,klm->kim":
            return real(spec, *ops) * 1.01
        return real(spec, *ops)

    monkeypatch.setattr(og.np, "einsum", bad)
    with pytest.raises(AssertionError):
        if mistake == "R_pre_not_transposed":
            test_means_match_homogeneous_similarity()
        else:
            test_local_coordinates_scale_and_eigenvalues_scale()

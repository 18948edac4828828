"""Pins of the oracle's vision (Eq. 1) and inertial (Eq. 3) residuals:
zero at discrete-consistent ground truth, hand closed forms, and analytic
Jacobians against central finite differences through the retraction."""
import numpy as np
import pytest

from oracle import imu, preint, so3, vision
from oracle import solve as osolve
from paper_2512_02293_amd import synth


def _gt_state(p):
    return osolve.state_from_arrays(p.pose_gt, p.vel_gt, p.bias_gt, p.invdepth_gt)


def test_vision_residual_zero_at_noiseless_ground_truth():
    cfg = synth.config_small()
    cfg.noiseless = True
    p = synth.make_problem(cfg, 1)
    cam, _, gr = osolve.from_problem(p, exact_targets=True)
    gt = _gt_state(p)
    worst = 0.0
    for e in range(p.n_edges):
        i, j = int(p.ii[e]), int(p.jj[e])
        r, valid = vision.edge_residual(cam.intr, gt.R[i], gt.p[i], gt.R[j], gt.p[j], gt.d[i],
                                        gr.target[e], p.z_min)
        assert valid.all()
        worst = max(worst, np.abs(r).max())
    assert worst < 1e-9, worst


def test_vision_closed_form_identity_rotation():
    """R_ij = I: u' = (x - cx + fx t_x d) / (1 + t_z d) + cx, same for y."""
    fx, fy, cx, cy, H, W = 60.0, 55.0, 32.0, 24.0, 6, 7
    rng = np.random.default_rng(0)
    d = rng.uniform(0.2, 2.0, (H, W))
    t = np.array([0.13, -0.07, 0.21])
    Ri = so3.Exp(np.array([0.1, 0.2, -0.3]))
    pi = np.array([0.5, -1.0, 2.0])
    Rj = Ri.copy()
    pj = pi - Ri @ t                  # t_ij = R_j^T (p_i - p_j) = t
    ys, xs = np.mgrid[0:H, 0:W].astype(float)
    u = (xs - cx + fx * t[0] * d) / (1 + t[2] * d) + cx
    v = (ys - cy + fy * t[1] * d) / (1 + t[2] * d) + cy
    r, valid = vision.edge_residual((fx, fy, cx, cy, H, W), Ri, pi, Rj, pj, d, np.zeros((2, H, W)), 0.1)
    assert valid.all()
    assert np.allclose(-r[0], u.ravel(), rtol=1e-14, atol=1e-12)
    assert np.allclose(-r[1], v.ravel(), rtol=1e-14, atol=1e-12)
    # pure x-translation: u' = x + fx t_x d, v' = y
    t2 = np.array([0.3, 0.0, 0.0])
    r2, _ = vision.edge_residual((fx, fy, cx, cy, H, W), Ri, pi, Ri, pi - Ri @ t2, d,
                                 np.zeros((2, H, W)), 0.1)
    assert np.allclose(-r2[0], (xs + fx * 0.3 * d).ravel(), atol=1e-12)
    assert np.allclose(-r2[1], ys.ravel(), atol=1e-12)


def test_vision_validity_depth_threshold():
    fx, fy, cx, cy, H, W = 10.0, 10.0, 2.0, 2.0, 4, 4
    d = np.full((H, W), 1.0)
    d[0, 0] = -0.5                    # non-positive inverse depth is never used
    R = np.eye(3)
    # camera j 0.95 m in front of camera i along its optical axis: depth 0.05 < z_min
    r, valid = vision.edge_residual((fx, fy, cx, cy, H, W), R, np.zeros(3), R,
                                    np.array([0, 0, 0.95]), d, np.zeros((2, H, W)), 0.1)
    assert not valid.any()
    r, valid = vision.edge_residual((fx, fy, cx, cy, H, W), R, np.zeros(3), R,
                                    np.array([0, 0, 0.85]), d, np.zeros((2, H, W)), 0.1)
    assert valid.sum() == H * W - 1 and not valid[0]
    assert np.all(r[:, 0] == 0)


def _perturb_pose(R, p, k, h):
    """Retraction of a 6-vector pose tangent along coordinate k by h."""
    dv = np.zeros(6)
    dv[k] = h
    return R @ so3.Exp(dv[:3]), p + dv[3:]


def test_vision_jacobians_finite_difference():
    p = synth.make_problem(synth.tiny_config(n_kf=3, H=4, W=5), 5)
    cam, st, gr = osolve.from_problem(p)
    h = 1e-6
    for e in range(p.n_edges):
        i, j = int(p.ii[e]), int(p.jj[e])
        args = dict(Ri=st.R[i], pi=st.p[i], Rj=st.R[j], pj=st.p[j], d=st.d[i])
        r0, valid, Jp, Jd = vision.edge_linearize(cam.intr, target=gr.target[e], z_min=0.1, **args)
        assert valid.all()
        for k in range(12):
            which, kk = ("i", k) if k < 6 else ("j", k - 6)
            plus = dict(args)
            minus = dict(args)
            plus["R" + which], plus["p" + which] = _perturb_pose(args["R" + which], args["p" + which], kk, h)
            minus["R" + which], minus["p" + which] = _perturb_pose(args["R" + which], args["p" + which], kk, -h)
            rp, _ = vision.edge_residual(cam.intr, target=gr.target[e], z_min=0.1, **plus)
            rm, _ = vision.edge_residual(cam.intr, target=gr.target[e], z_min=0.1, **minus)
            fd = (rp - rm) / (2 * h)
            assert np.allclose(Jp[:, :, k], fd, rtol=1e-6, atol=1e-6), (e, k)
        # inverse depth: per pixel
        dd = np.full(st.d[i].shape, h)
        rp, _ = vision.edge_residual(cam.intr, st.R[i], st.p[i], st.R[j], st.p[j], st.d[i] + dd, gr.target[e], 0.1)
        rm, _ = vision.edge_residual(cam.intr, st.R[i], st.p[i], st.R[j], st.p[j], st.d[i] - dd, gr.target[e], 0.1)
        assert np.allclose(Jd, (rp - rm) / (2 * h), rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("bias_hat_mode", ["gt"])
def test_imu_residual_zero_at_noiseless_ground_truth(bias_hat_mode):
    cfg = synth.config_small()
    cfg.noiseless = True            # constant, nonzero true bias; no white noise
    p = synth.make_problem(cfg, 1, bias_hat_mode=bias_hat_mode)
    assert np.abs(p.bias_gt).max() > 1e-3
    _, _, gr = osolve.from_problem(p)
    gt = _gt_state(p)
    for f, P in enumerate(gr.factors):
        r = imu.residual(gt.R[f], gt.p[f], gt.v[f], gt.b[f], gt.R[f + 1], gt.p[f + 1],
                         gt.v[f + 1], gt.b[f + 1], P, p.gravity)
        assert np.abs(r).max() < 1e-12, (f, np.abs(r).max())


def test_imu_residual_nonzero_for_wrong_gravity_sign():
    """The zero-residual pin above is sensitive to the gravity convention."""
    cfg = synth.config_small()
    cfg.noiseless = True
    p = synth.make_problem(cfg, 1, bias_hat_mode="gt")
    _, _, gr = osolve.from_problem(p)
    gt = _gt_state(p)
    P = gr.factors[0]
    r = imu.residual(gt.R[0], gt.p[0], gt.v[0], gt.b[0], gt.R[1], gt.p[1], gt.v[1], gt.b[1], P, -p.gravity)
    assert np.abs(r[3:9]).max() > 0.1


def test_imu_jacobian_finite_difference():
    rng = np.random.default_rng(9)
    n, hs = 20, 0.005
    gyro = rng.normal(0, 0.5, (n, 3))
    accel = rng.normal(0, 1.0, (n, 3)) + np.array([0, 0, 9.81])
    P = preint.preintegrate(gyro, accel, np.full(n, hs), np.array([0.01, 0.0, -0.01, 0.05, 0.02, -0.03]),
                            1.7e-4, 2e-3, 2e-5, 3e-3)
    g = np.array([0, 0, -9.81])
    x = dict(Ri=so3.Exp(rng.normal(0, 0.5, 3)), pi=rng.normal(0, 1, 3), vi=rng.normal(0, 1, 3),
             bi=rng.normal(0, 0.05, 6), Rj=so3.Exp(rng.normal(0, 0.5, 3)), pj=rng.normal(0, 1, 3),
             vj=rng.normal(0, 1, 3), bj=rng.normal(0, 0.05, 6))

    def res(x):
        return imu.residual(x["Ri"], x["pi"], x["vi"], x["bi"], x["Rj"], x["pj"], x["vj"], x["bj"], P, g)

    def moved(x, k, h):
        y = dict(x)
        s = "i" if k < 15 else "j"
        c = k % 15
        if c < 3:
            e = np.zeros(3)
            e[c] = h
            y["R" + s] = x["R" + s] @ so3.Exp(e)
        elif c < 6:
            y["p" + s] = x["p" + s] + h * np.eye(3)[c - 3]
        elif c < 9:
            y["v" + s] = x["v" + s] + h * np.eye(3)[c - 6]
        else:
            y["b" + s] = x["b" + s] + h * np.eye(6)[c - 9]
        return y

    J = imu.jacobian(x["Ri"], x["pi"], x["vi"], x["bi"], x["Rj"], x["pj"], x["vj"], x["bj"], P, g)
    h = 1e-6
    Jfd = np.stack([(res(moved(x, k, h)) - res(moved(x, k, -h))) / (2 * h) for k in range(30)], 1)
    assert np.allclose(J, Jfd, rtol=1e-6, atol=1e-7), np.abs(J - Jfd).max()


def test_imu_information_is_inverse_covariance():
    P = preint.preintegrate(np.tile([0.1, 0.2, 0.3], (20, 1)), np.tile([0, 0.5, 9.8], (20, 1)),
                            np.full(20, 0.005), np.zeros(6), 1.7e-4, 2e-3, 2e-5, 3e-3)
    L = imu.information(P)
    S = np.zeros((15, 15))
    S[:9, :9] = P.cov
    S[9:, 9:] = np.diag(P.cov_bias)
    assert np.allclose(L @ S, np.eye(15), atol=1e-8)
    assert np.allclose(L, L.T, rtol=1e-10)

"""Camera-IMU extrinsics in the oracle (Sec. 3.1, inertial residual: T_bc is
left out of the printed equations and used by the implementation).

Pins: the residual with a pure camera offset equals the residual of cameras
moved by that offset (closed form, body rotation identity); with T_bc =
identity the body Jacobian is the camera Jacobian exactly; the body-increment
Jacobian against central finite differences through the body retraction
(R <- R Exp(dtheta), p <- p + dp) with a non-identity T_bc; zero residual at
the noiseless ground truth of a window whose cameras are offset and rotated
from the IMU body; and Gauss-Newton from a perturbed state recovers that
ground truth (poses 1e-7), which fails if T_bc enters the vision terms and the
inertial terms inconsistently."""
import numpy as np

from oracle import normal_eq as ne, so3, solve, vision
from paper_2512_02293_amd import synth

T_BC = (0.04, -0.02, 0.015, *so3.R_to_quat(so3.Exp(np.deg2rad(np.array([6.0, -4.0, 9.0])))))


def _tbc():
    t = np.asarray(T_BC)
    return so3.quat_to_R(t[3:7]), t[:3]


def test_offset_camera_closed_form():
    cam = (50.0, 50.0, 8.0, 6.0, 12, 16)
    rng = np.random.default_rng(0)
    d = rng.uniform(0.2, 0.6, size=(12, 16))
    t_bc = np.array([0.05, -0.03, 0.02])
    Ri, pi = np.eye(3), np.zeros(3)
    Rj, pj = np.eye(3), np.array([0.1, 0.0, -0.05])
    tgt = rng.normal(8.0, 3.0, size=(2, 12, 16))
    r_body, _ = vision.edge_residual_body(cam, (np.eye(3), t_bc), Ri, pi, Rj, pj, d, tgt, 0.1)
    r_cam, _ = vision.edge_residual(cam, Ri, pi + t_bc, Rj, pj + t_bc, d, tgt, 0.1)
    assert np.array_equal(r_body, r_cam)
    # a rotated body carries the offset along: camera at p + R t_bc
    R = so3.Exp(np.array([0.0, 0.3, 0.0]))
    r_body, _ = vision.edge_residual_body(cam, (np.eye(3), t_bc), R, pi, R, pj, d, tgt, 0.1)
    r_cam, _ = vision.edge_residual(cam, R, pi + R @ t_bc, R, pj + R @ t_bc, d, tgt, 0.1)
    assert np.allclose(r_body, r_cam, atol=1e-12)


def test_identity_extrinsic_is_the_camera_jacobian():
    prob = synth.make_problem(synth.tiny_config(n_kf=3, H=6, W=8), 3)
    cam, st, gr = solve.from_problem(prob)
    i, j = int(gr.ii[0]), int(gr.jj[0])
    a = vision.edge_linearize(cam.intr, st.R[i], st.p[i], st.R[j], st.p[j], st.d[i], gr.target[0], 0.1)
    b = vision.edge_linearize_body(cam.intr, (np.eye(3), np.zeros(3)), st.R[i], st.p[i], st.R[j], st.p[j],
                                   st.d[i], gr.target[0], 0.1)
    for x, y in zip(a, b):
        assert np.allclose(x, y, atol=1e-14, rtol=0)


def test_body_jacobian_finite_differences():
    cfg = synth.tiny_config(n_kf=3, H=6, W=8)
    cfg.T_bc = T_BC
    prob = synth.make_problem(cfg, 4)
    cam, st, gr = solve.from_problem(prob)
    T = cam.T_bc
    for e in range(len(gr.ii)):
        i, j = int(gr.ii[e]), int(gr.jj[e])
        r0, valid, Jp, _ = vision.edge_linearize_body(cam.intr, T, st.R[i], st.p[i], st.R[j], st.p[j], st.d[i],
                                                      gr.target[e], 0.1)
        assert valid.mean() > 0.5
        h = 1e-6
        for k in range(12):
            which, comp = (i, k) if k < 6 else (j, k - 6)
            out = []
            for sgn in (1.0, -1.0):
                R = st.R.copy()
                p = st.p.copy()
                if comp < 3:
                    dth = np.zeros(3)
                    dth[comp] = sgn * h
                    R[which] = R[which] @ so3.Exp(dth)
                else:
                    p[which, comp - 3] += sgn * h
                r, _ = vision.edge_residual_body(cam.intr, T, R[i], p[i], R[j], p[j], st.d[i], gr.target[e], 0.1)
                out.append(r)
            fd = (out[0] - out[1]) / (2 * h)
            scale = max(np.abs(Jp[:, valid, k]).max(), 1.0)
            assert np.abs(fd[:, valid] - Jp[:, valid, k]).max() < 2e-5 * scale, (e, k)


def test_noiseless_truth_has_zero_vision_residual():
    cfg = synth.tiny_config(n_kf=4, H=8, W=10, noiseless=True)
    cfg.T_bc = T_BC
    prob = synth.make_problem(cfg, 5)
    cam, _, gr = solve.from_problem(prob, exact_targets=True)
    gt = ne.State(np.stack([so3.quat_to_R(q) for q in prob.pose_gt[:, 3:]]), prob.pose_gt[:, :3], prob.vel_gt,
                  prob.bias_gt, prob.invdepth_gt)
    for e in range(len(gr.ii)):
        i, j = int(gr.ii[e]), int(gr.jj[e])
        r, valid = vision.edge_residual_body(cam.intr, cam.T_bc, gt.R[i], gt.p[i], gt.R[j], gt.p[j], gt.d[i],
                                             gr.target[e], 0.1)
        assert valid.mean() > 0.5
        assert np.abs(r[:, valid]).max() < 1e-9
        # the same residual without the extrinsic is far from zero
        r0, v0 = vision.edge_residual(cam.intr, gt.R[i], gt.p[i], gt.R[j], gt.p[j], gt.d[i], gr.target[e], 0.1)
        assert np.abs(r0[:, v0 & valid]).max() > 1e-2


def test_gauss_newton_recovers_the_truth_with_extrinsics():
    cfg = synth.tiny_config(n_kf=5, H=10, W=12, noiseless=True)
    cfg.T_bc = T_BC
    prob = synth.make_problem(cfg, 6, bias_hat_mode="gt")
    cam, st, gr = solve.from_problem(prob, exact_targets=True)
    opts = ne.Options(lm_lambda=0.0, depth_eta=1e-12)
    for _ in range(8):
        st, _ = solve.step(cam, st, gr, opts)
    Rgt = np.stack([so3.quat_to_R(q) for q in prob.pose_gt[:, 3:]])
    assert np.abs(st.p - prob.pose_gt[:, :3]).max() < 1e-7
    assert max(np.linalg.norm(so3.Log(a.T @ b)) for a, b in zip(st.R, Rgt)) < 1e-7

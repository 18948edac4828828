"""Pins of the warm-start network oracle (oracle/cnn.py) against things other
than itself: scipy's 2-D correlation, central finite differences, the closed
form of an AdamW step from zero moments, exact bilinear reproduction of
constant and linear inputs, and zero residual features at noiseless ground
truth."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn, solve as osolve
from paper_2512_02293_amd import synth


def test_conv3x3_matches_scipy_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 5, 7))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = cnn.conv3x3(x, W, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(x[n, i], W[o, i], mode="same", boundary="fill") for i in range(3))
            assert np.allclose(y[n, o], ref, atol=1e-12)


def _tiny_batch(seed=1, B=2, h=4, w=5):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((B, cnn.C_IN, h, w))
    mask = np.ones((B, h, w))
    mask[1, :, -1] = 0.0          # a narrower image on the shared canvas
    dd_lab = rng.standard_normal((B, h, w)) * 0.02
    db_lab = rng.standard_normal((B, 6)) * cnn.S_B
    return x, mask, dd_lab, db_lab


def test_backward_matches_finite_differences():
    x, mask, dd_lab, db_lab = _tiny_batch()
    theta = cnn.init_params(3) * 0.5
    theta[cnn.n_params() - 6:] += 0.01
    _, g = cnn.backward(theta, x, mask, dd_lab, db_lab)
    rng = np.random.default_rng(7)
    # every parameter group, a few entries each
    offs, o = [], 0
    for name, shp in cnn.SHAPES:
        n = int(np.prod(shp))
        offs += list(o + rng.choice(n, size=min(n, 6), replace=False))
        o += n
    h = 1e-6
    for k in offs:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        dd_p, db_p, _ = cnn.forward(tp, x, mask)
        dd_m, db_m, _ = cnn.forward(tm, x, mask)
        fd = (cnn.loss(dd_p, db_p, dd_lab, db_lab, mask) - cnn.loss(dd_m, db_m, dd_lab, db_lab, mask)) / (2 * h)
        assert fd == pytest.approx(g[k], rel=1e-5, abs=1e-7), (k, fd, g[k])


def test_masked_cells_do_not_influence_outputs():
    x, mask, _, _ = _tiny_batch()
    theta = cnn.init_params(5)
    dd1, db1, _ = cnn.forward(theta, x, mask)
    x2 = x.copy()
    x2[1, :, :, -1] = 123.0       # garbage outside image 1's grid
    dd2, db2, _ = cnn.forward(theta, x2, mask)
    assert np.array_equal(dd1, dd2) and np.array_equal(db1, db2)


def test_adamw_first_step_closed_form():
    rng = np.random.default_rng(2)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, eps, wd = 1e-3, 1e-8, 1e-2
    th1, m, v = cnn.adamw_step(th, g, np.zeros(50), np.zeros(50), 1, lr, eps=eps, wd=wd)
    assert np.allclose(th1, th - lr * (g / (np.abs(g) + eps) + wd * th), rtol=1e-12, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_upsample_reproduces_constant_and_linear_fields():
    const = np.full((3, 4), 0.7)
    assert np.allclose(cnn.upsample4(const, 12, 16), 0.7)
    cy, cx = np.mgrid[0:5, 0:6].astype(float)
    lin = 0.3 + 0.05 * cy - 0.02 * cx
    up = cnn.upsample4(lin, 20, 24)
    y, x = np.mgrid[0:20, 0:24].astype(float)
    inner = (y >= 2) & (y <= 17) & (x >= 2) & (x <= 21)      # between the first and last cell centres
    ref = 0.3 + 0.05 * (y - 1.5) / 4 - 0.02 * (x - 1.5) / 4
    assert np.allclose(up[inner], ref[inner], atol=1e-14)


def test_features_vanish_at_noiseless_ground_truth():
    cfg = synth.config_small()
    cfg.noiseless = True
    cfg.zero_bias = True
    prob = synth.make_problem(cfg, 1)
    cam, st, gr = osolve.from_problem(prob, exact_targets=True)
    gt = osolve.state_from_arrays(prob.pose_gt, prob.vel_gt, prob.bias_gt, prob.invdepth_gt)
    X, mask = cnn.features(cam, gt, gr)
    assert X.shape == (8, 15, 12, 16) and mask.all()
    assert np.abs(X[:, 0:2]).max() < 1e-9          # residuals vanish at the truth
    assert np.abs(X[:, 4:13]).max() < 1e-8         # inertial residuals vanish (discrete-consistent truth)
    assert np.abs(X[:, 13]).max() < 1e-6           # so does the depth-only step
    assert np.allclose(X[:, 3], np.stack([cnn.cell_mean(d, 48, 64) for d in prob.invdepth_gt]))
    assert (X[:, 2] > 0).all()


def test_depth_step_channel_recovers_a_depth_offset():
    """Poses at the truth, noiseless targets, every inverse depth of the
    keyframes raised by delta: the residual is J_d delta to first order, so the
    depth-only step of every cell is -delta (channel 13 = -delta / 0.2) up to
    O(delta^2); channel 14 equals log(1 + h / n_cell) with h formed from
    central finite differences of the residual in the inverse depth."""
    from oracle import vision
    cfg = synth.config_small()
    cfg.noiseless = True
    cfg.zero_bias = True
    prob = synth.make_problem(cfg, 2)
    cam, _, gr = osolve.from_problem(prob, exact_targets=True)
    delta = 1e-4
    st = osolve.state_from_arrays(prob.pose_gt, prob.vel_gt, prob.bias_gt, prob.invdepth_gt + delta)
    X, _ = cnn.features(cam, st, gr)
    cells = X[:, 13]
    live = np.abs(cells) > 0
    assert live.mean() > 0.9
    np.testing.assert_allclose(cells[live], -delta / 0.2, rtol=2e-3)
    # channel 14 of keyframe 0 from finite differences
    fx, fy, cx, cy, H, W = cam.intr
    i, eps = 0, 1e-6
    h = np.zeros(H * W)
    for e in range(len(gr.ii)):
        if int(gr.ii[e]) != i:
            continue
        j = int(gr.jj[e])
        args = (cam.intr, st.R[i], st.p[i], st.R[j], st.p[j])
        rp, vp = vision.edge_residual(*args, st.d[i] + eps, gr.target[e], 0.1)
        rm, vm = vision.edge_residual(*args, st.d[i] - eps, gr.target[e], 0.1)
        Jd = (rp - rm) / (2 * eps)
        w = np.asarray(gr.weight[e], np.float64).reshape(2, -1) * (vp & vm)[None]
        h += (w * Jd * Jd).sum(axis=0)
    ref = np.log1p(cnn.cell_mean(h.reshape(H, W), H, W))
    np.testing.assert_allclose(X[i, 14], ref, rtol=1e-6)


def _hand_window():
    """Two keyframes, identity rotations, keyframe 1 at (-0.1, 0, 0): the
    edge 0 -> 1 has R_ji = I, t_ji = (0.1, 0, 0), so with fx = fy = 10 a pixel
    (x, y) of inverse depth d projects to (x + d, y) and the inverse-depth
    column of the Jacobian is (J_dx, J_dy) = (-1, 0).  4 x 8 pixels = two
    4 x 4 cells.  The targets are that projection plus chosen residuals."""
    from oracle.normal_eq import Camera, Graph, State
    from oracle.preint import Preintegrated
    from oracle.so3 import Exp
    H, W = 4, 8
    cam = Camera(10.0, 10.0, 0.0, 0.0, H, W, np.array([0.0, 0.0, -9.81]))
    d0 = np.zeros((H, W))
    d0[:, :4] = 0.5
    d0[:, 4:] = np.array([1.0, 1.2, 1.4, 1.6])[:, None]
    ys, xs = np.mgrid[0:H, 0:W].astype(float)
    rx, ry = np.zeros((H, W)), np.zeros((H, W))
    wx, wy = np.zeros((H, W)), np.zeros((H, W))
    # cell 0: r_x = 1 (w_x = 1) on even columns, 3 (w_x = 0.2) on odd ones; r_y = -1 (w_y = 0.25)
    even = (xs[:, :4] % 2) == 0
    rx[:, :4] = np.where(even, 1.0, 3.0)
    wx[:, :4] = np.where(even, 1.0, 0.2)
    ry[:, :4], wy[:, :4] = -1.0, 0.25
    # cell 1: r_x = 0 (w_x = 0.5); r_y = 2 (w_y = 0.1) on rows 0-1, 0 (w_y = 0.9) on rows 2-3
    rx[:, 4:], wx[:, 4:] = 0.0, 0.5
    ry[:2, 4:], wy[:2, 4:] = 2.0, 0.1
    ry[2:, 4:], wy[2:, 4:] = 0.0, 0.9
    target = np.stack([xs + d0 + rx, ys + ry])[None]
    weight = np.stack([wx, wy])[None]
    theta = np.array([0.01, -0.02, 0.005])
    fac = Preintegrated(dt=0.1, dR=Exp(theta), dv=np.array([0.0, 0.2, 0.0]), dp=np.array([0.3, 0.0, 0.0]),
                        J_rot=np.zeros((3, 3)), J_vel=np.zeros((3, 6)), J_pos=np.zeros((3, 6)), cov=np.eye(9),
                        bias_hat=np.zeros(6), cov_bias=np.ones(6))
    st = State(R=np.stack([np.eye(3)] * 2), p=np.array([[0.0, 0, 0], [-0.1, 0, 0]]),
               v=np.array([[1.0, 0, 0], [1.0, 0, 0]]), b=np.zeros((2, 6)), d=np.stack([d0, np.full((H, W), 0.7)]))
    gr = Graph(ii=np.array([0]), jj=np.array([1]), target=target, weight=weight, factors=[fac])
    return cam, st, gr


def test_features_hand_computed_cells():
    """Every channel of a hand-built window against values worked out from its
    geometry: weighted means with unequal x / y weights (ch 0-2), the cell
    mean depth (ch 3), the inertial residual of a factor with known deltas at
    a chosen state, scaled 100 / 10 / 10 (ch 4-12), and the depth-only step
    and information with J_d = (-1, 0) (ch 13-14)."""
    cam, st, gr = _hand_window()
    X, mask = cnn.features(cam, st, gr)
    assert X.shape == (2, 15, 1, 2) and mask.all()
    c0, c1 = X[0, :, 0, 0], X[0, :, 0, 1]
    # cell 0: sum w_x r_x = 8 * 1 + 8 * 0.2 * 3 = 12.8, sum w_x = 9.6; sum w_y r_y = -4, sum w_y = 4
    assert c0[0] == pytest.approx(12.8 / (9.6 + 1e-6), rel=1e-14)
    assert c0[1] == pytest.approx(-4.0 / (4.0 + 1e-6), rel=1e-14)
    assert c0[2] == pytest.approx((9.6 + 4.0) / 32.0, rel=1e-14)
    assert c0[3] == pytest.approx(0.5, rel=1e-14)
    # J_dx = -1: sum w J_d r = -12.8, h = sum w_x = 9.6
    assert c0[13] == pytest.approx(12.8 / (9.6 + 1e-6) / 0.2, rel=1e-12)
    assert c0[14] == pytest.approx(np.log1p(9.6 / 16.0), rel=1e-14)
    # cell 1: no x residual; sum w_y r_y = 8 * 0.1 * 2 = 1.6, sum w_y = 0.8 + 7.2 = 8
    assert abs(c1[0]) < 1e-14
    assert c1[1] == pytest.approx(1.6 / (8.0 + 1e-6), rel=1e-14)
    assert c1[2] == pytest.approx((8.0 + 8.0) / 32.0, rel=1e-14)
    assert c1[3] == pytest.approx(1.3, rel=1e-14)
    assert abs(c1[13]) < 1e-13
    assert c1[14] == pytest.approx(np.log1p(0.5), rel=1e-14)
    # inertial residual of factor (0, 1): rotation Log(dR^T) = -theta;
    # position p1 - p0 - v0 dt - g dt^2 / 2 - dp = (-0.5, 0, 0.04905);
    # velocity v1 - v0 - g dt - dv = (0, -0.2, 0.981)
    ref = np.concatenate([-100.0 * np.array([0.01, -0.02, 0.005]), 10.0 * np.array([-0.5, 0.0, 0.04905]),
                          10.0 * np.array([0.0, -0.2, 0.981])])
    for cell in (c0, c1):
        np.testing.assert_allclose(cell[4:13], ref, rtol=1e-12, atol=1e-14)
    # keyframe 1: no outgoing edge, last keyframe (no factor after it)
    assert np.all(X[1, [0, 1, 2, 13, 14]] == 0.0) and np.all(X[1, 4:13] == 0.0)
    np.testing.assert_allclose(X[1, 3], 0.7, rtol=1e-14)
    # without inertial terms the constant planes are zero
    Xn, _ = cnn.features(cam, st, gr, use_imu=False)
    assert np.all(Xn[:, 4:13] == 0.0) and np.array_equal(Xn[:, :4], X[:, :4])


def test_loss_closed_form():
    """Two images on a 1 x 2 canvas, the second one cell wide: every valid
    cell is off by s_d (term 1 each, mean over the 3 valid cells = 1; the
    masked cell is off by 0.5 and must not count), and the bias corrections
    are off by s_b in the first gyro axis of image 0 and by 2 s_b in the last
    accelerometer axis of image 1 (sum 1 + 4 = 5, mean over 2 images = 2.5)."""
    mask = np.array([[[1.0, 1.0]], [[1.0, 0.0]]])
    dd_lab = np.array([[[0.1, -0.2]], [[0.3, 0.0]]])
    dd = dd_lab + np.array([[[0.02, -0.02]], [[0.02, 0.5]]])
    db_lab = np.array([[0.001, 0, 0, 0, 0, 0.2], [0, 0, 0, 0, 0, -0.1]])
    db = db_lab + np.array([[0.005, 0, 0, 0, 0, 0], [0, 0, 0, 0, 0, 0.1]])
    assert cnn.loss(dd, db, dd_lab, db_lab, mask) == pytest.approx(3.5, rel=1e-12)

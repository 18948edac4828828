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

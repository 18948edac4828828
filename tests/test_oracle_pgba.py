"""Pins of the Sim(3) pose-graph bundle adjustment oracle (oracle/pgba.py):
closed forms of the group exponential, the right Jacobian and both residual
Jacobians against central finite differences, the Schur step against the
dense stacked-Jacobian solve, and noiseless recovery of a planted scale drift."""
import numpy as np
import pytest

from oracle import pgba
from oracle.so3 import Exp, quat_to_R
from paper_2512_02293_amd import synth


def _graph(prob, exact=False):
    Tm = np.stack([pgba.mat(m[7], quat_to_R(m[3:7]), m[0:3]) for m in prob.rel_meas]) if len(prob.rel_meas) else \
        np.zeros((0, 4, 4))
    return pgba.PGGraph(ii=prob.ii, jj=prob.jj, target=prob.target64 if exact else prob.target.astype(np.float64),
                        weight=prob.weight.astype(np.float64), rel_ii=prob.rel_ii, rel_jj=prob.rel_jj, rel_T=Tm,
                        rel_info=prob.rel_info)


def _state(pose, scale, d):
    return pgba.PGState(R=np.stack([quat_to_R(q) for q in pose[:, 3:7]]), p=np.array(pose[:, :3]),
                        s=np.array(scale, dtype=np.float64), d=np.array(d, dtype=np.float64))


def _tiny(noiseless=False, seed=3, N=4, H=6, W=8):
    cfg = synth.SceneConfig(n_kf=N, H=H, W=W, k_out=1)
    loops = [(0, N - 1), (N - 1, 0), (1, N - 2)]
    rel = [(i, i + 1) for i in range(N - 1)] + [(i, i + 2) for i in range(N - 2)]
    prob = synth.make_pgba_problem(cfg, seed, loops, rel, noiseless=noiseless)
    cam = (prob.fx, prob.fy, prob.cx, prob.cy, prob.H, prob.W)
    return prob, cam, _state(prob.pose, prob.scale, prob.invdepth), _graph(prob, exact=noiseless)


def test_exp_log_closed_forms():
    phi = np.array([0.1, -0.2, 0.3])
    T = pgba.Exp7(np.r_[phi, 0, 0, 0, 0])
    assert np.allclose(T[:3, :3], Exp(phi), atol=1e-14) and np.allclose(T[:3, 3], 0, atol=1e-15)
    T = pgba.Exp7(np.r_[0, 0, 0, 0.5, -1.0, 2.0, 0])
    assert np.allclose(T, np.block([[np.eye(3), np.array([[0.5], [-1.0], [2.0]])], [np.zeros((1, 3)), 1.0]]))
    T = pgba.Exp7(np.r_[0, 0, 0, 0, 0, 0, 0.3])
    assert np.allclose(T[:3, :3], np.exp(0.3) * np.eye(3), atol=1e-14)
    rng = np.random.default_rng(0)
    for _ in range(5):
        x = rng.normal(size=7) * 0.4
        assert np.allclose(pgba.Log7(pgba.Exp7(x)), x, atol=1e-12)
    # ad and Ad agree with their defining identities: Exp(Ad_T x) = T Exp(x) T^-1, d/dt Ad_Exp(tx) = ad_x at 0
    T = pgba.Exp7(rng.normal(size=7) * 0.3)
    x = rng.normal(size=7) * 0.2
    assert np.allclose(pgba.Exp7(pgba.Ad7(T) @ x), T @ pgba.Exp7(x) @ np.linalg.inv(T), atol=1e-12)
    h = 1e-6
    D = (pgba.Ad7(pgba.Exp7(h * x)) - pgba.Ad7(pgba.Exp7(-h * x))) / (2 * h)
    assert np.allclose(D, pgba.ad7(x), atol=1e-8)


def test_right_jacobian_by_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.normal(size=7) * 0.5
    J = pgba.Jr7(x)
    h = 1e-6
    Tx = pgba.Exp7(x)
    for k in range(7):
        e = np.zeros(7)
        e[k] = h
        fd = (pgba.Log7(np.linalg.inv(Tx) @ pgba.Exp7(x + e)) - pgba.Log7(np.linalg.inv(Tx) @ pgba.Exp7(x - e))) / (2 * h)
        assert np.allclose(fd, J[:, k], atol=1e-8), k


def _perturb(st, i, k, h):
    dxi = np.zeros((len(st.s), 7))
    dxi[i, k] = h
    return pgba.retract(st, dxi, np.zeros_like(st.d), -np.inf)


def test_relative_pose_jacobian_by_finite_differences():
    prob, cam, st, gr = _tiny()
    h = 1e-6
    for f in range(len(gr.rel_ii)):
        i, j = int(gr.rel_ii[f]), int(gr.rel_jj[f])
        Ji, Jj = pgba.rel_jacobian(st, i, j, gr.rel_T[f])
        for blk, kf in ((Ji, i), (Jj, j)):
            for k in range(7):
                fd = (pgba.rel_residual(_perturb(st, kf, k, h), i, j, gr.rel_T[f])
                      - pgba.rel_residual(_perturb(st, kf, k, -h), i, j, gr.rel_T[f])) / (2 * h)
                assert np.allclose(fd, blk[:, k], rtol=1e-6, atol=1e-6), (f, kf, k, fd, blk[:, k])


def test_vision_jacobians_by_finite_differences():
    prob, cam, st, gr = _tiny()
    h = 1e-6
    for e in range(len(gr.ii)):
        i, j = int(gr.ii[e]), int(gr.jj[e])
        r, valid, Jp, Jd = pgba.vision_edge(cam, st, i, j, gr.target[e], 0.1)
        assert valid.all()
        for col, (kf, k) in enumerate([(i, k) for k in range(7)] + [(j, k) for k in range(7)]):
            rp = pgba.vision_edge(cam, _perturb(st, kf, k, h), i, j, gr.target[e], 0.1)[0]
            rm = pgba.vision_edge(cam, _perturb(st, kf, k, -h), i, j, gr.target[e], 0.1)[0]
            assert np.allclose((rp - rm) / (2 * h), Jp[:, :, col], rtol=1e-5, atol=1e-5), (e, col)
        # the scale of the target keyframe does not move a projection
        assert np.abs(Jp[:, :, 13]).max() < 1e-9
        dp = st.d.copy()
        dm = st.d.copy()
        dp[i] += h
        dm[i] -= h
        rp = pgba.vision_edge(cam, pgba.PGState(st.R, st.p, st.s, dp), i, j, gr.target[e], 0.1)[0]
        rm = pgba.vision_edge(cam, pgba.PGState(st.R, st.p, st.s, dm), i, j, gr.target[e], 0.1)[0]
        assert np.allclose((rp - rm) / (2 * h), Jd, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("lam,eta", [(1e-4, 1e-8), (0.0, 1e-6), (1e-2, 1e-3)])
def test_schur_step_equals_dense_solve(lam, eta):
    prob, cam, st, gr = _tiny(H=4, W=5)
    opts = pgba.PGOptions(lm_lambda=lam, depth_eta=eta)
    _, rep = pgba.step(cam, st, gr, opts)
    dxi, dd = pgba.dense_step(cam, st, gr, opts)
    assert np.allclose(rep["dxi"], dxi, rtol=1e-7, atol=1e-10 * np.abs(dxi).max())
    assert np.allclose(rep["dd"], dd, rtol=1e-7, atol=1e-10 * np.abs(dd).max())
    assert np.all(rep["dxi"][0] == 0.0)


def test_noiseless_recovery_of_a_scale_drift():
    """Noiseless loop pairs and relative poses: pure Gauss-Newton from scale
    errors of up to 5 % (and the pose / depth perturbations of the generator)
    recovers the true similarities, including the planted scale drift of
    10 % along the trajectory, and the inverse depths."""
    prob, cam, st, gr = _tiny(noiseless=True, N=5, H=8, W=10)
    opts = pgba.PGOptions(lm_lambda=0.0, depth_eta=0.0)
    assert np.abs(np.log(prob.scale / prob.scale_gt)).max() > 0.01
    F0 = pgba.energy(cam, st, gr, opts)[0]
    st, reps = pgba.solve(cam, st, gr, opts, 10)
    F = pgba.energy(cam, st, gr, opts)[0]
    assert F < 1e-20 * F0
    np.testing.assert_allclose(st.s, prob.scale_gt, rtol=1e-9)
    np.testing.assert_allclose(st.p, prob.pose_gt[:, :3], atol=1e-9)
    R_gt = np.stack([quat_to_R(q) for q in prob.pose_gt[:, 3:7]])
    assert np.abs(st.R - R_gt).max() < 1e-9
    np.testing.assert_allclose(st.d[[0, 1, 4]], prob.invdepth_gt[[0, 1, 4]], rtol=1e-8)

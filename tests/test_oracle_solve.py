"""Pins of the oracle's normal equations, Schur elimination and iteration:
Eq. 4 against a dense textbook solve of the stacked system, Cholesky against
numpy, H symmetric PSD, noiseless convergence to the ground truth, and gauge
covariance under a global yaw and translation."""
import numpy as np
import pytest

from oracle import dense, normal_eq as ne, so3
from oracle import solve as osolve
from paper_2512_02293_amd import synth


def _tiny(seed=5, **kw):
    p = synth.make_problem(synth.tiny_config(**kw), seed)
    cam, st, gr = osolve.from_problem(p)
    return p, cam, st, gr


@pytest.mark.parametrize("opts,shape", [
    (ne.Options(), (3, 4, 5, 2)),
    # undamped: a 3-keyframe, 20-pixel window is numerically singular, use 5 x 30 px
    (ne.Options(lm_lambda=0.0, depth_eta=0.0), (5, 5, 6, 3)),
    (ne.Options(lm_lambda=0.0, depth_eta=0.0, bias_fixed=True), (5, 5, 6, 3)),
    (ne.Options(lm_lambda=0.3, depth_eta=0.05, n_fixed=2), (3, 4, 5, 2)),
    (ne.Options(use_imu=False), (3, 4, 5, 2)),
    (ne.Options(bias_fixed=True), (3, 4, 5, 2)),
])
def test_schur_equals_dense_solve(opts, shape):
    n, H, W, k = shape
    p, cam, st, gr = _tiny(n_kf=n, H=H, W=W, k_out=k)
    neq = ne.linearize(cam, st, gr, opts)
    dxi, dd = ne.schur_solve(neq, opts, n)
    dxi_d, dd_d = dense.dense_step(cam, st, gr, opts)
    # two backward-stable solves of the same system agree to ~ kappa * eps, with
    # kappa the condition number of the Jacobi-scaled full matrix
    Hf, _ = dense.full_system(cam, st, gr, opts)
    act = np.concatenate([ne.active_mask(n, opts).ravel(), np.ones(n * H * W, dtype=bool)])
    Ha = Hf[np.ix_(act, act)] + np.diag(np.r_[opts.lm_lambda * np.diag(Hf)[:15 * n][act[:15 * n]],
                                            np.full(n * H * W, opts.depth_eta)])
    sc = 1.0 / np.sqrt(np.diag(Ha))
    kappa = np.linalg.cond(Ha * sc[:, None] * sc[None, :])
    tol = max(1e-10, 100 * kappa * np.finfo(float).eps)
    print("kappa", kappa, "tol", tol)
    assert tol < 1e-2
    for c in range(15):
        ref = np.abs(dxi_d[:, c]).max()
        assert np.abs(dxi[:, c] - dxi_d[:, c]).max() <= tol * ref + 1e-300, c
    assert np.abs(dd - dd_d).max() <= tol * np.abs(dd_d).max()
    act = ne.active_mask(n, opts)
    assert np.all(dxi[~ne.active_mask(n, opts)] == 0)


def test_blocks_match_dense_hessian():
    p, cam, st, gr = _tiny(n_kf=3, H=3, W=4, k_out=2)
    opts = ne.Options()
    neq = ne.linearize(cam, st, gr, opts)
    H, g = dense.full_system(cam, st, gr, opts)
    nx = 15 * 3
    assert np.allclose(neq.B, H[:nx, :nx], rtol=1e-12, atol=1e-9 * np.abs(H).max())
    assert np.allclose(neq.w_xi, g[:nx], rtol=1e-12, atol=1e-9 * np.abs(g[:nx]).max())
    assert np.allclose(neq.C.ravel(), np.diag(H[nx:, nx:]), rtol=1e-12)
    # C is diagonal: each vision term touches one depth
    off = H[nx:, nx:] - np.diag(np.diag(H[nx:, nx:]))
    assert np.abs(off).max() == 0.0
    assert np.allclose(neq.w_d.ravel(), g[nx:], rtol=1e-12, atol=1e-12)
    # E blocks
    HW = 12
    for i, (T, Ei) in neq.E.items():
        for t, kf in enumerate(T):
            blk = H[15 * kf:15 * kf + 6, nx + i * HW:nx + (i + 1) * HW]
            assert np.allclose(Ei[t], blk, rtol=1e-12, atol=1e-12)
    # symmetric positive semi-definite
    assert np.allclose(H, H.T, rtol=1e-12, atol=1e-12 * np.abs(H).max())
    ev = np.linalg.eigvalsh(H / np.abs(H).max())
    assert ev.min() > -1e-12


def test_cholesky_matches_numpy():
    rng = np.random.default_rng(2)
    A = rng.normal(size=(40, 40))
    S = A @ A.T + 40 * np.eye(40)
    assert np.allclose(ne.cholesky(S), np.linalg.cholesky(S), atol=1e-12)
    x = ne.solve_spd(S, np.arange(40.0))
    assert np.allclose(S @ x, np.arange(40.0), atol=1e-10)
    S[5, 5] = -1.0
    with pytest.raises(ne.NotPositiveDefinite):
        ne.cholesky(S)


def test_noiseless_convergence_to_ground_truth():
    cfg = synth.config_small()
    cfg.noiseless = True
    cfg.zero_bias = True
    p = synth.make_problem(cfg, 1)
    cam, st, gr = osolve.from_problem(p, exact_targets=True)
    opts = ne.Options(lm_lambda=0.0, depth_eta=0.0)
    F0, _ = osolve.cost(cam, st, gr, opts)
    st, reps = osolve.solve(cam, st, gr, opts, 7)
    gt = osolve.state_from_arrays(p.pose_gt, p.vel_gt, p.bias_gt, p.invdepth_gt)
    assert reps[-1]["cost_after"] <= 1e-20 * F0
    assert np.abs(st.p - gt.p).max() < 1e-9
    assert max(np.abs(so3.Log(a.T @ b)).max() for a, b in zip(st.R, gt.R)) < 1e-9
    assert np.abs(st.v - gt.v).max() < 1e-9
    assert np.abs(st.b - gt.b).max() < 1e-9
    assert np.abs(st.d / gt.d - 1).max() < 1e-9


def test_noiseless_convergence_with_bias_linearisation_point_at_truth():
    """Nonzero constant true bias, factors linearised at it, solver starting
    from zero bias: the truth is still the exact minimiser (F = 0)."""
    cfg = synth.tiny_config(n_kf=5, H=12, W=16, k_out=3, noiseless=True)
    p = synth.make_problem(cfg, 3, bias_hat_mode="gt")
    cam, st, gr = osolve.from_problem(p, exact_targets=True)
    opts = ne.Options(lm_lambda=0.0, depth_eta=0.0)
    st, reps = osolve.solve(cam, st, gr, opts, 8)
    assert reps[-1]["cost_after"] < 1e-18 * reps[0]["cost_before"]
    assert np.abs(st.b - p.bias_gt).max() < 1e-8


def test_noisy_solve_reaches_stationary_point():
    """Pure Gauss-Newton on a noisy problem drives the gradient J^T W r to its
    rounding floor (a wrong Jacobian block would stall it far above)."""
    p = synth.make_problem(synth.tiny_config(n_kf=5, H=8, W=10, k_out=3), 4)
    cam, st, gr = osolve.from_problem(p)
    opts = ne.Options(lm_lambda=0.0, depth_eta=0.0, bias_fixed=True)
    g0 = None
    for _ in range(7):
        neq = ne.linearize(cam, st, gr, opts)
        act = ne.active_mask(5, opts).ravel()
        gn = np.linalg.norm(np.concatenate([neq.w_xi[act], neq.w_d.ravel()]))
        g0 = gn if g0 is None else g0
        st, _ = osolve.step(cam, st, gr, opts)
    assert gn < 1e-6 * g0


def test_gauge_yaw_translation_covariance():
    """Rotating the whole problem about gravity and shifting it moves the
    world-frame increments (dp, dv) by the same rotation and leaves the body-
    frame ones (dtheta, db) and the depths unchanged."""
    p = synth.make_problem(synth.tiny_config(n_kf=4, H=6, W=8, k_out=2), 8)
    cam, st, gr = osolve.from_problem(p)
    opts = ne.Options()
    _, rep = osolve.step(cam, st, gr, opts)
    Q = so3.Exp(np.array([0.0, 0.0, 0.7]))
    t = np.array([1.0, -2.0, 0.5])
    st2 = ne.State(R=np.einsum("ab,nbc->nac", Q, st.R), p=st.p @ Q.T + t, v=st.v @ Q.T,
                   b=st.b.copy(), d=st.d.copy())
    _, rep2 = osolve.step(cam, st2, gr, opts)
    d1, d2 = rep["dxi"], rep2["dxi"]
    # the two solves see differently rounded inputs of an ill-conditioned system
    # (accelerometer bias is weakly observable in a 0.3 s window): agreement per
    # group to 1e-5 of that group's size; a frame or sign error is O(1)
    for a, b, rotate in ((0, 3, False), (3, 6, True), (6, 9, True), (9, 15, False)):
        want = d1[:, a:b] @ Q.T if rotate else d1[:, a:b]
        assert np.abs(d2[:, a:b] - want).max() < 1e-5 * np.abs(want).max(), (a, b)
    assert np.abs(rep2["dd"] - rep["dd"]).max() < 1e-5 * np.abs(rep["dd"]).max()
    assert rep2["cost_before"] == pytest.approx(rep["cost_before"], rel=1e-12)


def test_step_cost_matches_cost_function():
    p = synth.make_problem(synth.tiny_config(n_kf=3, H=5, W=6, k_out=2), 6)
    cam, st, gr = osolve.from_problem(p)
    opts = ne.Options()
    new, rep = osolve.step(cam, st, gr, opts)
    assert rep["cost_before"] == pytest.approx(osolve.cost(cam, st, gr, opts)[0], rel=1e-13)
    assert rep["cost_after"] < rep["cost_before"]

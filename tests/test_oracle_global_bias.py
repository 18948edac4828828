"""One IMU bias shared by every keyframe of the window (Table 6 (f), the
"single global bias" ablation) in the oracle.

Pins: the Schur step of the folded normal equations equals the dense damped
solve in which each inertial factor's bias columns are summed into the shared
unknown's column (the two paths share no folding code); every keyframe's bias
moves by the same increment; the random-walk residual of equal biases drops
out (the folded step does not change when its information is scaled); and
Gauss-Newton from zero biases recovers a constant true bias and the poses on
noiseless data."""
import numpy as np
import pytest

from oracle import dense, imu, normal_eq as ne, so3, solve
from paper_2512_02293_amd import synth


@pytest.mark.parametrize("lam,eta", [(1e-4, 1e-8), (1e-3, 1e-4)])
def test_schur_step_equals_dense_with_summed_bias_columns(lam, eta):
    prob = synth.make_problem(synth.tiny_config(n_kf=4, H=4, W=5, k_out=2), 21)
    cam, st, gr = solve.from_problem(prob)
    st.b[:] = np.array([0.004, -0.003, 0.002, 0.03, -0.02, 0.05])      # one bias for all keyframes
    opts = ne.Options(lm_lambda=lam, depth_eta=eta, bias_global=True)
    _, rep = solve.step(cam, st, gr, opts)
    dxi, dd = dense.dense_step(cam, st, gr, opts)
    assert np.abs(rep["dxi"] - dxi).max() < 1e-9 * max(np.abs(dxi).max(), 1.0)
    assert np.abs(rep["dd"].reshape(dd.shape) - dd).max() < 1e-9 * max(np.abs(dd).max(), 1.0)
    assert np.all(rep["dxi"][:, 9:15] == rep["dxi"][-1, 9:15])
    assert np.abs(rep["dxi"][-1, 9:15]).max() > 0.0
    # and it differs from the per-keyframe step
    _, rep2 = solve.step(cam, st, gr, ne.Options(lm_lambda=lam, depth_eta=eta))
    assert np.abs(rep2["dxi"][:, 9:15] - rep["dxi"][:, 9:15]).max() > 1e-6


def test_random_walk_term_drops_out():
    prob = synth.make_problem(synth.tiny_config(n_kf=4, H=4, W=5, k_out=2), 22)
    cam, st, gr = solve.from_problem(prob)
    st.b[:] = np.array([0.001, 0.002, -0.001, 0.01, 0.02, -0.03])
    opts = ne.Options(bias_global=True)
    _, rep = solve.step(cam, st, gr, opts)
    _, per_kf = solve.step(cam, st, gr, ne.Options())
    for P in gr.factors:
        P.cov_bias = P.cov_bias * 1e-3                   # 1000 x stiffer random walk
    _, rep2 = solve.step(cam, st, gr, opts)
    _, per_kf2 = solve.step(cam, st, gr, ne.Options())
    # equal up to the rounding of the cancelling random-walk blocks (their scale grew 1000 x) ...
    assert np.abs(rep2["dxi"] - rep["dxi"]).max() < 1e-6 * np.abs(rep["dxi"]).max()
    # ... while the per-keyframe step does move
    assert np.abs(per_kf2["dxi"] - per_kf["dxi"]).max() > 1e-3 * np.abs(per_kf["dxi"]).max()


def test_gauss_newton_recovers_a_constant_bias():
    cfg = synth.tiny_config(n_kf=5, H=10, W=12, noiseless=True)
    prob = synth.make_problem(cfg, 23, bias_hat_mode="gt")      # factors linearised at the true bias
    assert np.ptp(prob.bias_gt, axis=0).max() == 0.0 and np.abs(prob.bias_gt).max() > 0
    cam, st, gr = solve.from_problem(prob, exact_targets=True)
    opts = ne.Options(lm_lambda=0.0, depth_eta=1e-12, bias_global=True)
    for _ in range(10):
        st, _ = solve.step(cam, st, gr, opts)
    assert np.abs(st.b - prob.bias_gt).max() < 1e-7
    assert np.abs(st.p - prob.pose_gt[:, :3]).max() < 1e-7
    Rgt = np.stack([so3.quat_to_R(q) for q in prob.pose_gt[:, 3:]])
    assert max(np.linalg.norm(so3.Log(a.T @ b)) for a, b in zip(st.R, Rgt)) < 1e-7

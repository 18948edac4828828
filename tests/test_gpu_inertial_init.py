"""IMU initialisation stage 2 (vi_inertial_init_solve) against the FP64 oracle,
through the C ABI.

Both sides take the same factors (the oracle's preintegration uploaded as
vi_preint records) and the same initial state, and compute in FP64; the GPU
solves the damped normal equations by a block Cholesky of their arrowhead
structure, the oracle by numpy.linalg.solve on the dense matrix, so results
differ by rounding amplified by the conditioning of H.  Bars: one step from the
initial state within 1e-7 relative per unknown group; converged states within
1e-7; on noiseless data both reach the truth (1e-9); cost traces within 1e-9
relative (before convergence; at convergence within 1e-12 of the first cost).
"""
import numpy as np
import pytest

from oracle import inertial_init as oi
from oracle import preint
from oracle.so3 import Log, quat_to_R
from paper_2512_02293_amd import synth

pytestmark = pytest.mark.gpu
G_I = np.array([0.0, 0.0, -9.81])


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2512_02293_amd import binding
    assert torch.cuda.is_available()
    c = binding.Context(0)
    yield c
    c.close()


def _record(P):
    return np.concatenate([[P.dt], P.dR.ravel(), P.dv, P.dp, P.J_rot.ravel(), P.J_vel.ravel(), P.J_pos.ravel(),
                           P.cov.ravel(), P.bias_hat, P.cov_bias])


def _problem(n_kf, seed, noiseless=False, mode="zero", pose_noise=(0.0, 0.0)):
    ip = synth.make_inertial_init_problem(synth.tiny_config(n_kf=n_kf, noiseless=noiseless), seed,
                                          bias_hat_mode=mode, pose_noise=pose_noise)
    fs = preint.preintegrate_all(ip.imu_off, ip.gyro, ip.accel, ip.imu_dt, ip.bias_hat, ip.noise)
    R = np.stack([quat_to_R(q) for q in ip.pose_vis[:, 3:7]])
    return ip, fs, R


def _upload(ip, fs, iters):
    import torch
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda:0")
    N = ip.pose_vis.shape[0]
    return {"pose_vis": dev(ip.pose_vis), "imu": dev(np.stack([_record(P) for P in fs])),
            "vel_vis": dev(np.zeros((N, 3))), "bias": dev(np.zeros((N, 6))), "rot_wg": dev([0, 0, 0, 1.0]),
            "log_scale": dev([0.0]), "cost": dev(np.zeros(iters + 1))}


def _zero(N):
    return oi.InitState(np.eye(3), 0.0, np.zeros((N, 3)), np.zeros((N, 6)))


def _compare(q, st, tol, label):
    R = quat_to_R(q["rot_wg"].cpu().numpy())
    errs = {"R_wg": float(np.linalg.norm(Log(R.T @ st.R_wg))),
            "s": abs(float(q["log_scale"].item()) - st.s) / max(abs(st.s), 1e-300),
            "v": float(np.linalg.norm(q["vel_vis"].cpu().numpy() - st.v_vis) / np.linalg.norm(st.v_vis)),
            "b_g": float(np.linalg.norm(q["bias"].cpu().numpy()[:, :3] - st.b[:, :3]) / np.linalg.norm(st.b[:, :3])),
            "b_a": float(np.linalg.norm(q["bias"].cpu().numpy()[:, 3:] - st.b[:, 3:]) / np.linalg.norm(st.b[:, 3:]))}
    print(label, {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= tol, (k, v)


def test_one_step_matches_oracle(ctx):
    ip, fs, R = _problem(16, 5, pose_noise=(2e-4, 0.01))
    q = _upload(ip, fs, 1)
    ctx.inertial_init_solve([q], iters=1)
    st, costs = oi.solve(R, ip.pose_vis[:, :3], _zero(16), fs, G_I, iters=1)
    _compare(q, st, 1e-7, "one step")
    assert q["cost"].cpu().numpy()[0] == pytest.approx(costs[0], rel=1e-10)


def test_noiseless_recovery_matches_truth(ctx):
    ip, fs, R = _problem(16, 3, noiseless=True, mode="gt")
    q = _upload(ip, fs, 10)
    ctx.inertial_init_solve([q], iters=10)
    truth = oi.InitState(ip.R_wg, ip.s, ip.v_vis, ip.b)
    g_gpu = quat_to_R(q["rot_wg"].cpu().numpy()) @ G_I
    assert np.linalg.norm(np.cross(g_gpu, ip.R_wg @ G_I)) / (G_I @ G_I) < 1e-9
    assert abs(q["log_scale"].item() - ip.s) < 1e-9
    np.testing.assert_allclose(q["vel_vis"].cpu().numpy(), truth.v_vis, atol=1e-9)
    np.testing.assert_allclose(q["bias"].cpu().numpy(), truth.b, atol=1e-9)
    _, costs = oi.solve(R, ip.pose_vis[:, :3], _zero(16), fs, G_I, iters=10)
    c = q["cost"].cpu().numpy()
    np.testing.assert_allclose(c[:4], costs[:4], rtol=1e-9)
    assert c[-1] < 1e-12 * c[0]


def test_batch_of_sizes_matches_oracle(ctx):
    """Problems of 3, 5, 16 and 32 keyframes in one call, 15 damped iterations
    each (lambda = 1e-6: with 3 keyframes the undamped system is singular)."""
    cases = [(3, 11), (5, 12), (16, 13), (32, 14)]
    probs = [_problem(n, s, pose_noise=(2e-4, 0.01)) for n, s in cases]
    qs = [_upload(ip, fs, 15) for ip, fs, _ in probs]
    ctx.inertial_init_solve(qs, lm_lambda=1e-6, iters=15)
    for (n, _), (ip, fs, R), q in zip(cases, probs, qs):
        st, costs = oi.solve(R, ip.pose_vis[:, :3], _zero(n), fs, G_I, iters=15, lm_lambda=1e-6)
        _compare(q, st, 1e-7, f"N={n}, 15 iterations")
        np.testing.assert_allclose(q["cost"].cpu().numpy(), costs, rtol=1e-8)


def test_errors_leave_the_state(ctx):
    import torch
    from paper_2512_02293_amd import binding
    ip, fs, R = _problem(6, 21)
    q = _upload(ip, fs, 3)
    rec = q["imu"].cpu().numpy()
    rec[2, -6:] = 0.0                    # a factor without bias random-walk variance
    q["imu"] = torch.as_tensor(rec, device="cuda:0")
    before = {k: v.clone() for k, v in q.items()}
    with pytest.raises(binding.ViError, match="ENOTPD"):
        ctx.inertial_init_solve([q], iters=3)
    for k in ("vel_vis", "bias", "rot_wg", "log_scale"):
        assert torch.equal(q[k], before[k])
    big = _upload(*_problem(33, 1)[:2], 1)
    with pytest.raises(binding.ViError, match="EINVAL"):
        ctx.inertial_init_solve([big], iters=1)


def test_zero_iterations_report_the_initial_cost_and_keep_the_state(ctx):
    ip, fs, R = _problem(8, 31, pose_noise=(2e-4, 0.01))
    q = _upload(ip, fs, 0)
    before = {k: v.clone() for k, v in q.items()}
    ctx.inertial_init_solve([q], iters=0)
    c0 = oi.cost(R, ip.pose_vis[:, :3], _zero(8), fs, G_I)
    assert q["cost"].cpu().numpy()[0] == pytest.approx(c0, rel=1e-12)
    import torch
    for k in ("vel_vis", "bias", "log_scale"):
        assert torch.equal(q[k], before[k])
    np.testing.assert_allclose(quat_to_R(q["rot_wg"].cpu().numpy()), np.eye(3), atol=1e-15)

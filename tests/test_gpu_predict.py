"""New-keyframe prediction from preintegration (vi_predict_keyframe) against
the FP64 oracle, through the C ABI.

Both sides compute in FP64 from the same inputs, so the predicted states agree
to rounding (bound 1e-12 relative, rotations compared as matrices, since q and
-q are the same rotation); the fallback decision and the copied states are
compared exactly, on factors whose covariance trace is not within 1e-9 of the
threshold (where the decision is unambiguous).  Factors are the oracle's own
preintegration, uploaded as vi_preint records; an end-to-end case also runs the
library's preintegration first (bound 1e-9: the two preintegrations differ by
rounding)."""
import dataclasses

import numpy as np
import pytest

from oracle import predict as op
from oracle import preint
from oracle.so3 import Log, quat_to_R
from paper_2512_02293_amd import synth

pytestmark = pytest.mark.gpu


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


def _cases(n_windows=6, seed0=50):
    """Windows with paper-like keyframe gaps (0.1-3 s at 200 Hz): previous
    states = the noisy initial estimates with perturbed biases."""
    probs, facs, prev = [], [], []
    rng = np.random.default_rng(seed0)
    for w in range(n_windows):
        cfg = dataclasses.replace(synth.tiny_config(n_kf=8), gap_range=(20, 600))
        p = synth.make_problem(cfg, seed0 + w)
        fs = preint.preintegrate_all(p.imu_off, p.gyro, p.accel, p.imu_dt, p.bias_hat, p.noise)
        for f, P in enumerate(fs):
            b = p.bias[f] + rng.normal(0, [0.002] * 3 + [0.02] * 3)
            prev.append((p.pose[f], p.vel[f], b))
            facs.append(P)
        probs.append(p)
    return probs, facs, prev


def _compare(pose, vel, bias, used, facs, prev, g, tau, tol):
    n_used = 0
    for k, (P, (q0, v0, b0)) in enumerate(zip(facs, prev)):
        rq, rv, rb, ru = op.predict_pose7(q0, v0, b0, P, g, tau)
        assert bool(used[k]) == ru, k
        if not ru:
            np.testing.assert_array_equal(pose[k], q0)
            np.testing.assert_array_equal(vel[k], v0)
            np.testing.assert_array_equal(bias[k], b0)
            continue
        n_used += 1
        ang = np.linalg.norm(Log(quat_to_R(pose[k, 3:7]).T @ quat_to_R(rq[3:7])))
        assert ang <= tol, (k, ang)
        assert abs(np.linalg.norm(pose[k, 3:7]) - 1.0) < 1e-14
        assert np.linalg.norm(pose[k, :3] - rq[:3]) <= tol * (1.0 + np.linalg.norm(rq[:3])), k
        assert np.linalg.norm(vel[k] - rv) <= tol * (1.0 + np.linalg.norm(rv)), k
        np.testing.assert_array_equal(bias[k], rb)
    return n_used


def test_predict_matches_oracle(ctx):
    import torch
    probs, facs, prev = _cases()
    g = probs[0].gravity
    traces = np.array([op.inertial_cov_trace(P) for P in facs])
    assert np.all(np.abs(traces - op.TAU_INIT) > 1e-9 * op.TAU_INIT)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")
    imu = dev(np.stack([_record(P) for P in facs]))
    q0, v0, b0 = (dev(np.stack([x[i] for x in prev])) for i in range(3))
    pose, vel, bias, used = ctx.predict_keyframe(q0, v0, b0, imu, g)
    torch.cuda.synchronize()
    used = used.cpu().numpy()
    n_used = _compare(pose.cpu().numpy(), vel.cpu().numpy(), bias.cpu().numpy(), used, facs, prev, g, op.TAU_INIT,
                      1e-12)
    print(f"{len(facs)} predictions, {n_used} from preintegration, {len(facs) - n_used} fallbacks", flush=True)
    assert 0 < n_used < len(facs)
    # in place gives the same
    ctx.predict_keyframe(q0, v0, b0, imu, g, pose_new=q0, vel_new=v0, bias_new=b0)
    torch.cuda.synchronize()
    assert torch.equal(q0, pose) and torch.equal(v0, vel) and torch.equal(b0, bias)


def test_predict_thresholds_and_nan(ctx):
    import torch
    probs, facs, prev = _cases(n_windows=2, seed0=90)
    g = probs[0].gravity
    recs = np.stack([_record(P) for P in facs])
    recs[3, 1 + 9 + 3 + 3 + 9 + 18 + 18] = np.nan       # cov[0][0] of factor 3
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")
    imu = dev(recs)
    q0, v0, b0 = (dev(np.stack([x[i] for x in prev])) for i in range(3))
    for tau, expect in ((0.0, 0), (np.inf, 1)):
        _, _, _, used = ctx.predict_keyframe(q0, v0, b0, imu, g, tau=tau)
        u = used.cpu().numpy()
        assert u[3] == 0                                  # a NaN trace always falls back
        assert np.all(np.delete(u, 3) == expect)
    _, _, _, used = ctx.predict_keyframe(q0[:0], v0[:0], b0[:0], imu[:0], g)   # n = 0
    torch.cuda.synchronize()


def test_predict_end_to_end_after_library_preintegration(ctx):
    import torch
    from paper_2512_02293_amd import binding
    cfg = dataclasses.replace(synth.tiny_config(n_kf=10), gap_range=(20, 600))
    p = synth.make_problem(cfg, 123)
    dp = binding.DeviceProblem(p)
    imu = ctx.imu_preintegrate(dp.off, dp.gyro, dp.accel, dp.imu_dt, dp.bias_hat, dp.noise)
    facs = preint.preintegrate_all(p.imu_off, p.gyro, p.accel, p.imu_dt, p.bias_hat, p.noise)
    traces = np.array([op.inertial_cov_trace(P) for P in facs])
    assert np.all(np.abs(traces - op.TAU_INIT) > 1e-9 * op.TAU_INIT)
    prev = [(p.pose[f], p.vel[f], p.bias[f]) for f in range(p.n_kf - 1)]
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")
    q0, v0, b0 = (dev(np.stack([x[i] for x in prev])) for i in range(3))
    pose, vel, bias, used = ctx.predict_keyframe(q0, v0, b0, imu, p.gravity)
    torch.cuda.synchronize()
    _compare(pose.cpu().numpy(), vel.cpu().numpy(), bias.cpu().numpy(), used.cpu().numpy(), facs, prev, p.gravity,
             op.TAU_INIT, 1e-9)


def test_predict_host_errors(ctx):
    import torch
    from paper_2512_02293_amd import binding
    probs, facs, prev = _cases(n_windows=1, seed0=7)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")
    imu = dev(np.stack([_record(P) for P in facs]))
    q0, v0, b0 = (dev(np.stack([x[i] for x in prev])) for i in range(3))
    with pytest.raises(binding.ViError, match="EINVAL"):
        ctx.predict_keyframe(q0, v0, b0, imu, probs[0].gravity, tau=-1.0)
    with pytest.raises(binding.ViError, match="EINVAL"):
        ctx.predict_keyframe(q0, v0, b0, imu, probs[0].gravity, tau=float("nan"))
    buf = torch.zeros(7 * len(facs) + 7, dtype=torch.float64, device="cuda:0")
    a = buf[:7 * len(facs)].view(-1, 7)
    a.copy_(q0)
    shifted = buf[7:].view(-1, 7)                        # overlaps its input, not equal to it
    with pytest.raises(binding.ViError, match="EINVAL"):
        ctx.predict_keyframe(a, v0, b0, imu, probs[0].gravity, pose_new=shifted)

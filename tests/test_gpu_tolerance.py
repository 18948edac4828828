"""Tolerance stop of the Gauss-Newton iterations (vi_ctx_set_tolerance).

A window is frozen before step t (t >= 1) when F_{t-1} - F_t <= tol F_{t-1}.
Checked against the solver without the stop, on the same inputs: each window
stops at the first step where the plain cost trace meets the rule, its costs
up to there are the plain ones and stay flat afterwards, and its final state
is the state after that many plain steps (a single-window solve, so equal to
the reduction rounding between batch and single-window launches, 1e-12); the
other windows of the batch go on.  The oracle is not involved: the stopping
rule is the library's own (the paper gives none), and the steps it keeps are
the ones the parity tests check against the oracle.
"""
import numpy as np
import pytest

from oracle import normal_eq as ne
from paper_2512_02293_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2512_02293_amd import binding
    assert torch.cuda.is_available()
    c = binding.Context(0)
    yield c
    c.set_tolerance(0.0)
    c.close()


def _bopts():
    from paper_2512_02293_amd import binding
    o = ne.Options()
    return binding.make_opts(n_fixed=o.n_fixed, use_imu=o.use_imu, bias_fixed=o.bias_fixed, lm_lambda=o.lm_lambda,
                             depth_eta=o.depth_eta, z_min=o.z_min, d_min=o.d_min)


def _state(dp):
    return [t.cpu().numpy().copy() for t in (dp.pose, dp.vel, dp.bias, dp.invdepth)]


def _close(a, b, rtol):
    for x, y in zip(a, b):
        scale = max(np.abs(y).max(), 1e-300)
        assert np.abs(x - y).max() <= rtol * scale, (np.abs(x - y).max(), scale)


def _expected_stop(costs, tol, iters):
    for t in range(1, iters):
        if not (costs[t - 1] - costs[t] > tol * costs[t - 1]):
            return t
    return iters


def test_tolerance_stop_per_window_in_a_batch(ctx):
    import torch
    from paper_2512_02293_amd import binding
    iters, n_win, tol = 10, 4, 1e-4
    probs = [synth.make_problem(synth.config_batched_window(w), 4100 + w) for w in range(n_win)]
    bopts = _bopts()
    ctx.set_autotune(False)
    dps = [binding.DeviceProblem(p) for p in probs]
    imus = [ctx.imu_preintegrate(d.off, d.gyro, d.accel, d.imu_dt, d.bias_hat, d.noise) for d in dps]
    ws = torch.empty(ctx.workspace_size_batched(dps, bopts), dtype=torch.uint8, device="cuda:0")
    ctx.set_tolerance(0.0)
    plain = ctx.solve_batched(dps, imus, bopts, iters, ws, costs=True)
    expected = [_expected_stop(plain[w]["costs"], tol, iters) for w in range(n_win)]
    print("plain traces", [np.array2string(np.asarray(r["costs"]), precision=6) for r in plain])
    print("expected stops", expected, flush=True)
    assert all(r["iters_done"] == iters for r in plain)
    assert any(e < iters for e in expected)

    for dp in dps:
        dp.reset_state()
    ctx.set_tolerance(tol)
    reps = ctx.solve_batched(dps, imus, bopts, iters, ws, costs=True)
    ctx.set_tolerance(0.0)
    frozen = [_state(dp) for dp in dps]
    for w, (dp, imu) in enumerate(zip(dps, imus)):
        k = expected[w]
        c = np.asarray(reps[w]["costs"])
        assert reps[w]["iters_done"] == k, (w, reps[w]["iters_done"], k)
        np.testing.assert_allclose(c[:k + 1], plain[w]["costs"][:k + 1], rtol=1e-12)
        np.testing.assert_allclose(c[k:], c[k], rtol=1e-12)
        assert reps[w]["cost_after"] == pytest.approx(c[k], rel=1e-12)
        dp.reset_state()
        wsw = torch.empty(ctx.workspace_size(dp.cam, dp.pose.shape[0], dp.ii, dp.jj, bopts), dtype=torch.uint8,
                          device="cuda:0")
        rep = ctx.solve(dp.cam, dp.pose, dp.vel, dp.bias, dp.invdepth, dp.ii, dp.jj, dp.target, dp.weight, imu,
                        bopts, k, wsw, costs=True)
        assert rep["iters_done"] == k
        _close(frozen[w], _state(dp), 1e-12)


def test_tolerance_stop_single_window_and_errors(ctx):
    import torch
    from paper_2512_02293_amd import binding
    iters, tol = 8, 1e-4
    prob = synth.make_problem(synth.config_small(), 7)
    bopts = _bopts()
    ctx.set_autotune(False)
    dp = binding.DeviceProblem(prob)
    imu = ctx.imu_preintegrate(dp.off, dp.gyro, dp.accel, dp.imu_dt, dp.bias_hat, dp.noise)
    ws = torch.empty(ctx.workspace_size(dp.cam, dp.pose.shape[0], dp.ii, dp.jj, bopts), dtype=torch.uint8,
                     device="cuda:0")
    solve = lambda n: ctx.solve(dp.cam, dp.pose, dp.vel, dp.bias, dp.invdepth, dp.ii, dp.jj, dp.target, dp.weight,
                                imu, bopts, n, ws, costs=True)
    ctx.set_tolerance(0.0)
    plain = solve(iters)
    k = _expected_stop(plain["costs"], tol, iters)
    print("plain trace", plain["costs"], "expected stop", k, flush=True)
    assert k < iters
    dp.reset_state()
    ctx.set_tolerance(tol)
    rep = solve(iters)
    ctx.set_tolerance(0.0)
    frozen = _state(dp)
    assert rep["iters_done"] == k
    np.testing.assert_allclose(rep["costs"][:k + 1], plain["costs"][:k + 1], rtol=1e-12)
    dp.reset_state()
    ref = solve(k)
    _close(frozen, _state(dp), 1e-12)
    assert rep["cost_after"] == pytest.approx(ref["cost_after"], rel=1e-12)
    for bad in (-1e-3, 1.0, float("nan")):
        with pytest.raises(binding.ViError, match="EINVAL"):
            ctx.set_tolerance(bad)


def test_tolerance_stop_after_the_warm_start(ctx):
    """vi_ba_solve_warm with the stop: the warm start is unchanged (the same
    corrections kept), and each window's Gauss-Newton part stops where the
    trace of the same call without the stop meets the rule."""
    import torch
    from paper_2512_02293_amd import binding, warmstart
    iters, tol = 8, 1e-6
    probs = warmstart.eval_windows(4)
    opts = warmstart.study_opts()
    dps = [binding.DeviceProblem(p) for p in probs]
    imus = [ctx.imu_preintegrate(d.off, d.gyro, d.accel, d.imu_dt, d.bias_hat, d.noise) for d in dps]
    ws = torch.empty(ctx.warm_start_workspace_size(dps, opts), dtype=torch.uint8, device="cuda:0")
    theta = torch.as_tensor(np.ascontiguousarray(np.load(warmstart.PARAMS_FILE)), dtype=torch.float32,
                            device="cuda:0")
    ctx.set_tolerance(0.0)
    plain = ctx.solve_warm(dps, imus, opts, theta, iters, ws, costs=True)
    expected = [_expected_stop(r["costs"], tol, iters) for r in plain]
    print("expected stops", expected, flush=True)
    assert any(k < iters for k in expected)
    for d in dps:
        d.reset_state()
    ctx.set_tolerance(tol)
    got = ctx.solve_warm(dps, imus, opts, theta, iters, ws, costs=True)
    ctx.set_tolerance(0.0)
    for r, g, k in zip(plain, got, expected):
        assert g["accepted"] == r["accepted"]
        assert g["iters_done"] == k, (g["iters_done"], k)
        np.testing.assert_allclose(g["costs"][:k + 1], r["costs"][:k + 1], rtol=1e-12)
        np.testing.assert_allclose(g["costs"][k:], g["costs"][k], rtol=1e-12)

"""One context serving several problems in turn.

The library keeps the window table and the IMU sample offsets it last sent to
the device and sends them again only when they change; these tests alternate
problems of the same shapes (so the plan is reused) with different tensors and
different offsets, and check each call against the oracle or a fresh context.
"""
import numpy as np
import pytest

from oracle import preint as opre
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


def test_preintegration_offsets_change_between_calls(ctx):
    """Same number of factors, different samples per factor: A, B, A again."""
    from paper_2512_02293_amd import binding
    cfg = synth.SceneConfig(n_kf=6, H=7, W=9, k_out=2, gap_range=(5, 40))
    pa, pb = synth.make_problem(cfg, 11), synth.make_problem(cfg, 12)
    assert len(pa.imu_off) == len(pb.imu_off) and not np.array_equal(pa.imu_off, pb.imu_off)
    for prob in (pa, pb, pa):
        dp = binding.DeviceProblem(prob)
        got = ctx.imu_preintegrate(dp.off, dp.gyro, dp.accel, dp.imu_dt, dp.bias_hat, dp.noise).cpu().numpy()
        ref = opre.preintegrate_all(prob.imu_off, prob.gyro, prob.accel, prob.imu_dt, prob.bias_hat, prob.noise)
        for f, P in enumerate(ref):
            g = got[f]
            fields = [(g[0:1], [P.dt]), (g[1:10], P.dR.ravel()), (g[10:13], P.dv), (g[13:16], P.dp),
                      (g[16:25], P.J_rot.ravel()), (g[25:43], P.J_vel.ravel()), (g[43:61], P.J_pos.ravel()),
                      (g[61:142], P.cov.ravel())]
            for k, (a, b) in enumerate(fields):
                b = np.asarray(b)
                assert np.abs(a - b).max() <= 1e-11 * max(np.abs(b).max(), 1e-300), (f, k)


def _one_step(c, prob, autotune):
    import torch
    from paper_2512_02293_amd import binding
    c.set_autotune(autotune)
    dp = binding.DeviceProblem(prob)
    imu = c.imu_preintegrate(dp.off, dp.gyro, dp.accel, dp.imu_dt, dp.bias_hat, dp.noise)
    opts = binding.make_opts()
    ws = torch.empty(c.workspace_size(dp.cam, prob.n_kf, dp.ii, dp.jj, opts), dtype=torch.uint8, device="cuda:0")
    dxi = torch.zeros((prob.n_kf, 15), dtype=torch.float64, device="cuda:0")
    dd = torch.zeros_like(dp.invdepth)
    c.solve(dp.cam, dp.pose, dp.vel, dp.bias, dp.invdepth, dp.ii, dp.jj, dp.target, dp.weight, imu, opts, 2, ws,
            dxi=dxi, dd=dd)
    return dxi.cpu().numpy(), dd.cpu().numpy(), dp.pose.cpu().numpy()


@pytest.mark.parametrize("autotune", [False, True])
def test_solve_alternating_problems_matches_fresh_context(ctx, autotune):
    """Two problems with the same edge pattern but their own tensors, solved
    A, B, A in one context, give what a fresh context gives for each: the
    same bits with the default tiling; with the autotuner, whose choice rests
    on timings and so may differ between contexts (a different summation
    order), within 1e-9, and A's two solves in the one context the same bits."""
    from paper_2512_02293_amd import binding
    cfg = synth.config_small()
    pa, pb = synth.make_problem(cfg, 21), synth.make_problem(cfg, 22)
    assert np.array_equal(pa.ii, pb.ii) and np.array_equal(pa.jj, pb.jj)
    got = [_one_step(ctx, p, autotune) for p in (pa, pb, pa)]
    want = {}
    for name, p in (("a", pa), ("b", pb)):
        fresh = binding.Context(0)
        try:
            want[name] = _one_step(fresh, p, autotune)
        finally:
            fresh.close()
    for g, name in zip(got, ("a", "b", "a")):
        for x, y in zip(g, want[name]):
            if autotune:
                assert np.abs(x - y).max() <= 1e-9 * max(np.abs(y).max(), 1e-300), name
            else:
                assert np.array_equal(x, y), name
    for x, y in zip(got[0], got[2]):
        assert np.array_equal(x, y)

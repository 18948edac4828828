"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: the required accuracy of the step is 1e-4 relative per group of
the pose, velocity and bias increments and 1e-3 on the inverse-depth
increments.  Both sides run in FP64 here and compute the same damped step up
to rounding order (measured 1e-13 .. 1e-10, printed), so the asserts are much
tighter, 1e-8 relative per group and on the inverse-depth increments, and a
dropped coupling or a mis-ordered update cannot hide below the required bar;
integer results (valid pixel counts, iterations done) agree exactly.
"""
import numpy as np
import pytest

from oracle import normal_eq as ne, preint as opre, so3
from oracle import solve as osolve
from paper_2512_02293_amd import synth

pytestmark = pytest.mark.gpu

GROUPS = {"dtheta": slice(0, 3), "dp": slice(3, 6), "dv": slice(6, 9), "dbg": slice(9, 12), "dba": slice(12, 15)}
FP64_TOL = 1e-8


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2512_02293_amd import binding
    assert torch.cuda.is_available()
    c = binding.Context(0)
    yield c
    c.close()


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)


def _opts_pair(**kw):
    from paper_2512_02293_amd import binding
    o = ne.Options(**kw)
    b = binding.make_opts(n_fixed=o.n_fixed, use_imu=o.use_imu, bias_fixed=o.bias_fixed, lm_lambda=o.lm_lambda,
                          depth_eta=o.depth_eta, z_min=o.z_min, d_min=o.d_min)
    return o, b


def _gpu_setup(ctx, prob):
    import torch
    from paper_2512_02293_amd import binding
    dp = binding.DeviceProblem(prob)
    imu = ctx.imu_preintegrate(dp.off, dp.gyro, dp.accel, dp.imu_dt, dp.bias_hat, dp.noise)
    return dp, imu


def _workspace(ctx, dp, bopts):
    import torch
    nb = ctx.workspace_size(dp.cam, dp.pose.shape[0], dp.ii, dp.jj, bopts)
    assert nb > 0
    return torch.empty(nb, dtype=torch.uint8, device="cuda:0")


def _load_state(dp, st):
    import torch
    dp.pose.copy_(torch.as_tensor(osolve.pose_array(st)))
    dp.vel.copy_(torch.as_tensor(st.v))
    dp.bias.copy_(torch.as_tensor(st.b))
    dp.invdepth.copy_(torch.as_tensor(st.d))


def _gpu_step(ctx, dp, imu, bopts, ws):
    import torch
    N = dp.pose.shape[0]
    dxi = torch.zeros((N, 15), dtype=torch.float64, device="cuda:0")
    dd = torch.zeros_like(dp.invdepth)
    rep = ctx.solve(dp.cam, dp.pose, dp.vel, dp.bias, dp.invdepth, dp.ii, dp.jj, dp.target, dp.weight, imu,
                    bopts, 1, ws, dxi=dxi, dd=dd)
    return rep, dxi.cpu().numpy(), dd.cpu().numpy()


def _compare_step(rep, dxi, dd, orep, tag):
    errs = {}
    for g, sl in GROUPS.items():
        ref = orep["dxi"][:, sl]
        if np.linalg.norm(ref) == 0:
            assert np.abs(dxi[:, sl]).max() == 0.0, (tag, g)
            continue
        errs[g] = _rel(dxi[:, sl], ref)
    errs["dd"] = _rel(dd.ravel(), orep["dd"].ravel())
    print(tag, {k: f"{v:.2e}" for k, v in errs.items()})
    for g in GROUPS:
        if g in errs:
            assert errs[g] <= FP64_TOL, (tag, g, errs[g])
    assert errs["dd"] <= FP64_TOL, (tag, errs["dd"])
    assert rep["n_valid"] == orep["n_valid"], tag
    assert rep["cost_before"] == pytest.approx(orep["cost_before"], rel=1e-9), tag
    assert rep["cost_after"] == pytest.approx(orep["cost_after"], rel=1e-9), tag


def test_library_is_native(ctx):
    from paper_2512_02293_amd import binding
    assert binding.load().vi_version().startswith(b"vi-ba-mi355x")


@pytest.mark.parametrize("cfg_name,seed", [("small", 1), ("ragged", 7)])
def test_preintegration_matches_oracle(ctx, cfg_name, seed):
    cfg = synth.config_small() if cfg_name == "small" else synth.SceneConfig(n_kf=6, H=7, W=9, k_out=2,
                                                                              gap_range=(5, 40))
    prob = synth.make_problem(cfg, seed)
    dp, imu = _gpu_setup(ctx, prob)
    got = imu.cpu().numpy()
    ref = opre.preintegrate_all(prob.imu_off, prob.gyro, prob.accel, prob.imu_dt, prob.bias_hat, prob.noise)
    for f, P in enumerate(ref):
        g = got[f]
        fields = [("dt", g[0:1], np.array([P.dt])), ("dR", g[1:10], P.dR.ravel()), ("dv", g[10:13], P.dv),
                  ("dp", g[13:16], P.dp), ("J_rot", g[16:25], P.J_rot.ravel()),
                  ("J_vel", g[25:43], P.J_vel.ravel()), ("J_pos", g[43:61], P.J_pos.ravel()),
                  ("cov", g[61:142], P.cov.ravel()), ("bias_hat", g[142:148], P.bias_hat),
                  ("cov_bias", g[148:154], P.cov_bias)]
        for name, a, b in fields:
            scale = max(np.abs(b).max(), 1e-300)
            assert np.abs(a - b).max() <= 1e-11 * scale, (f, name, np.abs(a - b).max(), scale)


def _single_step_case(ctx, prob, **optkw):
    oopts, bopts = _opts_pair(**optkw)
    cam, st, gr = osolve.from_problem(prob)
    dp, imu = _gpu_setup(ctx, prob)
    ws = _workspace(ctx, dp, bopts)
    rep, dxi, dd = _gpu_step(ctx, dp, imu, bopts, ws)
    new, orep = osolve.step(cam, st, gr, oopts)
    _compare_step(rep, dxi, dd, orep, f"N={prob.n_kf} E={prob.n_edges} {optkw}")
    # committed state
    R_gpu = np.stack([so3.quat_to_R(q) for q in dp.pose.cpu().numpy()[:, 3:]])
    ang = max(np.linalg.norm(so3.Log(a.T @ b)) for a, b in zip(R_gpu, new.R))
    assert ang <= FP64_TOL * max(np.abs(orep["dxi"][:, 0:3]).max(), 1e-12) + 1e-13
    assert np.abs(dp.invdepth.cpu().numpy() - new.d).max() <= FP64_TOL * np.abs(orep["dd"]).max()


def test_step_small_window(ctx):
    _single_step_case(ctx, synth.make_problem(synth.config_small(), 1))


def test_step_ragged_tiles(ctx):
    """Maps of 37x53 px: ragged tails in every pixel tiling; 6 edges per source."""
    cfg = synth.SceneConfig(n_kf=7, H=37, W=53, k_out=6)
    _single_step_case(ctx, synth.make_problem(cfg, 11))


@pytest.mark.parametrize("optkw", [
    dict(use_imu=False),
    dict(bias_fixed=True),
    dict(n_fixed=2, lm_lambda=1e-2, depth_eta=1e-4),
    dict(lm_lambda=0.0, depth_eta=0.0),
])
def test_step_option_variants(ctx, optkw):
    cfg = synth.SceneConfig(n_kf=6, H=24, W=32, k_out=4)
    _single_step_case(ctx, synth.make_problem(cfg, 3), **optkw)


def test_step_uneven_out_degree_and_gaps(ctx):
    cfg = synth.config_batched_window(5)
    prob = synth.make_problem(cfg, 4005)
    _single_step_case(ctx, prob)


@pytest.mark.parametrize("n_kf,loop_gap,seed", [(32, 20, 21), (16, 12, 22)])
def test_step_wide_band_small_system(ctx, n_kf, loop_gap, seed):
    """Windows with a few long-range edges solved by the one-workgroup
    Cholesky: 32 keyframes (480 x 480, a band of 14 tiles: more than the
    LDS-resident column buffers hold, so every updated tile goes through
    global memory) and 16 keyframes (240 x 240, a band of 7 tiles: the
    largest the LDS-resident buffers take)."""
    cfg = synth.SceneConfig(n_kf=n_kf, H=24, W=32, k_out=4, n_loop=4, loop_gap=loop_gap, gap_range=(15, 25))
    prob = synth.make_problem(cfg, seed)
    assert max(abs(int(a) - int(b)) for a, b in zip(prob.ii, prob.jj)) >= loop_gap
    _single_step_case(ctx, prob)


def test_step_sliding_window_full_size(ctx):
    """The 24-keyframe, 60x80, 288-edge window (the benchmarked shape)."""
    _single_step_case(ctx, synth.make_problem(synth.config_window(), 2))


def test_iterations_each_from_oracle_state(ctx):
    """Every iteration's increments, each step started from the oracle's own state."""
    prob = synth.make_problem(synth.config_small(), 1)
    oopts, bopts = _opts_pair()
    cam, st, gr = osolve.from_problem(prob)
    dp, imu = _gpu_setup(ctx, prob)
    ws = _workspace(ctx, dp, bopts)
    for it in range(4):
        _load_state(dp, st)
        rep, dxi, dd = _gpu_step(ctx, dp, imu, bopts, ws)
        st, orep = osolve.step(cam, st, gr, oopts)
        _compare_step(rep, dxi, dd, orep, f"iter {it}")


@pytest.mark.parametrize("which,iters", [("small", 4), ("window", 8)])
def test_graph_solve_matches_oracle_solve(ctx, which, iters):
    prob = synth.make_problem(synth.config_small() if which == "small" else synth.config_window(),
                              1 if which == "small" else 2)
    oopts, bopts = _opts_pair()
    cam, st, gr = osolve.from_problem(prob)
    dp, imu = _gpu_setup(ctx, prob)
    ws = _workspace(ctx, dp, bopts)
    rep = ctx.solve(dp.cam, dp.pose, dp.vel, dp.bias, dp.invdepth, dp.ii, dp.jj, dp.target, dp.weight, imu,
                    bopts, iters, ws, costs=True)
    assert rep["iters_done"] == iters
    ost, oreps = osolve.solve(cam, st, gr, oopts, iters)
    ocosts = [r["cost_before"] for r in oreps] + [oreps[-1]["cost_after"]]
    assert np.allclose(rep["costs"], ocosts, rtol=1e-6), (rep["costs"], ocosts)
    pose = dp.pose.cpu().numpy()
    R_gpu = np.stack([so3.quat_to_R(q) for q in pose[:, 3:]])
    ang = max(np.linalg.norm(so3.Log(a.T @ b)) for a, b in zip(R_gpu, ost.R))
    assert ang < 1e-8
    assert np.abs(pose[:, :3] - ost.p).max() < 1e-8
    assert np.abs(dp.vel.cpu().numpy() - ost.v).max() < 1e-7
    assert np.abs(dp.bias.cpu().numpy() - ost.b).max() < 1e-7
    assert np.abs(dp.invdepth.cpu().numpy() - ost.d).max() < 1e-7
    # replaying the cached graph from the same start gives the same result
    first = dp.pose.cpu().numpy().copy()
    dp.reset_state()
    rep2 = ctx.solve(dp.cam, dp.pose, dp.vel, dp.bias, dp.invdepth, dp.ii, dp.jj, dp.target, dp.weight, imu,
                     bopts, iters, ws, costs=True)
    assert np.array_equal(dp.pose.cpu().numpy(), first)
    assert np.array_equal(rep2["costs"], rep["costs"])


def test_eager_timed_run_matches_graph_run(ctx):
    prob = synth.make_problem(synth.config_small(), 1)
    _, bopts = _opts_pair()
    dp, imu = _gpu_setup(ctx, prob)
    ws = _workspace(ctx, dp, bopts)
    rep_g = ctx.solve(dp.cam, dp.pose, dp.vel, dp.bias, dp.invdepth, dp.ii, dp.jj, dp.target, dp.weight, imu,
                      bopts, 3, ws, costs=True)
    pose_g = dp.pose.cpu().numpy().copy()
    dp.reset_state()
    rep_e = ctx.solve(dp.cam, dp.pose, dp.vel, dp.bias, dp.invdepth, dp.ii, dp.jj, dp.target, dp.weight, imu,
                      bopts, 3, ws, costs=True, stage_ms=True)
    assert np.array_equal(dp.pose.cpu().numpy(), pose_g)
    assert np.array_equal(rep_e["costs"], rep_g["costs"])
    assert all(v >= 0 for v in rep_e["stage_ms"].values())
    assert rep_e["stage_ms"]["vis_gram_imu"] > 0


def test_noiseless_convergence_on_gpu(ctx):
    cfg = synth.config_small()
    cfg.noiseless = True
    cfg.zero_bias = True
    prob = synth.make_problem(cfg, 1)
    prob.target = prob.target64.astype(np.float32)
    _, bopts = _opts_pair(lm_lambda=0.0, depth_eta=0.0)
    dp, imu = _gpu_setup(ctx, prob)
    ws = _workspace(ctx, dp, bopts)
    rep = ctx.solve(dp.cam, dp.pose, dp.vel, dp.bias, dp.invdepth, dp.ii, dp.jj, dp.target, dp.weight, imu,
                    bopts, 7, ws, costs=True)
    # float32 targets leave ~1e-5 px of rounding: the cost falls by > 1e8 and the
    # state lands within float32 target rounding of the truth
    assert rep["costs"][-1] < 1e-8 * rep["costs"][0]
    assert np.abs(dp.pose.cpu().numpy()[:, :3] - prob.pose_gt[:, :3]).max() < 1e-5
    assert np.abs(dp.invdepth.cpu().numpy() / prob.invdepth_gt - 1).max() < 1e-4


def test_not_positive_definite_leaves_state_unchanged(ctx):
    """Zero weights, vision only, no damping: the reduced system is singular."""
    import torch
    from paper_2512_02293_amd import binding
    prob = synth.make_problem(synth.config_small(), 1)
    prob.weight = np.zeros_like(prob.weight)
    _, bopts = _opts_pair(use_imu=False, lm_lambda=0.0, depth_eta=0.0)
    dp, imu = _gpu_setup(ctx, prob)
    ws = _workspace(ctx, dp, bopts)
    before = [t.cpu().clone() for t in (dp.pose, dp.vel, dp.bias, dp.invdepth)]
    with pytest.raises(binding.ViError) as ei:
        ctx.solve(dp.cam, dp.pose, dp.vel, dp.bias, dp.invdepth, dp.ii, dp.jj, dp.target, dp.weight, imu,
                  bopts, 2, ws)
    assert ei.value.code == binding.VI_ENOTPD
    for a, t in zip(before, (dp.pose, dp.vel, dp.bias, dp.invdepth)):
        assert torch.equal(a, t.cpu())


def test_host_validation_errors(ctx):
    from paper_2512_02293_amd import binding
    prob = synth.make_problem(synth.config_small(), 1)
    _, bopts = _opts_pair()
    dp, imu = _gpu_setup(ctx, prob)
    ws = _workspace(ctx, dp, bopts)
    bad = dp.jj.copy()
    bad[3] = 99
    with pytest.raises(binding.ViError) as ei:
        ctx.solve(dp.cam, dp.pose, dp.vel, dp.bias, dp.invdepth, dp.ii, bad, dp.target, dp.weight, imu, bopts, 1, ws)
    assert ei.value.code == binding.VI_EINVAL
    self_loop = dp.jj.copy()
    self_loop[0] = dp.ii[0]
    with pytest.raises(binding.ViError) as ei:
        ctx.solve(dp.cam, dp.pose, dp.vel, dp.bias, dp.invdepth, dp.ii, self_loop, dp.target, dp.weight, imu,
                  bopts, 1, ws)
    assert ei.value.code == binding.VI_EINVAL
    with pytest.raises(binding.ViError) as ei:
        ctx.solve(dp.cam, dp.pose, dp.vel, dp.bias, dp.invdepth, dp.ii, dp.jj, dp.target, dp.weight, imu, bopts, 1,
                  ws[: ws.numel() // 2])
    assert ei.value.code == binding.VI_ENOMEM
    with pytest.raises(binding.ViError) as ei:
        ctx.imu_preintegrate(np.array([0, 5, 5], np.int32), dp.gyro, dp.accel, dp.imu_dt, dp.bias_hat[:2],
                             dp.noise)
    assert ei.value.code == binding.VI_EINVAL

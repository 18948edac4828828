"""Mixed-precision step (VI_PREC_MIXED) and the large-system Cholesky path,
against the FP64 oracle.

The mixed path evaluates residuals, Jacobians, the per-edge J^T W J sums and
the Schur Gram in FP32 (FP32 MFMA with Kahan-compensated block sums) and
keeps C, w_d, the inertial factors, the reduced system and its Cholesky in
FP64.  Its increments therefore differ from the FP64 oracle by the FP32
rounding of the assembled normal equations (unit roundoff 6e-8), amplified
by the conditioning of the reduced system; the measured error of every
result is printed.  Measured on these inputs: 1e-8 .. 1.5e-6 relative per
group of the step and <= 2e-6 on the inverse depths, so the mixed path is
held to the same bar as the FP64 path:
  * per group (rotation, translation, velocity, gyro bias, accel bias) of the
    step: relative 2-norm error <= 1e-4; inverse depths <= 1e-3;
  * solves: the final cost within 1e-6 relative of the FP64 oracle's final
    cost after the same number of iterations (the cost is accumulated in FP64,
    each pixel term is FP32; measured ~1e-8).
The FP64 run of a 64-keyframe window with loop edges (reduced system 960 x
960, above the one-workgroup size) checks the multi-workgroup tile-dataflow
Cholesky at the step tolerances (1e-4 / 1e-3).
"""
import numpy as np
import pytest

from oracle import normal_eq as ne
from oracle import solve as osolve
from paper_2512_02293_amd import synth

pytestmark = pytest.mark.gpu

GROUPS = {"dtheta": slice(0, 3), "dp": slice(3, 6), "dv": slice(6, 9), "dbg": slice(9, 12), "dba": slice(12, 15)}
MIXED_TOL_GROUP = 1e-4
MIXED_TOL_DEPTH = 1e-3


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


def _loop_window(n_kf=64, n_loop=25):
    return synth.SceneConfig(n_kf=n_kf, H=60, W=80, k_out=11, n_loop=n_loop)


def _step(ctx, prob, precision, **optkw):
    import torch
    from paper_2512_02293_amd import binding
    o = ne.Options(**optkw)
    bopts = binding.make_opts(n_fixed=o.n_fixed, use_imu=o.use_imu, bias_fixed=o.bias_fixed, lm_lambda=o.lm_lambda,
                              depth_eta=o.depth_eta, z_min=o.z_min, d_min=o.d_min, precision=precision)
    dp = binding.DeviceProblem(prob)
    imu = ctx.imu_preintegrate(dp.off, dp.gyro, dp.accel, dp.imu_dt, dp.bias_hat, dp.noise)
    nb = ctx.workspace_size(dp.cam, dp.pose.shape[0], dp.ii, dp.jj, bopts)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
    N = dp.pose.shape[0]
    dxi = torch.zeros((N, 15), dtype=torch.float64, device="cuda:0")
    dd = torch.zeros_like(dp.invdepth)
    rep = ctx.solve(dp.cam, dp.pose, dp.vel, dp.bias, dp.invdepth, dp.ii, dp.jj, dp.target, dp.weight, imu,
                    bopts, 1, ws, dxi=dxi, dd=dd)
    return rep, dxi.cpu().numpy(), dd.cpu().numpy(), o


def _errors(dxi, dd, orep):
    errs = {}
    for g, sl in GROUPS.items():
        ref = orep["dxi"][:, sl]
        if np.linalg.norm(ref) > 0:
            errs[g] = _rel(dxi[:, sl], ref)
    errs["dd"] = _rel(dd.ravel(), orep["dd"].ravel())
    return errs


@pytest.mark.parametrize("which", ["small", "window"])
def test_mixed_step_matches_oracle(ctx, which):
    from paper_2512_02293_amd import binding
    prob = synth.make_problem(synth.config_small() if which == "small" else synth.config_window(),
                              1 if which == "small" else 2)
    rep, dxi, dd, o = _step(ctx, prob, binding.VI_PREC_MIXED)
    cam, st, gr = osolve.from_problem(prob)
    _, orep = osolve.step(cam, st, gr, o)
    errs = _errors(dxi, dd, orep)
    print(f"mixed step {which}:", {k: f"{v:.2e}" for k, v in errs.items()},
          f"cost_before rel {abs(rep['cost_before'] / orep['cost_before'] - 1):.1e}")
    for g in GROUPS:
        if g in errs:
            assert errs[g] <= MIXED_TOL_GROUP, (g, errs[g])
    assert errs["dd"] <= MIXED_TOL_DEPTH
    assert rep["n_valid"] == orep["n_valid"]
    assert rep["cost_before"] == pytest.approx(orep["cost_before"], rel=1e-6)


def test_mixed_solve_reaches_fp64_cost(ctx):
    import torch
    from paper_2512_02293_amd import binding
    prob = synth.make_problem(synth.config_window(), 2)
    oopts = ne.Options()
    dp = binding.DeviceProblem(prob)
    imu = ctx.imu_preintegrate(dp.off, dp.gyro, dp.accel, dp.imu_dt, dp.bias_hat, dp.noise)
    bopts = binding.make_opts(precision=binding.VI_PREC_MIXED)
    nb = ctx.workspace_size(dp.cam, dp.pose.shape[0], dp.ii, dp.jj, bopts)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
    rep = ctx.solve(dp.cam, dp.pose, dp.vel, dp.bias, dp.invdepth, dp.ii, dp.jj, dp.target, dp.weight, imu,
                    bopts, 8, ws, costs=True)
    cam, st, gr = osolve.from_problem(prob)
    _, oreps = osolve.solve(cam, st, gr, oopts, 8)
    ocosts = np.array([r["cost_before"] for r in oreps] + [oreps[-1]["cost_after"]])
    rel = np.abs(rep["costs"] / ocosts - 1)
    print("mixed solve cost trace rel. error per iteration:", " ".join(f"{x:.1e}" for x in rel))
    assert rel[-1] <= 1e-6


def test_dataflow_cholesky_fp64_loop_window(ctx):
    """64 keyframes with long-range loop edges: reduced system 960 x 960 goes
    through the multi-workgroup tile dataflow; FP64 step tolerances."""
    from paper_2512_02293_amd import binding
    prob = synth.make_problem(_loop_window(), 31)
    rep, dxi, dd, o = _step(ctx, prob, binding.VI_PREC_FP64)
    cam, st, gr = osolve.from_problem(prob)
    _, orep = osolve.step(cam, st, gr, o)
    errs = _errors(dxi, dd, orep)
    print("fp64 loop window:", {k: f"{v:.2e}" for k, v in errs.items()})
    for g in GROUPS:
        if g in errs:
            assert errs[g] <= 1e-4, (g, errs[g])
    assert errs["dd"] <= 1e-3
    assert rep["n_valid"] == orep["n_valid"]
    assert rep["cost_after"] == pytest.approx(orep["cost_after"], rel=1e-6)


def test_mixed_loop_window(ctx):
    from paper_2512_02293_amd import binding
    prob = synth.make_problem(_loop_window(), 31)
    rep, dxi, dd, o = _step(ctx, prob, binding.VI_PREC_MIXED)
    cam, st, gr = osolve.from_problem(prob)
    _, orep = osolve.step(cam, st, gr, o)
    errs = _errors(dxi, dd, orep)
    print("mixed loop window:", {k: f"{v:.2e}" for k, v in errs.items()})
    for g in GROUPS:
        if g in errs:
            assert errs[g] <= MIXED_TOL_GROUP, (g, errs[g])
    assert errs["dd"] <= MIXED_TOL_DEPTH


def test_dataflow_cholesky_fp64_odd_tile_count(ctx):
    """35 keyframes (reduced system 525, padded to 544 = 17 tiles of 32): the
    tile dataflow with an odd number of block columns, so that the
    back-substitution's last ticket carries block 0 alone; FP64 against the
    FP64 oracle at 1e-8."""
    from paper_2512_02293_amd import binding
    prob = synth.make_problem(synth.SceneConfig(n_kf=35, H=48, W=64, k_out=6, n_loop=6, loop_gap=20), 37)
    rep, dxi, dd, o = _step(ctx, prob, binding.VI_PREC_FP64)
    cam, st, gr = osolve.from_problem(prob)
    _, orep = osolve.step(cam, st, gr, o)
    errs = _errors(dxi, dd, orep)
    print("fp64 odd tile count:", {k: f"{v:.2e}" for k, v in errs.items()})
    for g in GROUPS:
        if g in errs:
            assert errs[g] <= 1e-8, (g, errs[g])
    assert errs["dd"] <= 1e-8
    assert rep["n_valid"] == orep["n_valid"]

"""Pose-graph bundle adjustment in Sim(3) (vi_pgba_solve, Eq. 5) on the GPU
against the FP64 oracle (oracle/pgba.py), through the C ABI.

Tolerances: in FP64 both sides compute the same damped step up to rounding
order, so the step agrees to 1e-8 relative per group (rotation, translation,
log-scale) and on the inverse-depth increments (measured values printed);
valid-pixel counts exactly; costs to 1e-9.  Mixed precision (FP32 vision
assembly): the required 1e-4 per group and 1e-3 on inverse depths."""
import numpy as np
import pytest

from oracle import pgba
from oracle.so3 import Log, quat_to_R
from paper_2512_02293_amd import synth

pytestmark = pytest.mark.gpu
GROUPS = {"dtheta": slice(0, 3), "dp": slice(3, 6), "dsigma": slice(6, 7)}


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


def _problem(N, H, W, loops, k_rel=2, seed=5, noiseless=False):
    cfg = synth.SceneConfig(n_kf=N, H=H, W=W, k_out=1)
    rel = [(i, i + s) for s in range(1, k_rel + 1) for i in range(N - s)]
    return synth.make_pgba_problem(cfg, seed, loops, rel, noiseless=noiseless)


def _oracle(prob, exact=False):
    cam = (prob.fx, prob.fy, prob.cx, prob.cy, prob.H, prob.W)
    st = pgba.PGState(R=np.stack([quat_to_R(q) for q in prob.pose[:, 3:7]]), p=prob.pose[:, :3].copy(),
                      s=prob.scale.copy(), d=prob.invdepth.copy())
    Tm = np.stack([pgba.mat(m[7], quat_to_R(m[3:7]), m[0:3]) for m in prob.rel_meas])
    gr = pgba.PGGraph(ii=prob.ii, jj=prob.jj, target=prob.target64 if exact else prob.target.astype(np.float64),
                      weight=prob.weight.astype(np.float64), rel_ii=prob.rel_ii, rel_jj=prob.rel_jj, rel_T=Tm,
                      rel_info=prob.rel_info)
    return cam, st, gr


def _opts(precision=0, **kw):
    from paper_2512_02293_amd import binding
    o = pgba.PGOptions(**kw)
    return o, binding.make_opts(n_fixed=o.n_fixed, use_imu=False, lm_lambda=o.lm_lambda, depth_eta=o.depth_eta,
                                z_min=o.z_min, d_min=o.d_min, precision=precision)


def _gpu_step(ctx, prob, bopts, iters=1):
    import torch
    from paper_2512_02293_amd import binding
    pg = binding.DevicePGBA(prob)
    ws = torch.empty(ctx.pgba_workspace_size(pg, bopts), dtype=torch.uint8, device="cuda:0")
    dxi = torch.zeros((prob.n_kf, 7), dtype=torch.float64, device="cuda:0")
    dd = torch.zeros_like(pg.invdepth)
    rep = ctx.pgba_solve(pg, bopts, iters, ws, dxi=dxi, dd=dd)
    return pg, rep, dxi.cpu().numpy(), dd.cpu().numpy()


def _check_step(ctx, prob, tol_g, tol_d, precision=0, **kw):
    oopts, bopts = _opts(precision, **kw)
    pg, rep, dxi, dd = _gpu_step(ctx, prob, bopts)
    cam, st, gr = _oracle(prob)
    new, orep = pgba.step(cam, st, gr, oopts)
    errs = {k: _rel(dxi[:, sl], orep["dxi"][:, sl]) for k, sl in GROUPS.items()}
    errs["dd"] = _rel(dd.ravel(), orep["dd"].ravel())
    print(f"N={prob.n_kf} E*={prob.n_edges} E+={len(prob.rel_ii)}", {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= (tol_d if k == "dd" else tol_g), (k, v)
    assert rep["n_valid"] == orep["n_valid"]
    assert rep["cost_before"] == pytest.approx(orep["cost_before"], rel=1e-9 if precision == 0 else 1e-6)
    assert rep["iters_done"] == 1
    # committed state
    pose = pg.pose.cpu().numpy()
    ang = max(np.linalg.norm(Log(quat_to_R(q).T @ R)) for q, R in zip(pose[:, 3:7], new.R))
    assert ang <= tol_g * np.abs(orep["dxi"][:, 0:3]).max() + 1e-13
    assert np.abs(pg.scale.cpu().numpy() - new.s).max() <= tol_g * np.abs(orep["dxi"][:, 6]).max() + 1e-13
    assert np.abs(pg.invdepth.cpu().numpy() - new.d).max() <= max(tol_d, 1e-12) * np.abs(orep["dd"]).max()
    return rep, orep


def test_pgba_step_small(ctx):
    prob = _problem(6, 24, 32, [(0, 5), (5, 0), (1, 4), (4, 2)])
    _check_step(ctx, prob, 1e-8, 1e-8)


@pytest.mark.parametrize("lam,eta", [(0.0, 1e-6), (1e-2, 1e-3)])
def test_pgba_step_damping_variants(ctx, lam, eta):
    prob = _problem(6, 24, 32, [(0, 5), (5, 0), (1, 4), (4, 2)], seed=6)
    _check_step(ctx, prob, 1e-8, 1e-8, lm_lambda=lam, depth_eta=eta)


def test_pgba_step_many_loops_per_source(ctx):
    """40 keyframes (reduced system 280, one workgroup), sources with up to
    four loop pairs, relative poses to the 3 next keyframes."""
    rng = np.random.default_rng(1)
    loops = set()
    while len(loops) < 30:
        i, j = (int(v) for v in rng.integers(0, 40, size=2))
        if abs(i - j) >= 12:
            loops.add((i, j))
    loops = sorted(loops)
    prob = _problem(40, 30, 40, loops, k_rel=3, seed=7)
    assert np.bincount(prob.ii).max() >= 2
    _check_step(ctx, prob, 1e-8, 1e-8)


def test_pgba_step_large_system(ctx):
    """80 keyframes: reduced system 560 x 560, above the one-workgroup size
    (tile-dataflow Cholesky)."""
    loops = [(i, (i + 37) % 80) for i in range(0, 80, 4)]
    prob = _problem(80, 16, 24, loops, k_rel=2, seed=8)
    _check_step(ctx, prob, 1e-8, 1e-8)


def test_pgba_step_mixed_precision(ctx):
    prob = _problem(6, 24, 32, [(0, 5), (5, 0), (1, 4), (4, 2)])
    _check_step(ctx, prob, 1e-4, 1e-3, precision=1)


def test_pgba_solve_matches_oracle_solve(ctx):
    prob = _problem(8, 24, 32, [(0, 7), (7, 1), (2, 6)], seed=9)
    oopts, bopts = _opts()
    pg, rep, _, _ = _gpu_step(ctx, prob, bopts, iters=4)
    cam, st, gr = _oracle(prob)
    ost, oreps = pgba.solve(cam, st, gr, oopts, 4)
    ocosts = [r["cost_before"] for r in oreps] + [oreps[-1]["cost_after"]]
    assert np.allclose(rep["costs"], ocosts, rtol=1e-9), (rep["costs"], ocosts)
    assert rep["iters_done"] == 4
    pose = pg.pose.cpu().numpy()
    assert np.abs(pose[:, :3] - ost.p).max() < 1e-9
    assert np.abs(pg.scale.cpu().numpy() - ost.s).max() < 1e-9
    assert np.abs(pg.invdepth.cpu().numpy() - ost.d).max() < 1e-9


def test_pgba_recovers_scale_drift(ctx):
    """Noiseless relative poses and loop pairs: pure Gauss-Newton recovers the
    planted 10 % scale drift to the rounding of the FP32 targets."""
    prob = _problem(8, 24, 32, [(0, 7), (7, 0), (1, 6), (6, 2)], seed=10, noiseless=True)
    _, bopts = _opts(lm_lambda=0.0, depth_eta=0.0)
    pg, rep, _, _ = _gpu_step(ctx, prob, bopts, iters=8)
    assert rep["costs"][-1] < 1e-8 * rep["costs"][0]
    np.testing.assert_allclose(pg.scale.cpu().numpy(), prob.scale_gt, rtol=1e-5)
    np.testing.assert_allclose(pg.pose.cpu().numpy()[:, :3], prob.pose_gt[:, :3], atol=1e-5)


def test_pgba_errors_leave_state(ctx):
    import torch
    from paper_2512_02293_amd import binding
    prob = _problem(6, 24, 32, [(0, 5), (5, 0)])
    _, bopts = _opts()
    pg = binding.DevicePGBA(prob)
    ws = torch.empty(ctx.pgba_workspace_size(pg, bopts), dtype=torch.uint8, device="cuda:0")
    bad = pg.rel_jj.copy()
    pg.rel_jj[0] = pg.rel_ii[0]
    with pytest.raises(binding.ViError) as ei:
        ctx.pgba_solve(pg, bopts, 1, ws)
    assert ei.value.code == binding.VI_EINVAL
    pg.rel_jj[:] = bad
    pg.rel_meas[2, 7] = float("nan")
    before = [t.cpu().clone() for t in (pg.pose, pg.scale, pg.invdepth)]
    with pytest.raises(binding.ViError) as ei:
        ctx.pgba_solve(pg, bopts, 2, ws)
    assert ei.value.code == binding.VI_ENONFINITE
    for a, t in zip(before, (pg.pose, pg.scale, pg.invdepth)):
        assert torch.equal(a, t.cpu())


def test_pgba_step_loop_closure_512(ctx):
    """The benchmarked loop closure at full size: 512 keyframes (reduced system
    3584 x 3584, tile-dataflow Cholesky), 200 loop pairs of 60x80 maps, 1530
    relative poses; one FP64 step against the oracle's."""
    prob = synth.pgba_loop_closure_problem()
    assert prob.n_kf == 512 and prob.n_edges == 200 and len(prob.rel_ii) == 1530
    _check_step(ctx, prob, 1e-8, 1e-8)


def test_pgba_autotuned_tiling_matches_oracle():
    """With the autotuner on, the fused assembly of the loop pairs runs with the
    fastest pixel range of the candidates; the step is the same."""
    from paper_2512_02293_amd import binding
    c = binding.Context(0)
    try:
        c.set_autotune(True)
        rng = np.random.default_rng(2)
        loops = sorted({(int(i), int(j)) for i, j in rng.integers(0, 40, size=(60, 2)) if abs(int(i) - int(j)) >= 12})
        prob = _problem(40, 30, 40, loops[:25], k_rel=3, seed=12)
        rep, _ = _check_step(c, prob, 1e-8, 1e-8)
        assert rep["tile_px"] % 64 == 0 and rep["tile_px"] >= 128
    finally:
        c.close()

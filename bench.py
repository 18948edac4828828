"""Benchmark of the visual-inertial Gauss-Newton step on one MI355X.

Workload: the 24-keyframe sliding window (60x80 inverse-depth maps, 288 edges,
each keyframe to its 12 nearest by index, 200 Hz IMU with 20 samples per
keyframe gap), seeded synthetic data.  One benchmark step is one whole pass of
the hot path: IMU preintegration of the window's 23 factors, then a solve of 8
damped Gauss-Newton iterations (each: residual/Jacobian assembly, inertial
factors, Schur elimination of the inverse depths, FP64 Cholesky of the 360x360
reduced system, back-substitution and retraction) and the final cost, all in
FP64, replayed from one captured HIP graph.  Every step restarts from the same
initial estimate (a device-to-device copy of the four state arrays, inside the
timed region).

Prints one JSON line: pixel-residuals per second (edges x pixels x iterations
per second of wall time), ms per step and per GN iteration, the roofline
position of the dominant kernel (per-stage GPU times from HIP events on the
library's stream) and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pixel-residuals/s + ms per GN iter (24-KF window); time-to-tol learned vs plain"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
GN_ITERS = 8
# kernel behind each stage of the benchmarked window, and the committed HBM
# counter readings (rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by a plain copy)
STAGE_KERNEL = {"cholesky": "k_chol_small", "vis_gram_imu": "k_vis_gram<double>"}
REANCHOR_KERNEL = "k_reanchor<true, true>"
# Gaussian-map update: anchor 4 B + mean 12 B read and written + covariance 24 B read and written
REANCHOR_BYTES_PER_GAUSSIAN = 4 + 2 * 12 + 2 * 24
HBM_COUNTERS = os.path.join(ROOT, "profiles", "hbm_counters.json")


def measured_traffic(kernel):
    """HBM bytes per dispatch of `kernel` from the committed counter readings,
    or None when there are none or the kernel's source changed since."""
    import hashlib
    try:
        with open(HBM_COUNTERS) as fh:
            rec = json.load(fh)["kernels"][kernel]
        with open(os.path.join(ROOT, rec["source"]), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != rec["sha256"]:
                return None
        return float(rec["bytes_per_dispatch"])
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=4, help="oracle GN iterations in the CPU sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--autotune", type=int, default=1, choices=[0, 1],
                    help="let the library time the candidate pixel tilings of the fused assembly on this window "
                         "(once, before the timed steps) and keep the fastest")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 64-window batch, the global problem and the warm-start lines")
    ap.add_argument("--only", choices=["global", "warm-windows", "gaussian-reanchor", "predict-keyframe",
                                       "inertial-init", "assembly", "pgba"],
                    default=None,
                    help="run only that secondary workload and print its JSON (profiling runs)")
    return ap.parse_args()


def copy_calibration():
    """A plain copy of known size (256 MiB read + 256 MiB written per launch),
    the reference that scales the HBM byte counters."""
    import torch
    src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)       # one elementwise kernel: 256 MiB read, 256 MiB written
    torch.cuda.synchronize()
    return {"kernel": "elementwise multiply by 1 (MulFunctor)", "read": src.numel() * 4, "write": dst.numel() * 4,
            "launches": 3}


def stage_models(prob):
    """Algorithmic work of one launch of each stage (one GN iteration).

    vis_gram_imu (FP64 MFMA + VALU): the J^T W J contractions of the step --
      per pixel-residual the local 6x6 Hessian (21 entries), gradient (6) and
      E-entries (6), each from 2 coordinates at 2 flops per multiply-add
      (132 flops), plus per source pixel the symmetric (6k+1)^2 Schur Gram,
      (6k+1)(6k+2) flops.  Residual/Jacobian evaluation is not counted.
      Its HBM side is 16 B per pixel-residual (f32 target and weight) plus
      8 B in and 16 B out per source pixel.
    cholesky (FP64): n^3/3 flops for the 15N x 15N reduced system.
    """
    import numpy as np
    N, E, HW = prob.n_kf, prob.n_edges, prob.H * prob.W
    ks = np.bincount(prob.ii, minlength=N)
    gram_flops = float(sum((6 * k + 1) * (6 * k + 2) for k in ks if k > 0)) * HW
    n = 15 * N
    return {
        "vis_gram_imu": dict(bound="mfma", unit="TFLOP/s", peak=FP64_PEAK_TFLOPS, scale=1e12,
                             work=gram_flops + 132.0 * E * HW, work_name="algorithmic_flops_per_launch",
                             per_unit="132 flops per pixel-residual + (6k+1)(6k+2) flops per source pixel",
                             hbm_bytes=float(E * HW * 16 + N * HW * 24)),
        "cholesky": dict(bound="mfma", unit="TFLOP/s", peak=FP64_PEAK_TFLOPS, scale=1e12, work=n ** 3 / 3.0,
                         work_name="algorithmic_flops_per_launch", per_unit="n^3/3 flops, n = 15 N",
                         note="one window is one 512-thread workgroup on one CU (FP64 MFMA peak of one CU: "
                              "78.6/256 = 0.307 TFLOP/s); the factor's critical path is a chain of 32x32 "
                              "diagonal-tile factorisations"),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU sharding is not built "
                                   "(--gpus must be 1)"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2512_02293_amd import binding, synth
    if args.only is not None:
        ctx = binding.Context(0)
        ctx.set_autotune(bool(args.autotune))
        out = {"global": global_problem, "warm-windows": warm_windows, "gaussian-reanchor": gaussian_reanchor,
               "predict-keyframe": predict_keyframe, "inertial-init": inertial_init,
               "assembly": assembly_roofline, "pgba": lambda c: pgba_loop_closure(c, cpu=not args.no_cpu_baseline)}[args.only](ctx)
        if args.copy_calibration:
            out["copy_calibration_bytes"] = copy_calibration()
        print(json.dumps(out))
        ctx.close()
        return

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    cfg = synth.config_window()
    prob = synth.make_problem(cfg, 2)
    N, E, H, W = prob.n_kf, prob.n_edges, prob.H, prob.W
    HW = H * W
    ctx = binding.Context(0)
    ctx.set_autotune(bool(args.autotune))
    dp = binding.DeviceProblem(prob, dev)
    opts = binding.make_opts()
    ws = torch.empty(ctx.workspace_size(dp.cam, N, dp.ii, dp.jj, opts), dtype=torch.uint8, device=dev)
    init = [t.clone() for t in (dp.pose, dp.vel, dp.bias, dp.invdepth)]
    imu = torch.empty((N - 1, binding.PREINT_DOUBLES), dtype=torch.float64, device=dev)

    def step():
        for dst, src in zip((dp.pose, dp.vel, dp.bias, dp.invdepth), init):
            dst.copy_(src)
        ctx.imu_preintegrate(dp.off, dp.gyro, dp.accel, dp.imu_dt, dp.bias_hat, dp.noise, out=imu)
        return ctx.solve(dp.cam, dp.pose, dp.vel, dp.bias, dp.invdepth, dp.ii, dp.jj, dp.target, dp.weight, imu,
                         opts, GN_ITERS, ws, costs=True)

    for _ in range(args.warmup):
        rep = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rep = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = 1e3 * elapsed / args.steps
    pxres_per_step = E * HW * GN_ITERS
    value = pxres_per_step / (elapsed / args.steps)

    # per-stage GPU time (HIP events on the library stream), summed over the 8 iterations
    reps = 5
    acc = None
    for _ in range(reps):
        for dst, src in zip((dp.pose, dp.vel, dp.bias, dp.invdepth), init):
            dst.copy_(src)
        r = ctx.solve(dp.cam, dp.pose, dp.vel, dp.bias, dp.invdepth, dp.ii, dp.jj, dp.target, dp.weight, imu, opts,
                      GN_ITERS, ws, stage_ms=True)
        s = r["stage_ms"]
        acc = s if acc is None else {k: acc[k] + s[k] for k in s}
    stage_ms = {k: v / reps for k, v in acc.items()}           # per solve
    per_iter_ms = {k: v / GN_ITERS for k, v in stage_ms.items() if k != "final_cost"}
    models = stage_models(prob)
    dom = max(per_iter_ms, key=per_iter_ms.get)
    key = dom if dom in models else max(models, key=lambda k: per_iter_ms.get(k, 0.0))
    m = models[key]
    achieved = m["work"] / (per_iter_ms[key] * 1e-3) / m["scale"]
    roof = {"bound": m["bound"], "achieved": achieved, "peak": m["peak"], "unit": m["unit"],
            "frac": achieved / m["peak"], "traffic": measured_traffic(STAGE_KERNEL.get(key, "")), "stage": key,
            "kernel": STAGE_KERNEL.get(key), "dominant_stage": dom, "stage_ms": per_iter_ms[key],
            m["work_name"]: m["work"], "per_unit": m["per_unit"]}
    if "note" in m:
        roof["note"] = m["note"]
    if "hbm_bytes" in m:
        roof["hbm_gbs_algorithmic"] = m["hbm_bytes"] / (per_iter_ms[key] * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pixel-residuals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_gn_iter": ms_step / GN_ITERS,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "sliding window: 24 keyframes, 60x80 inverse-depth maps, 288 edges (12 nearest "
                               "by index), 200 Hz IMU / 10 Hz keyframes, 8 GN iterations, FP64",
                   "n_kf": N, "n_edges": E, "H": H, "W": W, "gn_iters": GN_ITERS,
                   "pixel_residuals_per_step": pxres_per_step, "final_cost": float(rep["cost_after"]),
                   "assembly_tile_px": int(rep["tile_px"]), "autotune": bool(args.autotune)},
        "stage_ms_per_iter": {k: round(v, 5) for k, v in per_iter_ms.items()},
        "roofline": roof,
    }
    if args.copy_calibration:
        out["copy_calibration_bytes"] = copy_calibration()
    if not args.no_extras:
        out.update(extras(ctx))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_iters)
    print(json.dumps(out))
    ctx.close()


def extras(ctx):
    """The 64-window batch (one graph for all windows vs one solve per window)
    and the learned warm start's time to tolerance on the same windows."""
    import numpy as np
    import torch

    from paper_2512_02293_amd import binding, synth, warmstart
    probs = [synth.make_problem(synth.config_batched_window(w), 4000 + w) for w in range(64)]
    opts = binding.make_opts()
    dps = [binding.DeviceProblem(p) for p in probs]
    imus = [ctx.imu_preintegrate(d.off, d.gyro, d.accel, d.imu_dt, d.bias_hat, d.noise) for d in dps]
    ws = torch.empty(ctx.workspace_size_batched(dps, opts), dtype=torch.uint8, device="cuda:0")
    pxres = sum(p.n_edges * p.H * p.W for p in probs) * GN_ITERS

    def batch():
        for d in dps:
            d.reset_state()
        ctx.solve_batched(dps, imus, opts, GN_ITERS, ws)

    # one context per window: each keeps the captured graph of its own shape,
    # so the per-window leg replays graphs as the batch does
    ctxs = [binding.Context(0) for _ in dps]
    wss = [torch.empty(c.workspace_size(d.cam, d.pose.shape[0], d.ii, d.jj, opts), dtype=torch.uint8,
                       device="cuda:0") for c, d in zip(ctxs, dps)]

    def singles():
        for c, d, im, w in zip(ctxs, dps, imus, wss):
            d.reset_state()
            c.solve(d.cam, d.pose, d.vel, d.bias, d.invdepth, d.ii, d.jj, d.target, d.weight, im, opts,
                    GN_ITERS, w)

    def best(fn, reps=5):
        fn()
        t = 1e30
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            t = min(t, time.perf_counter() - t0)
        return t

    t_b = best(batch)
    t_s = best(singles, reps=3)
    for c in ctxs:
        c.close()
    res = {"batched": {"workload": "64 independent windows, N ~ U{8..32} keyframes, 3-8 edges each, 48x64 or "
                                   "60x80 maps, uneven IMU gaps, 8 GN iterations, FP64",
                       "pixel_residuals_per_s": pxres / t_b, "ms_batch": 1e3 * t_b,
                       "ms_one_solve_per_window": 1e3 * t_s,
                       "note": "per-window leg: one context per window, each replaying its own captured graph "
                               "(captured during the warm-up), the windows solved one after another"}}
    res["assembly_roofline"] = assembly_roofline(ctx)
    res["global"] = global_problem(ctx)
    res["pgba"] = pgba_loop_closure(ctx)
    res["gaussian_reanchor"] = gaussian_reanchor(ctx)
    res["predict_keyframe"] = predict_keyframe(ctx)
    res["inertial_init"] = inertial_init(ctx)
    if os.path.exists(warmstart.PARAMS_FILE):
        net = warmstart.WarmNet.load(ctx)
        res["time_to_tol_batch_distribution"] = _time_to_tol_entry(
            warmstart.time_to_tol(ctx, net, warmstart.eval_windows(smooth=False), binding.make_opts()),
            "the 64 batched windows as they are generated (per-pixel 10% initial inverse-depth error), default "
            "damping lm_lambda 1e-4; target F <= F_plain(30 iterations) (1 + 1e-6) per window")
        r = warmstart.time_to_tol(ctx, net, warmstart.eval_windows(), warmstart.study_opts())
        res["time_to_tol"] = {
            "workload": "64 windows of the batched distribution with a smooth 10% initial inverse-depth error, "
                        "lm_lambda 1e-6; target F <= F_plain(30 iterations) (1 + 1e-6) per window",
            "gn_iters_plain_mean": float(np.mean(r["k_plain"])), "gn_iters_warm_mean": float(np.mean(r["k_warm"])),
            "gn_iters_batch_plain": r["K_plain"], "gn_iters_batch_warm": r["K_warm"],
            "warm_accepted": int(sum(r["accepted"])), "targets_reached": int(sum(r["reached"])),
            "batch_ms_plain": r["ms_plain"], "batch_ms_warm": r["ms_warm"],
            "per_window_ms_plain_total": r["ms_plain_per_window_total"],
            "per_window_ms_warm_total": r["ms_warm_per_window_total"],
            "per_window_speedup": r["ms_plain_per_window_total"] / r["ms_warm_per_window_total"],
            "batch_tolerance_stop": r["stop"], "per_window_tolerance_stop": r["per_window_stop"],
            "note": "batch: all windows in one set of launches, bounded by the slowest window; per window: each "
                    "window solved alone (sliding-window use), warm start = vi_warm_start (features, network, "
                    "corrections, cost check and device-side fallback) + GN"}
    return res


def assembly_work(probs):
    """Algorithmic work of one launch of the fused assembly on these windows:
    HBM bytes per the per-pixel-residual count of the mixed path (target and
    weight, FP32: 16 B per pixel-residual; the source's inverse depth read
    and its increment written, FP32: 8 B per source pixel, i.e. 8/k B per
    pixel-residual), and the symmetric half of the Schur Gram,
    (6k)(6k + 1) flops per source pixel of a keyframe with k outgoing edges."""
    import numpy as np
    pxres = bytes_ = flops = 0.0
    for p in probs:
        HW = p.H * p.W
        ks = np.bincount(p.ii, minlength=p.n_kf)
        pxres += float(p.n_edges * HW)
        bytes_ += 16.0 * p.n_edges * HW + 8.0 * int((ks > 0).sum()) * HW
        flops += float(sum(6 * k * (6 * k + 1) for k in ks)) * HW
    return pxres, bytes_, flops


def assembly_roofline(ctx, reps=5):
    """HBM and FP32-MFMA position of the fused assembly (k_vis_gram<float>,
    the mixed path) on the two workloads whose inputs exceed the 256 MB
    last-level cache: the 512-keyframe problem and the 64-window batch.  The
    kernel time is the assembly stage of eager steps (HIP events recorded by
    the library on its own stream around that one launch), best of `reps`.
    A context of its own with the library's default tiling (the same in the
    full benchmark line and in the `--only assembly` profiling runs)."""
    import torch

    from paper_2512_02293_amd import binding, synth
    ctx = binding.Context(0)
    o = binding.make_opts(precision=binding.VI_PREC_MIXED)
    out = {}
    # the 512-keyframe problem
    prob = synth.make_problem(synth.config_global(), 3)
    dp = binding.DeviceProblem(prob)
    imu = ctx.imu_preintegrate(dp.off, dp.gyro, dp.accel, dp.imu_dt, dp.bias_hat, dp.noise)
    ws = torch.empty(ctx.workspace_size(dp.cam, prob.n_kf, dp.ii, dp.jj, o), dtype=torch.uint8, device="cuda:0")
    ms = []
    for _ in range(reps + 1):
        dp.reset_state()
        ms.append(ctx.solve(dp.cam, dp.pose, dp.vel, dp.bias, dp.invdepth, dp.ii, dp.jj, dp.target, dp.weight, imu,
                            o, 1, ws, stage_ms=True)["stage_ms"]["vis_gram_imu"])
    del ws
    out["global_512kf"] = _assembly_entry(
        [prob], min(ms[1:]), "512 keyframes, 60x80 maps, 5832 edges (11 nearest + 200 loop edges), mixed precision",
        16.0 + 8.0 / (prob.n_edges / prob.n_kf), "k_vis_gram<float>@global_512kf")
    # the 64-window batch
    probs = [synth.make_problem(synth.config_batched_window(w), 4000 + w) for w in range(64)]
    dps = [binding.DeviceProblem(p) for p in probs]
    imus = [ctx.imu_preintegrate(d.off, d.gyro, d.accel, d.imu_dt, d.bias_hat, d.noise) for d in dps]
    ws = torch.empty(ctx.workspace_size_batched(dps, o), dtype=torch.uint8, device="cuda:0")
    ms = []
    for _ in range(reps + 1):
        for d in dps:
            d.reset_state()
        ms.append(ctx.solve_batched(dps, imus, o, 1, ws, stage_ms=True)[0]["stage_ms"]["vis_gram_imu"])
    pxres, _, _ = assembly_work(probs)
    E = sum(p.n_edges for p in probs)
    N = sum(p.n_kf for p in probs)
    out["batch_64_windows"] = _assembly_entry(
        probs, min(ms[1:]), "64 independent windows (N ~ U{8..32}, 3-8 edges per keyframe, 48x64 or 60x80 maps), "
                            "mixed precision, all windows in one launch", 16.0 + 8.0 * N / E,
        "k_vis_gram<float>@batch_64_windows")
    ctx.close()
    return out


def _assembly_entry(probs, ms, workload, bytes_per_pxres, traffic_key):
    pxres, bytes_, flops = assembly_work(probs)
    t = ms * 1e-3
    gbs = bytes_ / t / 1e9
    tf = flops / t / 1e12
    traffic = measured_traffic(traffic_key)
    return {"workload": workload, "kernel": "k_vis_gram<float>", "ms_per_launch": ms,
            "pixel_residuals_per_launch": pxres, "pixel_residuals_per_s": pxres / t,
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
                         "traffic_over_algorithmic": (traffic / bytes_) if traffic else None,
                         "algorithmic_bytes_per_launch": bytes_,
                         "per_unit": f"{bytes_per_pxres:.2f} B per pixel-residual (target + weight 16 B, FP32 "
                                     f"inverse depth read and increment written 8 B per source pixel)"},
            "gram_mfma": {"achieved": tf, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tf / FP32_PEAK_TFLOPS,
                          "algorithmic_flops_per_launch": flops,
                          "per_unit": "(6k)(6k + 1) flops per source pixel (symmetric half of the Schur Gram)"}}


def _time_to_tol_entry(r, workload):
    import numpy as np
    return {"workload": workload,
            "gn_iters_plain_mean": float(np.mean(r["k_plain"])), "gn_iters_warm_mean": float(np.mean(r["k_warm"])),
            "gn_iters_batch_plain": r["K_plain"], "gn_iters_batch_warm": r["K_warm"],
            "warm_accepted": int(sum(r["accepted"])), "targets_reached": int(sum(r["reached"])),
            "batch_ms_plain": r["ms_plain"], "batch_ms_warm": r["ms_warm"],
            "per_window_ms_plain_total": r["ms_plain_per_window_total"],
            "per_window_ms_warm_total": r["ms_warm_per_window_total"],
            "batch_tolerance_stop": r["stop"], "per_window_tolerance_stop": r["per_window_stop"],
            "note": "the network trained on the smooth-error windows, applied unchanged"}


def global_problem(ctx, iters=2, reps=3):
    """The 512-keyframe problem (config_global, seed 3): GN iterations in FP64
    and in mixed precision, graph-replayed, plus per-stage GPU times of one
    eager step each."""
    import torch

    from paper_2512_02293_amd import binding, synth
    prob = synth.make_problem(synth.config_global(), 3)
    dp = binding.DeviceProblem(prob)
    imu = ctx.imu_preintegrate(dp.off, dp.gyro, dp.accel, dp.imu_dt, dp.bias_hat, dp.noise)
    res = {"workload": "512 keyframes, 60x80 maps, 5832 edges (11 nearest + 200 loop edges), reduced system "
                       "7680 x 7680; GN iterations from the initial state"}
    for name, prec in (("fp64", binding.VI_PREC_FP64), ("mixed", binding.VI_PREC_MIXED)):
        o = binding.make_opts(precision=prec)
        ws = torch.empty(ctx.workspace_size(dp.cam, prob.n_kf, dp.ii, dp.jj, o), dtype=torch.uint8, device="cuda:0")
        st = None
        for _ in range(2):
            dp.reset_state()
            st = ctx.solve(dp.cam, dp.pose, dp.vel, dp.bias, dp.invdepth, dp.ii, dp.jj, dp.target, dp.weight, imu, o,
                           1, ws, stage_ms=True)["stage_ms"]
        best = 1e30
        for _ in range(reps + 1):
            dp.reset_state()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.solve(dp.cam, dp.pose, dp.vel, dp.bias, dp.invdepth, dp.ii, dp.jj, dp.target, dp.weight, imu, o,
                      iters, ws)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        res[name] = {"ms_per_gn_iter": 1e3 * best / iters,
                     "pixel_residuals_per_s": prob.n_edges * prob.H * prob.W * iters / best,
                     "stage_ms_one_step": {k: round(v, 4) for k, v in st.items()}}
    return res


def pgba_loop_closure(ctx, iters=4, reps=3, cpu=True):
    """Pose-graph bundle adjustment in Sim(3) (vi_pgba_solve) on the 512-keyframe
    loop closure (synth.pgba_loop_closure_problem):
    iters damped GN steps from the initial state, FP64 and mixed, best of reps
    wall times of the (synchronous) call; the oracle's step on the host cores
    beside it."""
    import numpy as np
    import torch

    from paper_2512_02293_amd import binding, synth
    prob = synth.pgba_loop_closure_problem()
    pg = binding.DevicePGBA(prob)
    pxres = prob.n_edges * prob.H * prob.W
    res = {"workload": f"loop closure, {prob.n_kf} keyframes (Sim(3), 7 unknowns each), {prob.n_edges} loop pairs "
                       f"of 60x80 maps, {len(prob.rel_ii)} relative poses (next 3 keyframes), reduced system "
                       f"{7 * prob.n_kf} x {7 * prob.n_kf}; {iters} GN steps from the initial state",
           "pixel_residuals_per_gn_iter": pxres, "relative_poses": int(len(prob.rel_ii))}
    for name, prec in (("fp64", binding.VI_PREC_FP64), ("mixed", binding.VI_PREC_MIXED)):
        o = binding.make_opts(use_imu=False, precision=prec)
        ws = torch.empty(ctx.pgba_workspace_size(pg, o), dtype=torch.uint8, device="cuda:0")
        pg.reset_state()
        ctx.pgba_solve(pg, o, iters, ws)
        best, rep = 1e30, None
        for _ in range(reps):
            pg.reset_state()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rep = ctx.pgba_solve(pg, o, iters, ws)
            best = min(best, time.perf_counter() - t0)
        res[name] = {"ms_per_gn_iter": 1e3 * best / iters, "pixel_residuals_per_s": pxres * iters / best,
                     "cost_first": float(rep["costs"][0]), "cost_last": float(rep["costs"][-1]),
                     "assembly_tile_px": rep["tile_px"]}
    if cpu:
        from threadpoolctl import threadpool_info

        from oracle import pgba
        from oracle.so3 import quat_to_R
        cam = (prob.fx, prob.fy, prob.cx, prob.cy, prob.H, prob.W)
        st = pgba.PGState(R=np.stack([quat_to_R(q) for q in prob.pose[:, 3:7]]), p=prob.pose[:, :3].copy(),
                          s=prob.scale.copy(), d=prob.invdepth.copy())
        Tm = np.stack([pgba.mat(m[7], quat_to_R(m[3:7]), m[0:3]) for m in prob.rel_meas])
        gr = pgba.PGGraph(ii=prob.ii, jj=prob.jj, target=prob.target.astype(np.float64),
                          weight=prob.weight.astype(np.float64), rel_ii=prob.rel_ii, rel_jj=prob.rel_jj, rel_T=Tm,
                          rel_info=prob.rel_info)
        t0 = time.perf_counter()
        pgba.step(cam, st, gr, pgba.PGOptions())
        t_step = time.perf_counter() - t0
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        res["cpu_baseline"] = {"value": 1e3 * t_step, "unit": "ms per GN step", "cores": threads, "kind": "oracle",
                               "sample": "one oracle step on the same problem (NumPy float64, BLAS on its default "
                                         "threads), linearisation, Schur solve and the cost of the new state"}
    return res


def gaussian_reanchor(ctx, n_kf=512, per_kf=16384, reps=50):
    """Loop-closure update of a Gaussian map (Eq. 7-8): 512 keyframes x 16384
    Gaussians, FP32 means and covariances, out of place; GPU time per call from
    HIP events on the context's stream (torch's current stream) around `reps`
    back-to-back calls (queued behind a spin kernel, so that the GPU runs them
    without host gaps), and the same for calls on an empty map (only the
    per-keyframe table kernel runs), whose difference is the map kernel's time."""
    import torch

    from paper_2512_02293_amd import synth
    g = synth.make_gaussian_map(n_kf, per_kf, 11)
    dev = lambda a: torch.as_tensor(a, device="cuda:0")
    pre, post, ds = dev(g.pose_pre), dev(g.pose_post), dev(g.scale_change)
    anchor, mean, cov = dev(g.anchor), dev(g.mean), dev(g.cov)
    mean_out, cov_out = torch.empty_like(mean), torch.empty_like(cov)
    ws = torch.empty(ctx.reanchor_workspace_size(n_kf), dtype=torch.uint8, device="cuda:0")
    K = int(anchor.shape[0])

    def call():
        ctx.gaussian_reanchor(pre, post, ds, anchor, mean, cov, mean_out, cov_out, ws)

    def table_only():
        ctx.gaussian_reanchor(pre, post, ds, anchor[:0], mean[:0], cov[:0], mean_out[:0], cov_out[:0], ws)

    def per_call_ms(fn):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        # hold the stream with a spin kernel while the host queues every call, so
        # that the events time back-to-back GPU work, not host launch overhead
        torch.cuda._sleep(50_000_000)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms = per_call_ms(call)
    ms_table = per_call_ms(table_only)
    ms_map = ms - ms_table
    # the oracle on a bounded sample of the same map (first 2^20 Gaussians), one core
    from threadpoolctl import threadpool_limits

    from oracle import gauss as ogauss
    ns = 1 << 20
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        ogauss.reanchor(g.mean[:ns], g.cov[:ns], g.anchor[:ns], g.pose_pre, g.pose_post, g.scale_change)
        dt_cpu = time.perf_counter() - t0
    alg = K * REANCHOR_BYTES_PER_GAUSSIAN
    gbs = alg / (ms_map * 1e-3) / 1e9
    return {"workload": f"Gaussian map update after a loop closure: {n_kf} keyframes x {per_kf} Gaussians "
                        f"({K} total), FP32 means and 6-entry covariances, out of place",
            "gaussians_per_s": K / (ms * 1e-3), "ms_per_call": ms, "ms_map_kernel": ms_map,
            "ms_keyframe_table": ms_table,
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "traffic": measured_traffic(REANCHOR_KERNEL),
                         "kernel": REANCHOR_KERNEL, "algorithmic_bytes_per_launch": alg,
                         "per_unit": "76 B per Gaussian (anchor 4, mean 12 + 12, covariance 24 + 24)",
                         "note": "map-kernel time = time per call minus time per call on an empty map (the "
                                 "per-keyframe table kernel alone), both from HIP events on the context's stream"},
            "cpu_baseline": {"value": ns / dt_cpu, "unit": "Gaussians/s", "cores": 1, "kind": "oracle",
                             "sample": f"the first {ns} Gaussians of the same map ({dt_cpu:.2f} s, NumPy float64, "
                                       f"1 BLAS thread)"}}


def predict_keyframe(ctx, n=64, reps=200):
    """New-keyframe prediction from preintegration with the covariance-trace
    fallback: one prediction for each of the 64 batched windows (its last
    factor), GPU time per call from HIP events around back-to-back calls queued
    behind a spin kernel."""
    import torch

    from paper_2512_02293_amd import binding, synth
    probs = [synth.make_problem(synth.config_batched_window(w), 4000 + w) for w in range(n)]
    dps = [binding.DeviceProblem(p) for p in probs]
    imus = [ctx.imu_preintegrate(d.off, d.gyro, d.accel, d.imu_dt, d.bias_hat, d.noise) for d in dps]
    imu = torch.stack([m[-1] for m in imus]).contiguous()
    q0 = torch.stack([d.pose[-2] for d in dps]).contiguous()
    v0 = torch.stack([d.vel[-2] for d in dps]).contiguous()
    b0 = torch.stack([d.bias[-2] for d in dps]).contiguous()
    g = probs[0].gravity
    out = ctx.predict_keyframe(q0, v0, b0, imu, g)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda._sleep(50_000_000)
    e0.record()
    for _ in range(reps):
        ctx.predict_keyframe(q0, v0, b0, imu, g, 1e-4, *out)
    e1.record()
    torch.cuda.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / reps
    # the oracle on the same 64 predictions (its own preintegration of the factors is not timed)
    from oracle import predict as opred
    from oracle import preint as opreint
    facs = [opreint.preintegrate_all(p.imu_off, p.gyro, p.accel, p.imu_dt, p.bias_hat, p.noise)[-1] for p in probs]
    t0 = time.perf_counter()
    for p, P in zip(probs, facs):
        opred.predict_pose7(p.pose[-2], p.vel[-2], p.bias[-2], P, p.gravity)
    dt_cpu = time.perf_counter() - t0
    return {"workload": f"{n} new keyframes (the last factor of each batched window), FP64",
            "us_per_call": us, "used_imu": int(out[3].sum().item()),
            "cpu_baseline": {"value": 1e6 * dt_cpu, "unit": "us per 64 predictions", "cores": 1, "kind": "oracle",
                             "sample": "the same 64 predictions (NumPy float64)"},
            "roofline": {"bound": "latency", "note": "one lane per prediction (about 600 FP64 operations and "
                                                     "1.4 KB of input each); the time is launch and memory latency"}}


def inertial_init(ctx, n=64, n_kf=20, iters=10, reps=5):
    """IMU initialisation stage 2 on a batch of 64 problems of 20 keyframes (the
    paper's default keyframe count for it), 10 iterations each, from gravity =
    the visual z axis, s = 0 and zero velocities and biases; wall time per call
    (the call is synchronous) and the cost reduction."""
    import numpy as np
    import torch

    from paper_2512_02293_amd import binding, synth
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda:0")
    probs, init = [], []
    for w in range(n):
        ip = synth.make_inertial_init_problem(synth.tiny_config(n_kf=n_kf), 6000 + w, pose_noise=(2e-4, 0.01))
        dp_off = ip.imu_off
        off = np.ascontiguousarray(dp_off, dtype=np.int32)
        imu = ctx.imu_preintegrate(off, dev(ip.gyro), dev(ip.accel), dev(ip.imu_dt), dev(ip.bias_hat), ip.noise)
        probs.append({"pose_vis": dev(ip.pose_vis), "imu": imu, "vel_vis": dev(np.zeros((n_kf, 3))),
                      "bias": dev(np.zeros((n_kf, 6))), "rot_wg": dev([0, 0, 0, 1.0]), "log_scale": dev([0.0]),
                      "cost": dev(np.zeros(iters + 1))})
    init = [{k: v.clone() for k, v in q.items()} for q in probs]

    def reset():
        for q, q0 in zip(probs, init):
            for k in ("vel_vis", "bias", "rot_wg", "log_scale"):
                q[k].copy_(q0[k])

    reset()
    ctx.inertial_init_solve(probs, iters=iters)
    best = 1e30
    for _ in range(reps):
        reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.inertial_init_solve(probs, iters=iters)
        best = min(best, time.perf_counter() - t0)
    c = torch.stack([q["cost"] for q in probs]).cpu().numpy()
    # the oracle on 2 of the 64 problems, same iterations, one core
    from threadpoolctl import threadpool_limits

    from oracle import inertial_init as oii
    from oracle import preint as opreint
    from oracle.so3 import quat_to_R
    n_cpu = 2
    dt_cpu = 0.0
    with threadpool_limits(limits=1):
        for w in range(n_cpu):
            ip = synth.make_inertial_init_problem(synth.tiny_config(n_kf=n_kf), 6000 + w, pose_noise=(2e-4, 0.01))
            fs = opreint.preintegrate_all(ip.imu_off, ip.gyro, ip.accel, ip.imu_dt, ip.bias_hat, ip.noise)
            Rv = np.stack([quat_to_R(q) for q in ip.pose_vis[:, 3:7]])
            st0 = oii.InitState(np.eye(3), 0.0, np.zeros((n_kf, 3)), np.zeros((n_kf, 6)))
            t0 = time.perf_counter()
            oii.solve(Rv, ip.pose_vis[:, :3], st0, fs, np.array([0.0, 0.0, -9.81]), iters)
            dt_cpu += time.perf_counter() - t0
    return {"cpu_baseline": {"value": 1e3 * dt_cpu / n_cpu, "unit": "ms per problem", "cores": 1, "kind": "oracle",
                             "sample": f"{n_cpu} of the {n} problems, {iters} iterations each (NumPy float64, "
                                       f"1 BLAS thread)"},
            "workload": f"{n} problems of {n_kf} keyframes (200 Hz IMU, 0.1 s gaps), visual poses with 0.2 mm / "
                        f"0.01 deg errors, frame tilted 25 deg and shrunk by e^-0.9, {iters} iterations, FP64",
            "ms_per_call": 1e3 * best, "median_cost_reduction": float(np.median(c[:, -1] / c[:, 0])),
            "roofline": {"bound": "latency", "note": "one 256-thread workgroup per problem; about 3 barriers per "
                                                     "keyframe per iteration in the block Cholesky"}}


def warm_windows(ctx, n=8, iters=5, reps=6):
    """Eight windows of the warm-start study, each solved alone: iters GN
    iterations plain, and the warm start followed by the same iterations."""
    import numpy as np
    import torch

    from paper_2512_02293_amd import warmstart
    probs = warmstart.eval_windows(n)
    opts = warmstart.study_opts()
    dps, imus = warmstart._upload(ctx, probs)
    nb = max(ctx.warm_start_workspace_size([d], opts) for d in dps)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
    theta = torch.as_tensor(np.load(warmstart.PARAMS_FILE), device="cuda:0")
    rows = []
    for d, im in zip(dps, imus):
        row = {"n_kf": int(d.pose.shape[0])}
        for mode in ("plain", "warm"):
            best = 1e30
            for _ in range(reps):
                d.reset_state()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if mode == "plain":
                    ctx.solve_batched([d], [im], opts, iters, ws)
                else:
                    ctx.solve_warm([d], [im], opts, theta, iters, ws)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            row[f"ms_{mode}"] = 1e3 * best
        rows.append(row)
    return {"workload": f"{n} warm-start evaluation windows, each alone, {iters} GN iterations plain vs warm start "
                        f"+ {iters} iterations", "windows": rows}


def host_description():
    """CPU model and core counts of the machine the benchmark runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cores": usable}


def _oracle_worker(j, n_workers, n_windows, barrier, queue):
    """Worker j of the all-core oracle timing: generates its share of the
    batched windows (j, j + n_workers, ...), waits for every worker, then runs
    one oracle GN step (with the oracle's own preintegration) on each and
    reports (pixel-residuals, start, end) on the wall clock."""
    from threadpoolctl import threadpool_limits

    from oracle import normal_eq as ne
    from oracle import solve as osolve
    from paper_2512_02293_amd import synth
    probs = [synth.make_problem(synth.config_batched_window(w), 4000 + w) for w in range(j, n_windows, n_workers)]
    barrier.wait()
    with threadpool_limits(limits=1):
        t0 = time.time()
        for prob in probs:
            cam, st, gr = osolve.from_problem(prob)
            osolve.step(cam, st, gr, ne.Options())
        t1 = time.time()
    queue.put((sum(p.n_edges * p.H * p.W for p in probs), t0, t1))


def cpu_baseline(prob, iters, all_cores=True):
    """The FP64 oracle on bounded samples: single-threaded on the benchmarked
    window, and on all usable host cores (a process pool, one batched window
    per task, each one GN step) on the 64-window batch."""
    from threadpoolctl import threadpool_limits

    from oracle import normal_eq as ne
    from oracle import solve as osolve
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        cam, st, gr = osolve.from_problem(prob)        # includes the oracle's preintegration
        st, _ = osolve.solve(cam, st, gr, ne.Options(), iters)
        dt = time.perf_counter() - t0
    pxres = prob.n_edges * prob.H * prob.W * iters
    host = host_description()
    out = {"value": pxres / dt, "unit": "pixel-residuals/s", "cores": 1, "kind": "oracle",
           "sample": f"oracle preintegration + {iters} of the 8 GN iterations on the same 24-KF window "
                     f"({dt:.1f} s, NumPy float64, 1 BLAS thread)", "host": host}
    if all_cores:
        import multiprocessing as mp
        workers = max(1, min(16, host["usable_cores"] or 1))
        n_windows = 64
        # fresh interpreters (spawn): the workers never touch the GPU
        mpc = mp.get_context("spawn")
        barrier, queue = mpc.Barrier(workers), mpc.Queue()
        procs = [mpc.Process(target=_oracle_worker, args=(j, workers, n_windows, barrier, queue))
                 for j in range(workers)]
        for pr in procs:
            pr.start()
        res = [queue.get(timeout=600) for _ in procs]
        for pr in procs:
            pr.join()
        wall = max(r[2] for r in res) - min(r[1] for r in res)
        px = sum(r[0] for r in res)
        out["all_cores"] = {"value": px / wall, "unit": "pixel-residuals/s", "cores": workers, "kind": "oracle",
                            "sample": f"one oracle GN step (with its preintegration) of each of the {n_windows} "
                                      f"batched windows, {workers} worker processes of 1 BLAS thread each "
                                      f"(windows generated before a common start), {wall:.1f} s wall"}
    return out


if __name__ == "__main__":
    main()

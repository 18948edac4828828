"""Learned warm start: training data from the solver itself, training with the
library's own network kernels, and the time-to-tolerance comparison against
plain Gauss-Newton.

Every arithmetic step runs in the library's kernels (vi_warm_features,
vi_warm_gradients, vi_warm_adamw, vi_warm_forward, vi_warm_apply and the
batched Gauss-Newton solve); this module only moves arrays and keeps the
bookkeeping (shuffling, label pooling of the solver's own outputs, timing).

Data: windows drawn from the batched-window distribution (N ~ U{8..32}
keyframes, 3-8 edges per keyframe, 48x64 or 60x80 maps, IMU gaps U{5..40})
with a spatially smooth 10 % initial inverse-depth error (a per-pixel white
error has no component a 4x4-cell correction can represent); training seeds
100000 and up, disjoint from the evaluation windows (seeds 4000..4063).  Labels: the converged plain Gauss-Newton solution minus the
initial state (inverse depths averaged over each 4 x 4 cell, biases per
keyframe).
"""
import os
import time
from multiprocessing import get_context

import numpy as np

from . import binding, synth

HQ, WQ = 15, 20                     # cell canvas of 48x64 and 60x80 maps
TRAIN_SEED0 = 100000
LABEL_ITERS = 10                    # plain GN iterations that define the converged solution
REF_ITERS = 30                      # plain GN iterations that define the reference (converged) cost
# Damping of the warm-start study.  The default Marquardt factor (1e-4 of the
# diagonal) nearly freezes the inertial bias/velocity directions, whose
# information entries reach ~1e10, so Gauss-Newton is still 1e-3 above its
# limit after 20 iterations; with 1e-6 it reaches 1e-6 of the converged cost
# in 4-6 iterations, which is the regime a warm start can shorten.
STUDY_LAMBDA = 1e-6


def study_opts():
    return binding.make_opts(lm_lambda=STUDY_LAMBDA)
PARAMS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "warm_params.npy")


def _make(seed, smooth=True):
    return synth.make_problem(synth.config_random_window(seed, smooth_depth_init=smooth), seed)


def eval_windows(n=64, smooth=True):
    """The evaluation windows of the time-to-tolerance comparison (smooth=False:
    the batched windows' own per-pixel initial depth error)."""
    return [_make(4000 + w, smooth) for w in range(n)]


def generate(seeds, workers=None):
    """Synthetic windows for the given seeds (CPU generator, in a process pool)."""
    workers = workers or min(16, os.cpu_count() or 1)
    if workers <= 1 or len(seeds) < 4:
        return [_make(s) for s in seeds]
    with get_context("spawn").Pool(workers) as pool:
        return pool.map(_make, list(seeds), chunksize=max(1, len(seeds) // (4 * workers)))


def cell_mean_canvas(a, H, W):
    """Mean of a (H, W) map over 4 x 4 cells, placed on the HQ x WQ canvas."""
    hq, wq = (H + 3) // 4, (W + 3) // 4
    pad = np.zeros((4 * hq, 4 * wq))
    cnt = np.zeros((4 * hq, 4 * wq))
    pad[:H, :W] = a
    cnt[:H, :W] = 1.0
    s = pad.reshape(hq, 4, wq, 4).sum(axis=(1, 3))
    n = cnt.reshape(hq, 4, wq, 4).sum(axis=(1, 3))
    out = np.zeros((HQ, WQ))
    out[:hq, :wq] = s / n
    return out


def he_normal(seed):
    """Initial parameters in the library's layout (W1 [32][15][3][3], b1, W2..W4
    [32][32][3][3], b2..b4, Wd [1][32][3][3], bd, Wb [6][32], bb): He-normal
    weights (std sqrt(2 / fan_in)) in the trunk, 1/100 of that in the two
    heads (the network starts close to the zero correction), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in ((32, 15, 3, 3), (32,), (32, 32, 3, 3), (32,), (32, 32, 3, 3), (32,), (32, 32, 3, 3), (32,),
                  (1, 32, 3, 3), (1,), (6, 32), (6,)):
        if len(shape) == 1:
            parts.append(np.zeros(shape))
        else:
            fan_in = int(np.prod(shape[1:]))
            head = shape[0] in (1, 6)
            parts.append(rng.standard_normal(shape) * np.sqrt(2.0 / fan_in) * (0.01 if head else 1.0))
    return np.concatenate([a.ravel() for a in parts]).astype(np.float32)


class WarmNet:
    """Parameters and AdamW state on the device."""

    def __init__(self, ctx, params=None, seed=0):
        import torch
        self.ctx = ctx
        self.P = int(ctx.lib.vi_warm_param_count())
        if params is None:
            params = he_normal(seed)
        p = np.asarray(params, np.float32)
        assert p.size == self.P
        self.params = torch.as_tensor(p, device="cuda:0").clone()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0

    def save(self, path=PARAMS_FILE):
        np.save(path, self.params.cpu().numpy())

    @classmethod
    def load(cls, ctx, path=PARAMS_FILE):
        return cls(ctx, params=np.load(path))

    def step(self, feat, dims, lab_dd, lab_db, n_valid, lr, workspace=None):
        loss, g = self.ctx.warm_gradients(self.params, feat, dims, lab_dd, lab_db, n_valid, workspace)
        self.t += 1
        self.ctx.warm_adamw(self.params, g, self.m, self.v, self.t, lr, weight_decay=1e-4)
        return loss


def _upload(ctx, probs):
    dps = [binding.DeviceProblem(p) for p in probs]
    imus = [ctx.imu_preintegrate(d.off, d.gyro, d.accel, d.imu_dt, d.bias_hat, d.noise) for d in dps]
    return dps, imus


def label_batch(ctx, probs, opts, iters=LABEL_ITERS):
    """Features at the initial state and the labels (converged plain GN minus
    the initial state) of a batch of windows.  Returns device tensors."""
    import torch
    dps, imus = _upload(ctx, probs)
    feat, dims = ctx.warm_features(dps, imus, opts, HQ, WQ)
    nb = ctx.workspace_size_batched(dps, opts)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
    ctx.solve_batched(dps, imus, opts, iters, ws)
    lab_dd, lab_db = [], []
    for p, d in zip(probs, dps):
        dfin = d.invdepth.cpu().numpy()
        bfin = d.bias.cpu().numpy()
        for i in range(p.n_kf):
            lab_dd.append(cell_mean_canvas(dfin[i] - p.invdepth[i], p.H, p.W))
        lab_db.append(bfin - p.bias)
    lab_dd = torch.as_tensor(np.stack(lab_dd).astype(np.float32), device="cuda:0")
    lab_db = torch.as_tensor(np.concatenate(lab_db).astype(np.float32), device="cuda:0")
    return feat, dims, lab_dd, lab_db


def build_dataset(ctx, n_windows, opts, batch=64, workers=None, log=print):
    """Generate, solve and label n_windows training windows."""
    import torch
    feats, dimss, ldds, ldbs = [], [], [], []
    t0 = time.time()
    seeds = list(range(TRAIN_SEED0, TRAIN_SEED0 + n_windows))
    chunk = 16 * batch
    for c0 in range(0, n_windows, chunk):
        probs_all = generate(seeds[c0:c0 + chunk], workers)
        for b0 in range(0, len(probs_all), batch):
            f, d, ldd, ldb = label_batch(ctx, probs_all[b0:b0 + batch], opts)
            feats.append(f)
            dimss.append(d)
            ldds.append(ldd)
            ldbs.append(ldb)
        log(f"dataset: {min(c0 + chunk, n_windows)}/{n_windows} windows, {time.time() - t0:.0f} s")
    return torch.cat(feats), torch.cat(dimss), torch.cat(ldds), torch.cat(ldbs)


def dataset_loss(ctx, params, data, batch=256, max_batches=32):
    """Mean training loss of the given parameters over the first batches."""
    import torch
    feat, dims, ldd, ldb = data
    n = feat.shape[0]
    ws = torch.empty(int(ctx.lib.vi_warm_workspace_size(batch, HQ, WQ)), dtype=torch.uint8, device=feat.device)
    tot, cnt = 0.0, 0
    for s in range(0, min(n - batch + 1, max_batches * batch), batch):
        sl = slice(s, s + batch)
        nv = float((dims[sl, 0] * dims[sl, 1]).sum())
        loss, _ = ctx.warm_gradients(params, feat[sl].contiguous(), dims[sl].contiguous(), ldd[sl].contiguous(),
                                     ldb[sl].contiguous(), nv, ws)
        tot += loss
        cnt += 1
    return tot / max(cnt, 1)


def train(ctx, net, data, epochs, batch=256, lr=2e-3, log=print, seed=0):
    import torch
    feat, dims, ldd, ldb = data
    n = feat.shape[0]
    valid = (dims[:, 0] * dims[:, 1]).to(torch.float64)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    ws = None
    hist = []
    steps_per_epoch = n // batch
    total = epochs * steps_per_epoch
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen).to(feat.device)
        run = 0.0
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            f, d, a, b = feat[idx].contiguous(), dims[idx].contiguous(), ldd[idx].contiguous(), ldb[idx].contiguous()
            nv = float(valid[idx].sum())
            # cosine learning-rate decay
            lr_k = lr * 0.5 * (1.0 + np.cos(np.pi * k / max(total, 1)))
            if ws is None:
                import torch as _t
                ws = _t.empty(int(ctx.lib.vi_warm_workspace_size(batch, HQ, WQ)), dtype=_t.uint8, device=feat.device)
            run += net.step(f, d, a, b, nv, lr_k, ws)
            k += 1
        hist.append(run / max(steps_per_epoch, 1))
        log(f"epoch {ep}: mean loss {hist[-1]:.4f}")
    return hist


# ---------------------------------------------------------------------------
# time to tolerance
# ---------------------------------------------------------------------------
def _iters_to_tol(costs, target):
    hit = np.nonzero(costs <= target)[0]
    return int(hit[0]) if hit.size else None


def time_to_tol(ctx, net, probs, opts, max_iters=REF_ITERS, rel_tol=1e-6, reps=3, stop_tol=1e-7):
    """Plain GN from the initial state vs the learned warm start (with the
    plain cost as the arbiter, vi_warm_start) followed by GN.

    The target of every window is its plain-GN cost after max_iters
    iterations (converged) times (1 + rel_tol); k_plain / k_warm are the GN
    iterations each way until a window's cost is at or below its target (a
    window whose corrections were rejected starts from its initial state, so
    its k_warm is its k_plain).  Wall times (best of reps, GPU synchronised):
      * batch: all windows in the same launches, which need the largest
        count of any window: K_plain vs warm start + K_warm iterations;
      * per window: each window alone, as a sliding-window solver runs it,
        k_plain(w) iterations vs warm start + k_warm(w) iterations, summed
        over the windows.
    The warm path is one vi_ba_solve_warm call (warm start and GN in one
    graph); the plain path one vi_ba_solve_batched call.
      * batch with the tolerance stop (vi_ctx_set_tolerance, stop_tol): the
        same max(K_plain, K_warm) launches each way, every window frozen once
        its relative cost decrease falls to stop_tol, so that the time follows
        the work of the windows still iterating; reported with how many
        windows end at or below their target."""
    import torch
    dps, imus = _upload(ctx, probs)
    nb = max(ctx.workspace_size_batched(dps, opts), ctx.warm_start_workspace_size(dps, opts))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda:0")

    def reset(sel=None):
        for d in (dps if sel is None else sel):
            d.reset_state()
        torch.cuda.synchronize()

    # reference costs of plain GN
    reset()
    reps_plain = ctx.solve_batched(dps, imus, opts, max_iters, ws, costs=True)
    plain_costs = [r["costs"] for r in reps_plain]
    target = [c[-1] * (1.0 + rel_tol) for c in plain_costs]
    k_plain = [_iters_to_tol(c, t) for c, t in zip(plain_costs, target)]
    # warm start (rejections put back on the device), then GN
    reset()
    wres = ctx.warm_start(dps, imus, opts, net.params, ws)
    reps_w = ctx.solve_batched(dps, imus, opts, max_iters, ws, costs=True)
    warm_costs = [r["costs"] for r in reps_w]
    accepted = [r["accepted"] for r in wres]
    k_warm, reached = [], []
    for w, t in zip(warm_costs, target):
        k = _iters_to_tol(w, t)
        reached.append(k is not None)
        k_warm.append(k if k is not None else max_iters)
    K_plain, K_warm = max(k_plain), max(k_warm)

    def timed(fn, sel=None):
        best = 1e30
        for _ in range(reps):
            reset(sel)
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best

    def gn(sel_d, sel_i, k):
        if k > 0:
            ctx.solve_batched(sel_d, sel_i, opts, k, ws)

    def warm(sel_d, sel_i, k):
        ctx.solve_warm(sel_d, sel_i, opts, net.params, k, ws)

    t_batch_plain = timed(lambda: gn(dps, imus, K_plain))
    t_batch_warm = timed(lambda: warm(dps, imus, K_warm))
    K = max(K_plain, K_warm)
    ctx.set_tolerance(stop_tol)
    try:
        reset()
        stop_plain = ctx.solve_batched(dps, imus, opts, K, ws)
        reset()
        stop_warm = ctx.solve_warm(dps, imus, opts, net.params, K, ws)
        t_stop_plain = timed(lambda: gn(dps, imus, K))
        t_stop_warm = timed(lambda: warm(dps, imus, K))
    finally:
        ctx.set_tolerance(0.0)
    stop = dict(tol=stop_tol, iters=K, ms_plain=1e3 * t_stop_plain, ms_warm=1e3 * t_stop_warm,
                steps_plain=int(sum(r["iters_done"] for r in stop_plain)),
                steps_warm=int(sum(r["iters_done"] for r in stop_warm)),
                reached_plain=int(sum(bool(r["cost_after"] <= t) for r, t in zip(stop_plain, target))),
                reached_warm=int(sum(bool(r["cost_after"] <= t) for r, t in zip(stop_warm, target))))
    t_win_plain = t_win_warm = 0.0
    for d, im, kp, kw in zip(dps, imus, k_plain, k_warm):
        gn([d], [im], kp)                               # graph of this shape and count, captured once
        t_win_plain += timed(lambda: gn([d], [im], kp), [d])
        warm([d], [im], kw)
        t_win_warm += timed(lambda: warm([d], [im], kw), [d])
    # each window alone with the stopping rule instead of a known iteration
    # count: up to K iterations, frozen once its relative cost decrease falls
    # to stop_tol (what a sliding-window solver without a reference run does)
    t_ws_plain = t_ws_warm = 0.0
    ws_reached_plain = ws_reached_warm = 0
    ws_steps_plain = ws_steps_warm = 0
    ctx.set_tolerance(stop_tol)
    try:
        for d, im, t in zip(dps, imus, target):
            reset([d])
            r = ctx.solve_batched([d], [im], opts, K, ws)[0]
            ws_reached_plain += int(r["cost_after"] <= t)
            ws_steps_plain += int(r["iters_done"])
            t_ws_plain += timed(lambda: gn([d], [im], K), [d])
            reset([d])
            r = ctx.solve_warm([d], [im], opts, net.params, K, ws)[0]
            ws_reached_warm += int(r["cost_after"] <= t)
            ws_steps_warm += int(r["iters_done"])
            t_ws_warm += timed(lambda: warm([d], [im], K), [d])
    finally:
        ctx.set_tolerance(0.0)
    per_window_stop = dict(tol=stop_tol, max_iters=K, ms_plain_total=1e3 * t_ws_plain,
                           ms_warm_total=1e3 * t_ws_warm, steps_plain=ws_steps_plain, steps_warm=ws_steps_warm,
                           reached_plain=ws_reached_plain, reached_warm=ws_reached_warm)
    return dict(k_plain=k_plain, k_warm=k_warm, accepted=accepted, reached=reached, K_plain=K_plain, K_warm=K_warm,
                ms_plain=1e3 * t_batch_plain, ms_warm=1e3 * t_batch_warm,
                ms_plain_per_window_total=1e3 * t_win_plain, ms_warm_per_window_total=1e3 * t_win_warm,
                final_plain=[c[-1] for c in plain_costs], final_warm=[c[-1] for c in warm_costs], stop=stop,
                per_window_stop=per_window_stop)

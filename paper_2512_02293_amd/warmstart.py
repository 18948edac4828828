"""Learned warm start: training data from the solver itself, training with the
library's own network kernels, and the time-to-tolerance comparison against
plain Gauss-Newton.

Every arithmetic step runs in the library's kernels (vi_warm_features,
vi_warm_gradients, vi_warm_adamw, vi_warm_forward, vi_warm_apply and the
batched Gauss-Newton solve); this module only moves arrays and keeps the
bookkeeping (shuffling, label pooling of the solver's own outputs, timing).

Data: windows drawn from the batched-window distribution (N ~ U{8..32}
keyframes, 3-8 edges per keyframe, 48x64 or 60x80 maps, IMU gaps U{5..40}),
training seeds 100000 and up, disjoint from the evaluation windows (seeds
4000..4063).  Labels: the converged plain Gauss-Newton solution minus the
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


def _make(seed):
    return synth.make_problem(synth.config_random_window(seed), seed)


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
    """Initial parameters in the library's layout (W1 [32][13][3][3], b1, W2..W4
    [32][32][3][3], b2..b4, Wd [1][32][3][3], bd, Wb [6][32], bb): He-normal
    weights (std sqrt(2 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in ((32, 13, 3, 3), (32,), (32, 32, 3, 3), (32,), (32, 32, 3, 3), (32,), (32, 32, 3, 3), (32,),
                  (1, 32, 3, 3), (1,), (6, 32), (6,)):
        if len(shape) == 1:
            parts.append(np.zeros(shape))
        else:
            fan_in = int(np.prod(shape[1:]))
            parts.append(rng.standard_normal(shape) * np.sqrt(2.0 / fan_in))
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


def time_to_tol(ctx, net, probs, opts, max_iters=REF_ITERS, rel_tol=1e-6, reps=5):
    """Plain GN from the initial state vs warm start + GN, on one batch.

    The target of every window is its plain-GN cost after max_iters
    iterations (converged) times (1 + rel_tol).  A window's warm start is kept
    only if its cost is below the plain initial cost (else it restarts from
    the initial state).  Returns per-window iteration counts and the wall time
    of the whole batch to reach every window's target, both ways."""
    import torch
    dps, imus = _upload(ctx, probs)
    nb = ctx.workspace_size_batched(dps, opts)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda:0")

    def reset():
        for d in dps:
            d.reset_state()
        torch.cuda.synchronize()

    # reference costs of plain GN
    reset()
    reps_plain = ctx.solve_batched(dps, imus, opts, max_iters, ws, costs=True)
    plain_costs = [r["costs"] for r in reps_plain]
    target = [c[-1] * (1.0 + rel_tol) for c in plain_costs]
    k_plain = [_iters_to_tol(c, t) for c, t in zip(plain_costs, target)]
    # warm start: features, network, apply, then GN
    reset()
    feat, dims = ctx.warm_features(dps, imus, opts, HQ, WQ)
    dd, db = ctx.warm_forward(net.params, feat, dims)
    ctx.warm_apply(dps, imus, opts, dd, db)
    reps_w = ctx.solve_batched(dps, imus, opts, max_iters, ws, costs=True)
    warm_costs = [r["costs"] for r in reps_w]
    accepted = [w[0] < p[0] for w, p in zip(warm_costs, plain_costs)]
    k_warm, reached = [], []
    for w, t, a, kp in zip(warm_costs, target, accepted, k_plain):
        k = _iters_to_tol(w, t) if a else kp
        reached.append(k is not None)
        k_warm.append(k if k is not None else max_iters)
    K_plain = max(k_plain)
    K_warm = max(k_warm)
    # a window whose warm start was rejected restarts from the initial state
    # inside the same batch, so the batch needs the larger of the two counts

    # wall time: the batch needs K iterations (all windows run in the same launches)
    def timed(fn):
        best = 1e30
        for _ in range(reps):
            reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best

    def plain_run():
        ctx.solve_batched(dps, imus, opts, max(K_plain, 1), ws)

    def warm_run():
        f, d = ctx.warm_features(dps, imus, opts, HQ, WQ)
        a, b = ctx.warm_forward(net.params, f, d)
        ctx.warm_apply(dps, imus, opts, a, b)
        if K_warm > 0:
            ctx.solve_batched(dps, imus, opts, K_warm, ws)

    t_plain = timed(plain_run)
    t_warm = timed(warm_run)
    return dict(k_plain=k_plain, k_warm=k_warm, accepted=accepted, reached=reached, K_plain=K_plain, K_warm=K_warm,
                ms_plain=1e3 * t_plain, ms_warm=1e3 * t_warm,
                final_plain=[c[-1] for c in plain_costs], final_warm=[c[-1] for c in warm_costs])

"""Train the warm-start network on windows the solver itself generates and
solves, then compare time to tolerance against plain Gauss-Newton.

    python -m paper_2512_02293_amd.train_warm [--windows 20000] [--epochs 40] [--out PATH]

Needs a GPU.  Prints one progress line per dataset chunk and per epoch, then a
JSON summary line (loss history, iteration counts and times to tolerance of
the 64-window evaluation batch, both ways).
"""
import argparse
import json
import sys
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--windows", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=40)   # the committed parameters were trained with 40
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out", default=None)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args(argv)

    from . import binding, warmstart
    log = lambda m: print(m, flush=True)
    import torch
    ctx = binding.Context(0)
    opts = warmstart.study_opts()
    t0 = time.time()
    data = warmstart.build_dataset(ctx, args.windows, opts, workers=args.workers, log=log)
    t_data = time.time() - t0
    log(f"dataset ready: {data[0].shape[0]} keyframe images in {t_data:.0f} s")
    # held-out tail for an evaluation loss; the zero predictor as the baseline
    n = data[0].shape[0]
    n_val = min(n // 10, 8192)
    train_data = tuple(t[: n - n_val] for t in data)
    val_data = tuple(t[n - n_val:] for t in data)
    zero = torch.zeros(int(ctx.lib.vi_warm_param_count()), dtype=torch.float32, device="cuda:0")
    loss_zero = warmstart.dataset_loss(ctx, zero, val_data)
    net = warmstart.WarmNet(ctx, seed=args.seed)
    t1 = time.time()
    hist = warmstart.train(ctx, net, train_data, args.epochs, batch=args.batch, lr=args.lr, log=log,
                           seed=args.seed)
    t_train = time.time() - t1
    loss_val = warmstart.dataset_loss(ctx, net.params, val_data)
    log(f"held-out loss {loss_val:.4f} (zero predictor {loss_zero:.4f})")
    out = args.out or warmstart.PARAMS_FILE
    net.save(out)
    log(f"trained in {t_train:.1f} s, parameters saved to {out}")
    evalp = warmstart.eval_windows()
    res = warmstart.time_to_tol(ctx, net, evalp, opts)
    summary = dict(windows=args.windows, images=int(data[0].shape[0]), epochs=args.epochs, loss=hist,
                   loss_heldout=loss_val, loss_heldout_zero_predictor=loss_zero,
                   dataset_s=t_data, train_s=t_train, eval_windows=64,
                   iters_plain_mean=float(np.mean(res["k_plain"])), iters_warm_mean=float(np.mean(res["k_warm"])),
                   K_plain=res["K_plain"], K_warm=res["K_warm"], accepted=int(sum(res["accepted"])),
                   ms_plain=res["ms_plain"], ms_warm=res["ms_warm"],
                   ms_plain_per_window_total=res["ms_plain_per_window_total"],
                   ms_warm_per_window_total=res["ms_warm_per_window_total"])
    print(json.dumps(summary), flush=True)
    ctx.close()


if __name__ == "__main__":
    sys.exit(main())

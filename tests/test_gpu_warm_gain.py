"""What the trained warm-start network gains over plain Gauss-Newton.

The committed parameters (paper_2512_02293_amd/warm_params.npy) were trained
by the library's own kernels (python -m paper_2512_02293_amd.train_warm) on
20 000 windows with seeds 100000 and up.  Here, on the 64 evaluation windows
(seeds 4000..4063, never seen in training), each window's target is its plain
GN cost after 30 iterations times (1 + 1e-6); the test counts the GN
iterations each way to reach it, with vi_warm_start (corrections kept only
where the cost falls) before GN.

Asserted: every window reaches its target both ways (the fallback keeps the
warm path from ending worse), and the mean iteration count falls by at least
0.5 (measured when the parameters were committed: 5.89 -> 5.02).  Wall times
are printed, not asserted: the batch (one set of launches for all windows)
is bounded by the slowest window, which the warm start does not speed up.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_trained_warm_start_saves_gauss_newton_iterations():
    import torch
    from paper_2512_02293_amd import binding, warmstart
    assert torch.cuda.is_available()
    ctx = binding.Context(0)
    try:
        net = warmstart.WarmNet.load(ctx)
        r = warmstart.time_to_tol(ctx, net, warmstart.eval_windows(), warmstart.study_opts())
    finally:
        ctx.close()
    kp, kw = np.array(r["k_plain"]), np.array(r["k_warm"])
    print(f"GN iterations to 1e-6 of the converged cost: plain mean {kp.mean():.3f} max {kp.max()}, "
          f"warm mean {kw.mean():.3f} max {kw.max()}; warm start kept in {sum(r['accepted'])}/64 windows; "
          f"fewer iterations in {int((kw < kp).sum())}, more in {int((kw > kp).sum())}")
    print(f"wall time: batch {r['ms_plain']:.2f} ms plain vs {r['ms_warm']:.2f} ms warm; one window at a time "
          f"{r['ms_plain_per_window_total']:.2f} ms vs {r['ms_warm_per_window_total']:.2f} ms in total")
    assert all(r["reached"])
    assert kw.mean() <= kp.mean() - 0.5

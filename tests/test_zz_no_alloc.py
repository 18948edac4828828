"""The allocation-free Gaussian-map update (vi_gaussian_reanchor_noalloc)
against the workspace entry point (vi_gaussian_reanchor), through the C ABI.

Both run the same kernels on the same inputs, so their outputs and rejection
counts must agree bit for bit.  Two calls in a row on one context, the second
with fewer keyframes and Gaussians (the library's table then still holds rows
of the first call beyond the second call's keyframes; anchors pointing there
must be rejected, not read), plus the size limit of the fixed table.
"""
import numpy as np
import pytest

from paper_2512_02293_amd import synth

pytestmark = pytest.mark.gpu


def _map(n_kf, per_kf, seed, bad_anchor_at=None):
    import torch
    g = synth.make_gaussian_map(n_kf, per_kf, seed, H=120, W=160)
    anchor = g.anchor.copy()
    ds = g.scale_change.copy()
    ds[1] = -1.0                                  # an invalid keyframe update: its Gaussians are rejected
    if bad_anchor_at is not None:
        anchor[::97] = bad_anchor_at              # anchors beyond this call's keyframes
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")
    return dict(pre=dev(g.pose_pre), post=dev(g.pose_post), ds=dev(ds), anchor=dev(anchor), mean=dev(g.mean),
                cov=dev(g.cov))


def _run(ctx, m, ws):
    import torch
    mo, co = torch.empty_like(m["mean"]), torch.empty_like(m["cov"])
    nrej = torch.full((1,), -7, dtype=torch.int32, device="cuda:0")
    ctx.gaussian_reanchor(m["pre"], m["post"], m["ds"], m["anchor"], m["mean"], m["cov"], mo, co, ws=ws,
                          n_rejected=nrej)
    torch.cuda.synchronize()
    return mo.cpu().numpy(), co.cpu().numpy(), int(nrej.cpu().item())


def test_noalloc_matches_workspace_entry_point():
    import torch
    from paper_2512_02293_amd import binding
    assert torch.cuda.is_available()
    ctx = binding.Context(0)
    try:
        big = _map(300, 700, 21)
        small = _map(40, 333, 22, bad_anchor_at=150)
        for m, n_kf in ((big, 300), (small, 40)):
            ws = torch.empty(ctx.reanchor_workspace_size(n_kf), dtype=torch.uint8, device="cuda:0")
            ref = _run(ctx, m, ws)
            got = _run(ctx, m, "noalloc")
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), n_kf
            assert got[2] == ref[2] and ref[2] > 0, (got[2], ref[2])
        # means only (no covariances), in place
        m = small
        ws = torch.empty(ctx.reanchor_workspace_size(40), dtype=torch.uint8, device="cuda:0")
        a, b = m["mean"].clone(), m["mean"].clone()
        ctx.gaussian_reanchor(m["pre"], m["post"], m["ds"], m["anchor"], a, ws=ws)
        ctx.gaussian_reanchor(m["pre"], m["post"], m["ds"], m["anchor"], b, ws="noalloc")
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        # beyond the fixed table: a clear error, nothing launched
        n = 16385
        pose = torch.zeros((n, 7), dtype=torch.float64, device="cuda:0")
        pose[:, 6] = 1.0
        ds = torch.ones(n, dtype=torch.float64, device="cuda:0")
        with pytest.raises(binding.ViError) as ei:
            ctx.gaussian_reanchor(pose, pose, ds, m["anchor"], m["mean"].clone(), ws="noalloc")
        assert ei.value.code == binding.VI_EINVAL and "16384" in str(ei.value)
    finally:
        ctx.close()

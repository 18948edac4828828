"""Loop-closure update of a Gaussian map (Eq. 7-8) on the GPU against the FP64
oracle, through the C ABI.

Tolerances come from the arithmetic of the GPU path: it folds each keyframe's
poses and scale into x -> A x + b in FP64, rounds A and b to FP32 and applies
them with FP32 fused multiply-adds to inputs that are exact FP32 values.  Per
output entry the error is then at most a few units of eps = 2^-24 times the
sum of the magnitudes it is built from:
  mean:        |err_r| <= 10 eps (sum_c |A_rc| |mu_c| + |b_r|)
  covariance:  |err_rc| <= 16 eps (|A| |Sigma| |A|^T)_rc
with |A|, |b| computed here in FP64 from the poses.  Rejected Gaussians and
the rejection count are compared exactly.
"""
import numpy as np
import pytest

from oracle import gauss as og
from oracle.so3 import quat_to_R
from paper_2512_02293_amd import synth

pytestmark = pytest.mark.gpu
EPS32 = 2.0 ** -24


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2512_02293_amd import binding
    assert torch.cuda.is_available()
    c = binding.Context(0)
    yield c
    c.close()


def _abs_affine(g):
    """|A| [N][3][3] and |b| [N][3] of every keyframe, FP64."""
    N = len(g.pose_pre)
    A = np.zeros((N, 3, 3))
    b = np.zeros((N, 3))
    valid = og.keyframe_valid(g.pose_pre, g.pose_post, g.scale_change)
    for k in np.flatnonzero(valid):
        Rm, Rp = quat_to_R(g.pose_pre[k, 3:7]), quat_to_R(g.pose_post[k, 3:7])
        Ak = g.scale_change[k] * Rp @ Rm.T
        A[k] = np.abs(Ak)
        b[k] = np.abs(g.pose_post[k, :3] - Ak @ g.pose_pre[k, :3])
    return A, b


def _check(g, idx, mean_gpu, cov_gpu, mean_ref, cov_ref, rej):
    A, b = _abs_affine(g)
    ok = ~rej
    k = g.anchor[idx][ok]
    mu = np.abs(g.mean[idx][ok].astype(np.float64))
    bound_m = 10 * EPS32 * (np.einsum("kij,kj->ki", A[k], mu) + b[k])
    err_m = np.abs(mean_gpu[ok].astype(np.float64) - mean_ref[ok])
    assert np.all(err_m <= bound_m), float((err_m / bound_m).max())
    # rejected: copied exactly
    np.testing.assert_array_equal(mean_gpu[~ok], g.mean[idx][~ok])
    if cov_gpu is not None:
        S = np.abs(og.cov6_to_mat(g.cov[idx][ok]))
        bound_c = og.mat_to_cov6(16 * EPS32 * np.einsum("kij,kjl,kml->kim", A[k], S, A[k]))
        err_c = np.abs(cov_gpu[ok].astype(np.float64) - cov_ref[ok])
        assert np.all(err_c <= bound_c), float((err_c / bound_c).max())
        np.testing.assert_array_equal(cov_gpu[~ok], g.cov[idx][~ok])
    return float((err_m / bound_m).max()) if ok.any() else 0.0


def _run(ctx, g, cov=True, inplace=False, offset=0):
    """Upload, update on the GPU, return host results and the rejection count.
    offset > 0 places every array `offset` elements into a larger buffer, so
    that none is 16-byte aligned (the element-wise path)."""
    import torch

    def dev(a):
        a = np.ascontiguousarray(a)
        if offset == 0:
            return torch.as_tensor(a, device="cuda:0")
        flat = torch.zeros(a.size + offset, dtype=torch.as_tensor(a[:0]).dtype, device="cuda:0")
        flat[offset:] = torch.as_tensor(a.reshape(-1), device="cuda:0")
        return flat[offset:].view(a.shape)

    pre, post, ds = (torch.as_tensor(x, device="cuda:0") for x in (g.pose_pre, g.pose_post, g.scale_change))
    anchor, mean = dev(g.anchor), dev(g.mean)
    c = dev(g.cov) if cov else None
    if inplace:
        mo, co = None, None
    else:
        mo = dev(np.full_like(g.mean, np.nan))
        co = dev(np.full_like(g.cov, np.nan)) if cov else None
    nrej = torch.full((1,), -7, dtype=torch.int32, device="cuda:0")
    ctx.gaussian_reanchor(pre, post, ds, anchor, mean, c, mo, co, n_rejected=nrej)
    torch.cuda.synchronize()
    m_out = (mean if inplace else mo).cpu().numpy()
    c_out = None if not cov else (c if inplace else co).cpu().numpy()
    return m_out, c_out, int(nrej.item())


CASES = [  # (n_kf, per_kf, reorder_frac, cov, inplace, offset)
    (3, 0, 0.0, True, False, 0),          # empty map
    (2, 1, 0.0, True, False, 0),          # 2 Gaussians: one partial quad
    (5, 1, 0.0, True, True, 0),           # 5: one full quad + a ragged tail
    (7, 587, 0.5, True, False, 0),        # 4109: mixed anchors in most quads
    (16, 6250, 0.05, True, True, 0),      # 100000, in place
    (16, 6250, 0.05, False, False, 0),    # means only
    (9, 1111, 0.05, True, False, 1),      # misaligned arrays: element-wise path
    (9, 1111, 0.05, False, True, 3),      # misaligned, means only, in place
]


@pytest.mark.parametrize("n_kf,per_kf,frac,cov,inplace,offset", CASES)
def test_reanchor_matches_oracle(ctx, n_kf, per_kf, frac, cov, inplace, offset):
    g = synth.make_gaussian_map(n_kf, per_kf, 100 + n_kf * 7 + per_kf, reorder_frac=frac)
    m, c, nrej = _run(ctx, g, cov, inplace, offset)
    mr, cr, rej = og.reanchor(g.mean, g.cov if cov else None, g.anchor, g.pose_pre, g.pose_post, g.scale_change)
    assert nrej == int(rej.sum()) == 0
    r = _check(g, np.arange(len(g.mean)), m, c, mr, cr, rej)
    print(f"K={len(g.mean)} cov={cov} inplace={inplace} offset={offset}: max error / bound {r:.3f}", flush=True)


def test_reanchor_rejections(ctx):
    g = synth.make_gaussian_map(8, 301, 77, reorder_frac=0.3)
    g.scale_change[1] = 0.0
    g.scale_change[2] = np.nan
    g.scale_change[3] = -1.0
    g.pose_post[4, 0] = np.inf
    g.pose_pre[5, 3:7] = 0.0
    g.anchor[::97] = -1
    g.anchor[5::89] = 8
    m, c, nrej = _run(ctx, g)
    mr, cr, rej = og.reanchor(g.mean, g.cov, g.anchor, g.pose_pre, g.pose_post, g.scale_change)
    assert rej.sum() > 0 and (~rej).sum() > 0
    assert nrej == int(rej.sum())
    _check(g, np.arange(len(g.mean)), m, c, mr, cr, rej)


@pytest.mark.timeout(300)
def test_reanchor_full_size_sampled(ctx):
    """The benchmarked map (512 keyframes x 16384 Gaussians, seed 11), in the
    same out-of-place launch; 200k sampled Gaussians against the oracle, all
    outputs finite."""
    import torch
    g = synth.make_gaussian_map(512, 16384, 11)
    dev = lambda a: torch.as_tensor(a, device="cuda:0")
    mean, cov = dev(g.mean), dev(g.cov)
    mo, co = torch.empty_like(mean), torch.empty_like(cov)
    nrej = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    ctx.gaussian_reanchor(dev(g.pose_pre), dev(g.pose_post), dev(g.scale_change), dev(g.anchor), mean, cov, mo, co,
                          n_rejected=nrej)
    torch.cuda.synchronize()
    assert int(nrej.item()) == 0
    assert bool(torch.isfinite(mo).all()) and bool(torch.isfinite(co).all())
    idx = np.sort(np.random.default_rng(0).choice(len(g.mean), 200_000, replace=False))
    idx_t = torch.as_tensor(idx, device="cuda:0")
    m, c = mo[idx_t].cpu().numpy(), co[idx_t].cpu().numpy()
    mr, cr, rej = og.reanchor(g.mean[idx], g.cov[idx], g.anchor[idx], g.pose_pre, g.pose_post, g.scale_change)
    r = _check(g, idx, m, c, mr, cr, rej)
    print(f"full size: max error / bound {r:.3f}", flush=True)


def test_reanchor_host_errors(ctx):
    import torch
    from paper_2512_02293_amd import binding
    g = synth.make_gaussian_map(4, 64, 5)
    dev = lambda a: torch.as_tensor(a, device="cuda:0")
    pre, post, ds, anchor = dev(g.pose_pre), dev(g.pose_post), dev(g.scale_change), dev(g.anchor)
    buf = torch.zeros(3 * 256 + 6, dtype=torch.float32, device="cuda:0")
    mean = buf[:768].view(256, 3)
    shifted = buf[6:774].view(256, 3)             # overlaps mean, not equal to it
    with pytest.raises(binding.ViError, match="EINVAL"):
        ctx.gaussian_reanchor(pre, post, ds, anchor, mean, None, shifted)
    small = torch.empty(16, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(binding.ViError, match="ENOMEM"):
        ctx.gaussian_reanchor(pre, post, ds, anchor, dev(g.mean), ws=small)
    lib, h = ctx.lib, ctx.h
    gs = binding.Gaussians(256, anchor.data_ptr(), mean.data_ptr(), dev(g.cov).data_ptr(), mean.data_ptr(), None)
    ws = torch.empty(256, dtype=torch.uint8, device="cuda:0")
    import ctypes as C
    rc = lib.vi_gaussian_reanchor(h, 4, C.c_void_p(pre.data_ptr()), C.c_void_p(post.data_ptr()),
                                  C.c_void_p(ds.data_ptr()), C.byref(gs), C.c_void_p(ws.data_ptr()), 256, None)
    assert rc == binding.VI_EINVAL                 # cov_in without cov_out
    gs = binding.Gaussians(-1, anchor.data_ptr(), mean.data_ptr(), None, mean.data_ptr(), None)
    rc = lib.vi_gaussian_reanchor(h, 4, C.c_void_p(pre.data_ptr()), C.c_void_p(post.data_ptr()),
                                  C.c_void_p(ds.data_ptr()), C.byref(gs), C.c_void_p(ws.data_ptr()), 256, None)
    assert rc == binding.VI_EINVAL                 # negative count

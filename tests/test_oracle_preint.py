"""Pins of the oracle's IMU preintegration: exact closed forms, first-order
convergence to the continuous closed form, bias Jacobians by finite
differences, and the covariance by Monte Carlo."""
import numpy as np
import pytest
import scipy.linalg

from oracle import preint, so3

NO_NOISE = (0.0, 0.0, 0.0, 0.0)


def _run(omega, acc, n, h, bias=np.zeros(6), noise=(1.7e-4, 2e-3, 2e-5, 3e-3)):
    gyro = np.tile(omega, (n, 1))
    accel = np.tile(acc, (n, 1))
    return preint.preintegrate(gyro, accel, np.full(n, h), bias, *noise)


def test_constant_acceleration_zero_rate_is_exact():
    a = np.array([0.3, -1.2, 9.9])
    n, h = 37, 0.005
    P = _run(np.zeros(3), a, n, h)
    t = n * h
    assert np.allclose(P.dR, np.eye(3), atol=0)
    assert np.allclose(P.dv, a * t, rtol=1e-14, atol=1e-15)
    assert np.allclose(P.dp, 0.5 * a * t * t, rtol=1e-14, atol=1e-15)
    assert P.dt == pytest.approx(t, rel=1e-15)


def test_constant_rate_zero_acceleration_is_exact():
    w = np.array([0.4, -0.7, 1.3])
    n, h = 50, 0.005
    P = _run(w, np.zeros(3), n, h)
    assert np.allclose(P.dR, scipy.linalg.expm(so3.hat(w * n * h)), atol=1e-14)
    assert np.abs(P.dv).max() == 0.0 and np.abs(P.dp).max() == 0.0


def _geometric_closed_form(w, a, n, h):
    """dR, dv, dp for constant rate and acceleration held over n samples:
    dv = h sum_m R^m a, dp = h^2 sum_m (n-1-m) R^m a + h dv / 2, R = Exp(w h),
    with the sums of R^m = I + sin(m th) K + (1 - cos(m th)) K^2 in closed form
    through complex geometric series."""
    phi = w * h
    th = np.linalg.norm(phi)
    K = so3.hat(phi / th)
    z = np.exp(1j * th)
    s1 = (1 - z ** n) / (1 - z)                                 # sum z^m
    sm = z * (1 - n * z ** (n - 1) + (n - 1) * z ** n) / (1 - z) ** 2   # sum m z^m
    s2 = (n - 1) * s1 - sm                                      # sum (n-1-m) z^m
    c0 = n * (n - 1) / 2.0
    M1 = n * np.eye(3) + s1.imag * K + (n - s1.real) * (K @ K)
    M2 = c0 * np.eye(3) + s2.imag * K + (c0 - s2.real) * (K @ K)
    dv = h * M1 @ a
    dp = h * h * M2 @ a + 0.5 * h * dv
    return scipy.linalg.expm(so3.hat(phi * n)), dv, dp


@pytest.mark.parametrize("n", [1, 2, 20, 63])
def test_constant_rate_and_acceleration_discrete_closed_form(n):
    w = np.array([0.5, -0.3, 0.8])
    a = np.array([0.2, 9.7, -0.6])
    h = 0.005
    P = _run(w, a, n, h)
    dR, dv, dp = _geometric_closed_form(w, a, n, h)
    assert np.allclose(P.dR, dR, atol=1e-14)
    # the closed form divides by (1 - e^{i th})^2 with th = |w| h ~ 5e-3, which
    # amplifies its own rounding by ~1/th^2 ~ 4e4: relative 1e-10 covers that,
    # while an ordering mistake in the recursion is O(h) ~ 1e-3 relative
    assert np.abs(P.dv - dv).max() <= 1e-10 * np.abs(dv).max()
    assert np.abs(P.dp - dp).max() <= 1e-10 * np.abs(dp).max()


def test_first_order_convergence_to_continuous_closed_form():
    w = np.array([0.9, -0.4, 1.1])
    a = np.array([0.5, 9.5, -1.0])
    T = 0.1
    wn = np.linalg.norm(w)
    Kw = so3.hat(w)
    th = wn * T
    dv_c = (T * np.eye(3) + (1 - np.cos(th)) / wn ** 2 * Kw + (T - np.sin(th) / wn) / wn ** 2 * Kw @ Kw) @ a
    dp_c = (T * T / 2 * np.eye(3) + (T / wn ** 2 - np.sin(th) / wn ** 3) * Kw
            + (T * T / (2 * wn ** 2) - (1 - np.cos(th)) / wn ** 4) * Kw @ Kw) @ a
    errs = []
    for n in (20, 40, 80, 160):
        P = _run(w, a, n, T / n)
        errs.append((np.linalg.norm(P.dv - dv_c), np.linalg.norm(P.dp - dp_c)))
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert np.all(np.abs(ratios - 2.0) < 0.05), ratios


def test_bias_jacobians_finite_difference():
    rng = np.random.default_rng(3)
    n, h = 25, 0.005
    gyro = rng.normal(0, 0.5, (n, 3))
    accel = rng.normal(0, 1.0, (n, 3)) + np.array([0, 0, 9.81])
    bh = np.array([0.01, -0.02, 0.005, 0.1, -0.05, 0.08])
    P = preint.preintegrate(gyro, accel, np.full(n, h), bh, *NO_NOISE)
    eps = 1e-6
    Jrot = np.zeros((3, 3))
    Jvel = np.zeros((3, 6))
    Jpos = np.zeros((3, 6))
    for k in range(6):
        e = np.zeros(6)
        e[k] = eps
        Pp = preint.preintegrate(gyro, accel, np.full(n, h), bh + e, *NO_NOISE)
        Pm = preint.preintegrate(gyro, accel, np.full(n, h), bh - e, *NO_NOISE)
        if k < 3:
            Jrot[:, k] = (so3.Log(P.dR.T @ Pp.dR) - so3.Log(P.dR.T @ Pm.dR)) / (2 * eps)
        else:
            assert np.allclose(Pp.dR, Pm.dR, atol=0)      # rotation ignores b_a
        Jvel[:, k] = (Pp.dv - Pm.dv) / (2 * eps)
        Jpos[:, k] = (Pp.dp - Pm.dp) / (2 * eps)
    assert np.allclose(P.J_rot, Jrot, atol=1e-8)
    assert np.allclose(P.J_vel, Jvel, atol=1e-8)
    assert np.allclose(P.J_pos, Jpos, atol=1e-9)


def _batch_exp(phi):
    th = np.linalg.norm(phi, axis=1)
    K = np.zeros((phi.shape[0], 3, 3))
    K[:, 0, 1], K[:, 0, 2], K[:, 1, 2] = -phi[:, 2], phi[:, 1], -phi[:, 0]
    K[:, 1, 0], K[:, 2, 0], K[:, 2, 1] = phi[:, 2], -phi[:, 1], phi[:, 0]
    s = np.where(th > 1e-12, np.sin(th) / np.maximum(th, 1e-300), 1.0)
    c = np.where(th > 1e-12, (1 - np.cos(th)) / np.maximum(th, 1e-300) ** 2, 0.5)
    return np.eye(3)[None] + s[:, None, None] * K + c[:, None, None] * (K @ K)


def test_covariance_monte_carlo():
    """Sample covariance of the residual at the true state, over independent
    white-noise draws, against the propagated covariance (whitened)."""
    rng = np.random.default_rng(11)
    n, h = 20, 0.005
    sg, sa = 1.7e-3, 2e-2                      # 10x the workload densities, still linear
    gyro = rng.normal(0, 0.6, (n, 3))
    accel = rng.normal(0, 1.5, (n, 3)) + np.array([0.0, 9.81, 0.0])
    P = preint.preintegrate(gyro, accel, np.full(n, h), np.zeros(6), sg, sa, 0.0, 0.0)
    M = 200_000
    dR = np.tile(np.eye(3), (M, 1, 1))
    dv = np.zeros((M, 3))
    dp = np.zeros((M, 3))
    for k in range(n):
        wk = gyro[k] + rng.normal(0, sg / np.sqrt(h), (M, 3))
        ak = accel[k] + rng.normal(0, sa / np.sqrt(h), (M, 3))
        Ra = np.einsum("mab,mb->ma", dR, ak)
        dp = dp + dv * h + 0.5 * Ra * h * h
        dv = dv + Ra * h
        dR = dR @ _batch_exp(wk * h)
    # residual of the noisy measurement at the true (noise-free) motion
    E = np.einsum("mba,bc->mac", dR, P.dR)        # dR_meas^T dR_true
    tr = np.clip((np.trace(E, axis1=1, axis2=2) - 1) / 2, -1, 1)
    th = np.arccos(tr)
    v = np.stack([E[:, 2, 1] - E[:, 1, 2], E[:, 0, 2] - E[:, 2, 0], E[:, 1, 0] - E[:, 0, 1]], 1)
    r_rot = 0.5 * v * np.where(th > 1e-12, th / np.sin(np.maximum(th, 1e-300)), 1.0)[:, None]
    r = np.concatenate([r_rot, P.dp - dp, P.dv - dv], 1)
    S_mc = np.cov(r.T)
    L = np.linalg.cholesky(P.cov)
    Wm = np.linalg.solve(L, np.linalg.solve(L, S_mc).T)
    assert np.abs(Wm - np.eye(9)).max() < 0.03, np.abs(Wm - np.eye(9)).max()


def test_bias_random_walk_variance_and_time():
    P = _run(np.zeros(3), np.zeros(3), 40, 0.005, noise=(0.0, 0.0, 2e-5, 3e-3))
    assert P.dt == pytest.approx(0.2)
    assert np.allclose(P.cov_bias, np.r_[np.full(3, 4e-10 * 0.2), np.full(3, 9e-6 * 0.2)], rtol=1e-14)

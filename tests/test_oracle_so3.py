"""Pins of the oracle's SO(3) helpers against library routines, series and
finite differences (not against themselves)."""
import numpy as np
import pytest
import scipy.linalg
from scipy.spatial.transform import Rotation

from oracle import so3

RNG = np.random.default_rng(7)


def _rand_vecs(n, scale):
    v = RNG.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True) * scale


@pytest.mark.parametrize("scale", [1e-9, 1e-4, 0.3, 2.0, np.pi - 1e-3])
def test_exp_matches_matrix_exponential(scale):
    for phi in _rand_vecs(5, scale):
        assert np.allclose(so3.Exp(phi), scipy.linalg.expm(so3.hat(phi)), atol=1e-14, rtol=0)


@pytest.mark.parametrize("scale", [1e-9, 1e-5, 0.3, 2.0, np.pi - 1e-4, np.pi - 1e-8])
def test_log_inverts_exp(scale):
    for phi in _rand_vecs(5, scale):
        back = so3.Log(so3.Exp(phi))
        assert np.allclose(back, phi, atol=1e-7 if scale > 3.1 else 1e-13, rtol=1e-12)


def test_log_matches_scipy_rotvec():
    for phi in _rand_vecs(8, 1.7):
        R = Rotation.from_rotvec(phi).as_matrix()
        assert np.allclose(so3.Log(R), Rotation.from_matrix(R).as_rotvec(), atol=1e-13)


@pytest.mark.parametrize("scale", [1e-7, 0.2, 1.5])
def test_right_jacobian_finite_difference(scale):
    h = 1e-6
    for phi in _rand_vecs(3, scale):
        J = so3.Jr(phi)
        Jfd = np.zeros((3, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            Rp = so3.Exp(phi).T @ so3.Exp(phi + e)
            Rm = so3.Exp(phi).T @ so3.Exp(phi - e)
            Jfd[:, k] = (so3.Log(Rp) - so3.Log(Rm)) / (2 * h)
        assert np.allclose(J, Jfd, atol=1e-8)


@pytest.mark.parametrize("scale", [1e-7, 0.2, 1.5])
def test_inverse_right_jacobian(scale):
    h = 1e-6
    for phi in _rand_vecs(3, scale):
        Ji = so3.Jr_inv(phi)
        assert np.allclose(Ji @ so3.Jr(phi), np.eye(3), atol=1e-12)
        Jfd = np.zeros((3, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            Jfd[:, k] = (so3.Log(so3.Exp(phi) @ so3.Exp(e)) - so3.Log(so3.Exp(phi) @ so3.Exp(-e))) / (2 * h)
        assert np.allclose(Ji, Jfd, atol=1e-8)


def test_quaternion_conventions():
    for phi in _rand_vecs(6, 1.1):
        rot = Rotation.from_rotvec(phi)
        q = rot.as_quat()                       # scipy stores (x, y, z, w)
        assert np.allclose(so3.quat_to_R(q), rot.as_matrix(), atol=1e-14)
        q2 = so3.R_to_quat(rot.as_matrix())
        assert min(np.abs(q2 - q).max(), np.abs(q2 + q).max()) < 1e-14

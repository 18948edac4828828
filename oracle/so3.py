"""SO(3) helpers used by the inertial residual (Eq. 3 uses Log and Exp) and by
the right-perturbation retraction R <- R Exp(dtheta).

Test infrastructure (see the package header).  Pinned by: Exp/Log round trips,
Exp against a matrix-exponential series, Jr and Jr^-1 against finite
differences of Exp/Log and against each other (Jr Jr^-1 = I).
"""
import numpy as np

I3 = np.eye(3)


def hat(w):
    """Skew matrix [w]x with [w]x v = w x v."""
    w = np.asarray(w, dtype=np.float64)
    return np.array([[0.0, -w[2], w[1]],
                     [w[2], 0.0, -w[0]],
                     [-w[1], w[0], 0.0]])


def vee(S):
    return np.array([S[2, 1], S[0, 2], S[1, 0]])


def Exp(phi):
    """Rotation by angle |phi| about phi/|phi| (Rodrigues' formula)."""
    phi = np.asarray(phi, dtype=np.float64)
    th2 = float(phi @ phi)
    K = hat(phi)
    if th2 < 1e-16:
        return I3 + K + 0.5 * (K @ K)
    th = np.sqrt(th2)
    return I3 + (np.sin(th) / th) * K + ((1.0 - np.cos(th)) / th2) * (K @ K)


def Log(R):
    """Rotation vector of R (inverse of Exp on angles in [0, pi])."""
    R = np.asarray(R, dtype=np.float64)
    v = vee(R - R.T)                       # = 2 sin(th) * axis
    s = 0.5 * np.linalg.norm(v)
    c = 0.5 * (np.trace(R) - 1.0)
    th = np.arctan2(s, c)
    if th < 1e-6:
        # th / sin th = 1 + th^2/6 + ...
        return 0.5 * v * (1.0 + th * th / 6.0)
    if np.pi - th > 1e-6:
        return 0.5 * v * (th / np.sin(th))
    # near pi: axis from the symmetric part u u^T = (R + R^T - 2c I) / (2 (1 - c))
    M = (R + R.T - 2.0 * c * I3) / (2.0 * (1.0 - c))
    k = int(np.argmax(np.diag(M)))
    u = M[:, k] / np.sqrt(max(M[k, k], 1e-300))
    if u @ v < 0:
        u = -u
    return th * u


def Jr(phi):
    """Right Jacobian: Exp(phi + d) ~= Exp(phi) Exp(Jr(phi) d)."""
    phi = np.asarray(phi, dtype=np.float64)
    th2 = float(phi @ phi)
    K = hat(phi)
    if th2 < 1e-12:
        return I3 - 0.5 * K + (K @ K) / 6.0
    th = np.sqrt(th2)
    return I3 - ((1.0 - np.cos(th)) / th2) * K + ((th - np.sin(th)) / (th2 * th)) * (K @ K)


def Jr_inv(phi):
    """Inverse right Jacobian: Log(Exp(phi) Exp(d)) ~= phi + Jr_inv(phi) d."""
    phi = np.asarray(phi, dtype=np.float64)
    th2 = float(phi @ phi)
    K = hat(phi)
    if th2 < 1e-12:
        return I3 + 0.5 * K + (K @ K) / 12.0
    th = np.sqrt(th2)
    coef = 1.0 / th2 - (1.0 + np.cos(th)) / (2.0 * th * np.sin(th))
    return I3 + 0.5 * K + coef * (K @ K)


def quat_to_R(q):
    """Unit quaternion (x, y, z, w) -> rotation matrix."""
    x, y, z, w = (float(a) for a in q)
    n = x * x + y * y + z * z + w * w
    x, y, z, w = (a / np.sqrt(n) for a in (x, y, z, w))
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def R_to_quat(R):
    """Rotation matrix -> unit quaternion (x, y, z, w), w >= 0 (largest-pivot form)."""
    R = np.asarray(R, dtype=np.float64)
    tr = np.trace(R)
    if tr > 0:
        s = 2.0 * np.sqrt(tr + 1.0)
        w = 0.25 * s
        x = (R[2, 1] - R[1, 2]) / s
        y = (R[0, 2] - R[2, 0]) / s
        z = (R[1, 0] - R[0, 1]) / s
    elif R[0, 0] > R[1, 1] and R[0, 0] > R[2, 2]:
        s = 2.0 * np.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2])
        w = (R[2, 1] - R[1, 2]) / s
        x = 0.25 * s
        y = (R[0, 1] + R[1, 0]) / s
        z = (R[0, 2] + R[2, 0]) / s
    elif R[1, 1] > R[2, 2]:
        s = 2.0 * np.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2])
        w = (R[0, 2] - R[2, 0]) / s
        x = (R[0, 1] + R[1, 0]) / s
        y = 0.25 * s
        z = (R[1, 2] + R[2, 1]) / s
    else:
        s = 2.0 * np.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1])
        w = (R[1, 0] - R[0, 1]) / s
        x = (R[0, 2] + R[2, 0]) / s
        y = (R[1, 2] + R[2, 1]) / s
        z = 0.25 * s
    q = np.array([x, y, z, w])
    if q[3] < 0:
        q = -q
    return q / np.linalg.norm(q)

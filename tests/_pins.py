"""Independent mathematics used to pin the oracle (tests only).

Nothing here calls the oracle's formulas: the projected covariance comes from
a finite-difference Jacobian of the pinhole map and scipy's quaternion
rotation, and Gaussian values come from a matrix inverse, so a transposed
operand, a wrong sign or a dropped term in the oracle shows up as a mismatch.
"""
import numpy as np
from scipy.spatial.transform import Rotation


def pinhole(p, fx, fy, cx, cy):
    return np.array([fx * p[0] / p[2] + cx, fy * p[1] / p[2] + cy])


def fd_jacobian(p, fx, fy, cx, cy, h=None):
    """Central finite-difference Jacobian (2x3) of the pinhole map at p."""
    p = np.asarray(p, np.float64)
    h = 1e-6 * max(1.0, abs(p[2])) if h is None else h
    J = np.zeros((2, 3))
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        J[:, i] = (pinhole(p + e, fx, fy, cx, cy) - pinhole(p - e, fx, fy, cx, cy)) / (2 * h)
    return J


def cov3_world(q_wxyz, s):
    """Sigma3 = Rq diag(s^2) Rq^T via scipy (quaternion in scalar-last order there)."""
    w, x, y, z = [float(v) for v in q_wxyz]
    Rq = Rotation.from_quat([x, y, z, w]).as_matrix()
    return Rq @ np.diag(np.asarray(s, np.float64) ** 2) @ Rq.T


def cov2_expected(scene, g, v, lowpass):
    """EWA 2D covariance (incl. low-pass) and mean, by finite differences."""
    R = scene.R[v].astype(np.float64)
    t = scene.t[v].astype(np.float64)
    m = np.array([scene.mx[g], scene.my[g], scene.mz[g]], np.float64)
    p = R @ m + t
    fx, fy, cx, cy = [float(a[v]) for a in (scene.fx, scene.fy, scene.cx, scene.cy)]
    J = fd_jacobian(p, fx, fy, cx, cy)
    S3 = cov3_world([scene.qw[g], scene.qx[g], scene.qy[g], scene.qz[g]],
                    [scene.sx[g], scene.sy[g], scene.sz[g]])
    S2 = J @ (R @ S3 @ R.T) @ J.T + lowpass * np.eye(2)
    return S2, pinhole(p, fx, fy, cx, cy), p


def gaussian_alpha(S2, mean, pix, opacity, k=3.0, alpha_max=1.0):
    """alpha at a pixel centre from an explicit matrix inverse; 0 outside k-sigma."""
    d = np.asarray(pix, np.float64) - mean
    q = float(d @ np.linalg.inv(S2) @ d)
    if q > k * k:
        return 0.0
    return min(alpha_max, opacity * np.exp(-0.5 * q))

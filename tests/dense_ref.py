"""Independent dense reference used to pin the oracle on tiny problems.

Derivatives here come from complex-step differentiation of the retraction and
the camera model evaluated in complex arithmetic (Martins et al., "The
complex-step derivative approximation"): d f(x)/dx = Im f(x + i h) / h with
h = 1e-30, exact to rounding and independent of the hand-derived chain rule
in the oracle.  The damped normal equations are formed densely and solved by
LAPACK (numpy.linalg.solve), with no Schur complement and no CG.
"""
from __future__ import annotations

import numpy as np

H = 1e-30


def _quat_to_rot(q):
    x, y, z, w = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3), dtype=q.dtype)
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - z * w)
    R[..., 0, 2] = 2 * (x * z + y * w)
    R[..., 1, 0] = 2 * (x * y + z * w)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - x * w)
    R[..., 2, 0] = 2 * (x * z - y * w)
    R[..., 2, 1] = 2 * (y * z + x * w)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _hat(v):
    K = np.zeros(v.shape[:-1] + (3, 3), dtype=v.dtype)
    K[..., 0, 1] = -v[..., 2]
    K[..., 0, 2] = v[..., 1]
    K[..., 1, 0] = v[..., 2]
    K[..., 1, 2] = -v[..., 0]
    K[..., 2, 0] = -v[..., 1]
    K[..., 2, 1] = v[..., 0]
    return K


def _exp_se3(delta):
    """(R, t) of Exp(delta), delta = (rho, phi), evaluated by the closed-form
    series in complex arithmetic (works for the tiny imaginary steps used)."""
    rho, phi = delta[..., 0:3], delta[..., 3:6]
    th2 = np.sum(phi * phi, axis=-1)
    # series are exact enough: |th| ~ 1e-30 or exactly 0 in every use here
    a = 1 - th2 / 6 + th2 * th2 / 120
    b = 0.5 - th2 / 24 + th2 * th2 / 720
    c = 1.0 / 6 - th2 / 120 + th2 * th2 / 5040
    K = _hat(phi)
    K2 = K @ K
    I = np.eye(3, dtype=delta.dtype)
    R = I + a[..., None, None] * K + b[..., None, None] * K2
    V = I + b[..., None, None] * K + c[..., None, None] * K2
    t = np.einsum("...ij,...j->...i", V, rho)
    return R, t


def pixels(cams, X, delta_cam=None, d=9):
    """Pixels of X[k] seen by cams[k] after the camera update Exp(delta) T and
    intrinsics + delta[6:9]; complex-capable."""
    R = _quat_to_rot(cams[..., 3:7])
    t = cams[..., 0:3]
    f, k1, k2 = cams[..., 7], cams[..., 8], cams[..., 9]
    Y = np.einsum("...ij,...j->...i", R, X) + t
    if delta_cam is not None:
        Rd, td = _exp_se3(delta_cam[..., 0:6])
        Y = np.einsum("...ij,...j->...i", Rd, Y) + td
        if d == 9:
            f = f + delta_cam[..., 6]
            k1 = k1 + delta_cam[..., 7]
            k2 = k2 + delta_cam[..., 8]
    u = -Y[..., 0] / Y[..., 2]
    v = -Y[..., 1] / Y[..., 2]
    s = u * u + v * v
    D = 1 + k1 * s + k2 * s * s
    return np.stack([f * D * u, f * D * v], axis=-1)


def jacobian_blocks(cams, pts, cidx, pidx, d=9):
    """Complex-step Jc [n,2,d] and Jp [n,2,3] of every observation."""
    cams = cams.astype(np.complex128)
    pts = pts.astype(np.complex128)
    C = cams[cidx]
    X = pts[pidx]
    n = len(cidx)
    Jc = np.zeros((n, 2, d))
    Jp = np.zeros((n, 2, 3))
    for m in range(d):
        delta = np.zeros((n, d), np.complex128)
        delta[:, m] = 1j * H
        Jc[:, :, m] = pixels(C, X, delta, d).imag / H
    for m in range(3):
        Xp = X.copy()
        Xp[:, m] += 1j * H
        Jp[:, :, m] = pixels(C, Xp, None, d).imag / H
    return Jc, Jp


def residual_weights(r, omega, delta):
    s = np.sum(r * r, axis=1)
    if delta <= 0:
        return omega * 1.0, 0.5 * np.sum(omega * s)
    rs = np.sqrt(s)
    drho = np.where(s <= delta * delta, 1.0, delta / np.where(rs > 0, rs, 1))
    rho = np.where(s <= delta * delta, s, 2 * delta * rs - delta * delta)
    return omega * drho, 0.5 * np.sum(omega * rho)


def dense_system(cams, pts, cidx, pidx, obs, omega=None, huber=0.0, d=9, fixed=()):
    """Dense J (2n x (d nc + 3 np)), residual r, weights w, cost F."""
    nc, npt, n = cams.shape[0], pts.shape[0], len(cidx)
    omega = np.ones(n) if omega is None else omega
    r = pixels(cams[cidx], pts[pidx], None, d).real - obs
    w, F = residual_weights(r, omega, huber)
    Jc, Jp = jacobian_blocks(cams, pts, cidx, pidx, d)
    if len(fixed):
        Jc[np.isin(cidx, fixed)] = 0
    J = np.zeros((2 * n, d * nc + 3 * npt))
    for k in range(n):
        J[2 * k:2 * k + 2, d * cidx[k]:d * cidx[k] + d] = Jc[k]
        J[2 * k:2 * k + 2, d * nc + 3 * pidx[k]:d * nc + 3 * pidx[k] + 3] = Jp[k]
    return J, r.reshape(-1), np.repeat(w, 2), F


def dense_step(J, r, w, lam, dmin=1e-6, dmax=1e32):
    """Solve (A + lam diag(clamp(diag A))) delta = -g with A = J^T W J, g = J^T W r."""
    A = J.T @ (w[:, None] * J)
    g = J.T @ (w * r)
    D = np.clip(np.diag(A), dmin, dmax)
    Ad = A + lam * np.diag(D)
    return np.linalg.solve(Ad, -g), A, g

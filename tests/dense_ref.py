"""Dense matrices of every operator, built entry by entry from closed forms.

These are independent of the oracle's loops: the oracle walks rays (Joseph),
interpolates (backprojection, rotation) and convolves (ramp); here every
matrix entry is written as a product of tent functions Lambda(t) = max(0, 1-|t|)
evaluated at the geometric distance between a pixel centre and a ray (or a
sample point), and the ramp kernel is obtained by numerically integrating the
band-limited ramp |w| rather than from its closed form.  Only usable for tiny
images (the matrices are n x d).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate


def tent(t):
    return np.maximum(0.0, 1.0 - np.abs(t))


def geometry(n, n_det):
    cN, cD = (n - 1) / 2.0, (n_det - 1) / 2.0
    jj, ii = np.meshgrid(np.arange(n), np.arange(n))
    X = (jj - cN).reshape(-1)          # pixel p = i*n + j
    Y = (ii - cN).reshape(-1)
    s = np.arange(n_det) - cD
    return X, Y, s


def joseph_matrix(n, n_angles, n_det, idx=None):
    """A[(r,k), p] = Lambda((s_k - s_p)/w)/w,  s_p = X cos + Y sin, w = max(|cos|,|sin|)."""
    idx = np.arange(n_angles) if idx is None else np.asarray(idx)
    X, Y, s = geometry(n, n_det)
    rows = []
    for a in idx:
        th = math.pi * a / n_angles
        c, sn = math.cos(th), math.sin(th)
        w = max(abs(c), abs(sn))
        sp = X * c + Y * sn
        rows.append(tent((s[:, None] - sp[None, :]) / w) / w)
    return np.concatenate(rows, axis=0)


def backprojection_matrix(n, n_angles, n_det, idx=None):
    """B[p, (r,k)] = Lambda(s_p - s_k): linear interpolation of each row at s_p."""
    idx = np.arange(n_angles) if idx is None else np.asarray(idx)
    X, Y, s = geometry(n, n_det)
    cols = []
    for a in idx:
        th = math.pi * a / n_angles
        sp = X * math.cos(th) + Y * math.sin(th)
        cols.append(tent(sp[:, None] - s[None, :]))
    return np.concatenate(cols, axis=1)


def ramp_kernel_by_quadrature(n_max):
    """h[k] = integral over |w| <= 1/2 of |w| exp(2 pi i w k) dw (unit spacing)."""
    h = np.empty(n_max + 1)
    for k in range(n_max + 1):
        val, _ = integrate.quad(lambda w: 2.0 * w * math.cos(2.0 * math.pi * w * k), 0.0, 0.5,
                                limit=400, epsabs=1e-14, epsrel=1e-12)
        h[k] = val
    return h


def ramp_matrix(n_det):
    h = ramp_kernel_by_quadrature(n_det)
    k = np.arange(n_det)
    return h[np.abs(k[:, None] - k[None, :])]


def rotation_matrix(n, c, s):
    """T[p, p'] = Lambda(u_p - j') Lambda(v_p - i'),  (u, v) = R(-phi) p + centre."""
    cN = (n - 1) / 2.0
    X, Y, _ = geometry(n, 1)
    u = c * X + s * Y + cN
    v = -s * X + c * Y + cN
    jj, ii = np.meshgrid(np.arange(n), np.arange(n))
    jp, ip = jj.reshape(-1), ii.reshape(-1)
    return tent(u[:, None] - jp[None, :]) * tent(v[:, None] - ip[None, :])


def ei_loss_grad_dense(x, y, n_angles, idx, cos_sin, lam, mc_idx=None):
    """Loss and gradient of the sketched EI objective by matrix algebra (single image)."""
    n = x.shape[0]
    n_det = y.shape[-1]
    mc_idx = np.arange(n_angles) if mc_idx is None else np.asarray(mc_idx)
    idx = np.asarray(idx)
    m = idx.size
    A_mc = joseph_matrix(n, n_angles, n_det, mc_idx)
    A_s = joseph_matrix(n, n_angles, n_det, idx)
    F_s = (math.pi / m) * backprojection_matrix(n, n_angles, n_det, idx) @ np.kron(np.eye(m), ramp_matrix(n_det))
    xv = x.reshape(-1)
    r_mc = y[mc_idx].reshape(-1) - A_mc @ xv
    loss = float(r_mc @ r_mc)
    grad = -2.0 * A_mc.T @ r_mc
    M = np.eye(n * n) - F_s @ A_s
    C = len(cos_sin)
    for c, s in cos_sin:
        T = rotation_matrix(n, c, s)
        r = M @ (T @ xv)
        loss += lam / C * float(r @ r)
        grad += 2.0 * lam / C * T.T @ (M.T @ r)
    return loss, grad.reshape(n, n)

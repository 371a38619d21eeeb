"""ctypes binding for the FP64 CPU oracle in ``skei_oracle.c``.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product package.  All arrays
are float64 (int32 for angle lists), C-contiguous; every function returns a
new array.  Geometry and operator definitions are documented in
``skei_oracle.c`` (Joseph projector, Ram-Lak FBP, bilinear rotation, and the
sketched test-time EI loss of Eq. (skeilossttt) / Algorithm 2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "skei_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
LIB_PATH = os.environ.get("SKEI_ORACLE_LIB") or os.path.join(_BUILD, "libskei_oracle.so")

__all__ = [
    "build", "radon_fwd", "radon_adj", "ramlak_tap", "ramp", "backproject",
    "backproject_T", "fbp", "fbp_adj", "rotate", "rotate_adj", "ei_loss_grad", "sketch_rows", "sketch_rows_T",
    "num_threads", "LIB_PATH",
]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, IEEE arithmetic)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    os.makedirs(_BUILD, exist_ok=True)
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int32)
_int = ctypes.c_int


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        lib.oracle_radon_fwd.argtypes = [_D, _int, _int, _int, _int, _I, _int, _D]
        lib.oracle_radon_adj.argtypes = [_D, _int, _int, _int, _int, _I, _int, _D]
        lib.oracle_ramlak_tap.argtypes = [_int]
        lib.oracle_ramlak_tap.restype = ctypes.c_double
        lib.oracle_ramp.argtypes = [_D, _int, _int, _D]
        lib.oracle_backproject.argtypes = [_D, _int, _int, _int, _int, _I, _int, _D]
        lib.oracle_backproject_T.argtypes = [_D, _int, _int, _int, _int, _I, _int, _D]
        lib.oracle_fbp.argtypes = [_D, _int, _int, _int, _int, _I, _int, _D]
        lib.oracle_fbp_adj.argtypes = [_D, _int, _int, _int, _int, _I, _int, _D]
        lib.oracle_rotate.argtypes = [_D, _int, _int, _int, _D, _D]
        lib.oracle_rotate_adj.argtypes = [_D, _int, _int, _int, _D, _D]
        lib.oracle_ei_loss_grad.argtypes = [_D, _D, _int, _int, _int, _int, _I, _int, _I, _int,
                                            _int, _D, ctypes.c_double, _D]
        lib.oracle_ei_loss_grad.restype = ctypes.c_double
        _lib = lib
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(_D)


def _idx(idx, n_angles):
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    if idx.ndim != 1 or idx.size == 0:
        raise ValueError("angle list must be a non-empty 1-D array")
    if idx.min() < 0 or idx.max() >= n_angles:
        raise ValueError("angle index out of range")
    return idx


def _img(x):
    x = _d(x)
    squeeze = x.ndim == 2
    if squeeze:
        x = x[None]
    if x.ndim != 3 or x.shape[1] != x.shape[2]:
        raise ValueError("image must be [N,N] or [B,N,N]")
    return x, squeeze


def num_threads() -> int:
    """OpenMP threads the oracle uses (OMP_NUM_THREADS, else all cores)."""
    v = os.environ.get("OMP_NUM_THREADS")
    return int(v) if v else (os.cpu_count() or 1)


def radon_fwd(x, n_angles, n_det, idx=None):
    """y = A_S x (Joseph).  x: [N,N] or [B,N,N] -> [m,N_det] or [B,m,N_det]."""
    x, sq = _img(x)
    idx = _idx(np.arange(n_angles) if idx is None else idx, n_angles)
    b, n = x.shape[0], x.shape[1]
    y = np.empty((b, idx.size, n_det))
    _load().oracle_radon_fwd(_p(x), b, n, n_angles, n_det, idx.ctypes.data_as(_I), idx.size, _p(y))
    return y[0] if sq else y


def _sino(y, m, n_det):
    y = _d(y)
    squeeze = y.ndim == 2
    if squeeze:
        y = y[None]
    if y.ndim != 3 or y.shape[1] != m or y.shape[2] != n_det:
        raise ValueError(f"sinogram must be [{m},{n_det}] or [B,{m},{n_det}], got {y.shape}")
    return y, squeeze


def radon_adj(y, n, n_angles, idx=None):
    """x = A_S^T y (literal transpose of the Joseph walk)."""
    idx = _idx(np.arange(n_angles) if idx is None else idx, n_angles)
    y = _d(y)
    n_det = y.shape[-1]
    y, sq = _sino(y, idx.size, n_det)
    b = y.shape[0]
    x = np.empty((b, n, n))
    _load().oracle_radon_adj(_p(y), b, n, n_angles, n_det, idx.ctypes.data_as(_I), idx.size, _p(x))
    return x[0] if sq else x


def ramlak_tap(k: int) -> float:
    return float(_load().oracle_ramlak_tap(int(k)))


def ramp(p):
    """Ram-Lak filtering of every detector row (last axis), linear convolution."""
    p = _d(p)
    n_det = p.shape[-1]
    q = np.empty_like(p)
    _load().oracle_ramp(_p(p), p.size // n_det, n_det, _p(q))
    return q


def backproject(q, n, n_angles, idx=None):
    """Pixel-driven linear-interpolation backprojection B_S (no pi/m scale)."""
    idx = _idx(np.arange(n_angles) if idx is None else idx, n_angles)
    q = _d(q)
    n_det = q.shape[-1]
    q, sq = _sino(q, idx.size, n_det)
    b = q.shape[0]
    x = np.empty((b, n, n))
    _load().oracle_backproject(_p(q), b, n, n_angles, n_det, idx.ctypes.data_as(_I), idx.size, _p(x))
    return x[0] if sq else x


def backproject_T(x, n_angles, n_det, idx=None):
    """B_S^T (literal transpose of the backprojection)."""
    x, sq = _img(x)
    idx = _idx(np.arange(n_angles) if idx is None else idx, n_angles)
    b, n = x.shape[0], x.shape[1]
    q = np.empty((b, idx.size, n_det))
    _load().oracle_backproject_T(_p(x), b, n, n_angles, n_det, idx.ctypes.data_as(_I), idx.size, _p(q))
    return q[0] if sq else q


def fbp(y, n, n_angles, idx=None):
    """fbp_S y = (pi/m) B_S H y."""
    idx = _idx(np.arange(n_angles) if idx is None else idx, n_angles)
    y = _d(y)
    n_det = y.shape[-1]
    y, sq = _sino(y, idx.size, n_det)
    b = y.shape[0]
    x = np.empty((b, n, n))
    _load().oracle_fbp(_p(y), b, n, n_angles, n_det, idx.ctypes.data_as(_I), idx.size, _p(x))
    return x[0] if sq else x


def fbp_adj(x, n_angles, n_det, idx=None):
    """fbp_S^T x = (pi/m) H B_S^T x."""
    x, sq = _img(x)
    idx = _idx(np.arange(n_angles) if idx is None else idx, n_angles)
    b, n = x.shape[0], x.shape[1]
    y = np.empty((b, idx.size, n_det))
    _load().oracle_fbp_adj(_p(x), b, n, n_angles, n_det, idx.ctypes.data_as(_I), idx.size, _p(y))
    return y[0] if sq else y


def _cs(cos_sin):
    cs = _d(cos_sin).reshape(-1, 2)
    return cs


def rotate(x, cos_sin):
    """out[b][c] = T_{phi_c} x[b]; x [N,N] or [B,N,N]; cos_sin [C,2] -> [B,C,N,N] ([C,N,N] if 2-D)."""
    x, sq = _img(x)
    cs = _cs(cos_sin)
    b, n, c = x.shape[0], x.shape[1], cs.shape[0]
    out = np.empty((b, c, n, n))
    _load().oracle_rotate(_p(x), b, c, n, _p(cs), _p(out))
    return out[0] if sq else out


def rotate_adj(h, cos_sin):
    """g[b] = sum_c T_{phi_c}^T h[b][c]; h [C,N,N] or [B,C,N,N]."""
    h = _d(h)
    cs = _cs(cos_sin)
    sq = h.ndim == 3
    if sq:
        h = h[None]
    b, c, n = h.shape[0], h.shape[1], h.shape[2]
    if c != cs.shape[0]:
        raise ValueError("copies mismatch")
    g = np.empty((b, n, n))
    _load().oracle_rotate_adj(_p(h), b, c, n, _p(cs), _p(g))
    return g[0] if sq else g


def ei_loss_grad(x, y, n_angles, idx, cos_sin, lam=1.0, mc_idx=None, want_grad=True):
    """Sketched test-time EI loss (network = identity) and its image gradient.

    x: [N,N] or [B,N,N]; y: full measured sinogram [N_theta,N_det] or
    [B,N_theta,N_det]; idx: sketch angle list; mc_idx: angles of the MC term
    (default: all angles); cos_sin: [C,2].  Returns (loss, grad or None).
    """
    x, sq = _img(x)
    y = _d(y)
    if y.ndim == 2:
        y = y[None]
    b, n = x.shape[0], x.shape[1]
    n_det = y.shape[-1]
    if y.shape != (b, n_angles, n_det):
        raise ValueError("y must be the full sinogram [B,N_theta,N_det]")
    idx = _idx(idx, n_angles)
    mc = _idx(np.arange(n_angles) if mc_idx is None else mc_idx, n_angles)
    cs = _cs(cos_sin)
    g = np.empty((b, n, n)) if want_grad else None
    loss = _load().oracle_ei_loss_grad(_p(x), _p(y), b, n, n_angles, n_det, mc.ctypes.data_as(_I), mc.size,
                                       idx.ctypes.data_as(_I), idx.size, cs.shape[0], _p(cs), float(lam),
                                       _p(g) if want_grad else None)
    if g is not None and sq:
        g = g[0]
    return loss, g


def sketch_rows(G, y):
    """Dense measurement-space sketch S = G (x) I applied to sinograms: the
    Gaussian / Rademacher sketches of Sec. 2.3 acting on whole projections.
    out[b][i][c] = sum_a G[i][a] y[b][a][c]; G [m, n_rows], y [n_rows, L] or
    [B, n_rows, L].  Float64 matrix products."""
    G = _d(G)
    y = _d(y)
    sq = y.ndim == 2
    y3 = y[None] if sq else y
    if y3.shape[1] != G.shape[1]:
        raise ValueError("rows of y must match the columns of G")
    out = np.stack([G @ y3[b] for b in range(y3.shape[0])])
    return out[0] if sq else out


def sketch_rows_T(G, r):
    """The transpose S^T: out[b][a][c] = sum_i G[i][a] r[b][i][c]."""
    G = _d(G)
    r = _d(r)
    sq = r.ndim == 2
    r3 = r[None] if sq else r
    if r3.shape[1] != G.shape[0]:
        raise ValueError("rows of r must match the rows of G")
    out = np.stack([G.T @ r3[b] for b in range(r3.shape[0])])
    return out[0] if sq else out

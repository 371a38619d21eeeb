"""Torch-facing operators over the C ABI, with hand-written autograd transposes.

PyTorch supplies device memory and the current HIP stream; every operator is
one or two C-ABI calls into the HIP kernels.  Tensors must be contiguous
float32 on the geometry's device (angle lists: int32).  There is no CPU path:
calling these with CPU tensors raises.

Operators (Sec. 2.1 problem set-up, Sec. 3.1 sketched EI, Sec. 4.1 CT set-up):
  radon_fwd   y = A_S x          (Joseph)         backward: A_S^T
  radon_adj   x = A_S^T y                          backward: A_S
  fbp         x = (pi/m) B_S H y  (FBP / A^dagger) backward: (pi/m) H B_S^T
  fbp_adj     its transpose                        backward: fbp
  rotate      out[b][c] = T_{phi_c} x[b]           backward: sum_c T_c^T
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import capi


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _check(t: torch.Tensor, dtype, device, name: str):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on a HIP device (no CPU path)")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Geometry:
    """N x N image, N_theta angles theta_a = a*pi/N_theta, N_det unit detectors.

    Owns the library's device angle table (created on the current device).
    """

    def __init__(self, n: int, n_angles: int, n_det: int, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.n, self.n_angles, self.n_det = int(n), int(n_angles), int(n_det)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            capi.call("skei_geom_create", self.n, self.n_angles, self.n_det, ctypes.byref(h))
        self._h = h
        self._full = None

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            capi.call("skei_geom_destroy", self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sketch(self, indices) -> "Sketch":
        return Sketch(self, indices)

    def full(self) -> "Sketch":
        if self._full is None:
            self._full = Sketch(self, np.arange(self.n_angles, dtype=np.int32))
        return self._full

    def __repr__(self):
        return f"Geometry(n={self.n}, n_angles={self.n_angles}, n_det={self.n_det}, device={self.device})"


class Sketch:
    """An angle-subsampling sketch S (Sec. 3.1): a validated list of angle
    indices into the full scan, kept both on the host and on the device."""

    def __init__(self, geom: Geometry, indices):
        idx = np.ascontiguousarray(np.asarray(indices).reshape(-1), dtype=np.int64)
        if idx.size == 0:
            raise ValueError("a sketch needs at least one angle")
        if idx.min() < 0 or idx.max() >= geom.n_angles:
            raise ValueError(f"angle index out of range [0, {geom.n_angles})")
        self.geom = geom
        self.host = idx.astype(np.int32)
        self.dev = torch.from_numpy(self.host).to(geom.device)
        self.m = int(idx.size)

    def __len__(self):
        return self.m


def _as_sketch(geom: Geometry, idx) -> Sketch:
    if isinstance(idx, Sketch):
        if idx.geom is not geom and idx.geom.n_angles != geom.n_angles:
            raise ValueError("sketch belongs to a different geometry")
        return idx
    if idx is None:
        return geom.full()
    return Sketch(geom, idx.cpu().numpy() if isinstance(idx, torch.Tensor) else idx)


def _img(geom: Geometry, x: torch.Tensor, name="x"):
    _check(x, torch.float32, geom.device, name)
    if x.dim() == 2:
        x = x.unsqueeze(0)
    if x.dim() != 3 or x.shape[1] != geom.n or x.shape[2] != geom.n:
        raise ValueError(f"{name} must be [B,{geom.n},{geom.n}], got {tuple(x.shape)}")
    return x


def _sino(geom: Geometry, y: torch.Tensor, m: int, name="y"):
    _check(y, torch.float32, geom.device, name)
    if y.dim() == 2:
        y = y.unsqueeze(0)
    if y.dim() != 3 or y.shape[1] != m or y.shape[2] != geom.n_det:
        raise ValueError(f"{name} must be [B,{m},{geom.n_det}], got {tuple(y.shape)}")
    return y


# ----------------------------------------------------------------- raw calls
def radon_fwd_(geom: Geometry, x: torch.Tensor, sk: Sketch, out: torch.Tensor | None = None) -> torch.Tensor:
    x3 = _img(geom, x)
    b = x3.shape[0]
    y = torch.empty((b, sk.m, geom.n_det), device=geom.device, dtype=torch.float32) if out is None else out
    capi.call("skei_radon_fwd", geom.handle, _ptr(x3), b, _ptr(sk.dev), sk.m, _ptr(y), _stream())
    return y if x.dim() == 3 else y[0]


def radon_resid_(geom: Geometry, x: torch.Tensor, y_full: torch.Tensor, sk: Sketch,
                 out: torch.Tensor | None = None) -> torch.Tensor:
    """S y - A_S x with the projection and the difference in double (skei_radon_resid)."""
    x3 = _img(geom, x)
    b = x3.shape[0]
    y3 = _sino(geom, y_full, geom.n_angles, "y_full")
    if y3.shape[0] != b:
        raise ValueError("y_full and x must have the same batch")
    r = torch.empty((b, sk.m, geom.n_det), device=geom.device, dtype=torch.float32) if out is None else out
    capi.call("skei_radon_resid", geom.handle, _ptr(x3), _ptr(y3), b, _ptr(sk.dev), sk.m, _ptr(r), _stream())
    return r if x.dim() == 3 else r[0]


class DenseSketch:
    """A dense measurement-space sketch S = G (x) I_{N_det} (Sec. 2.3): G in
    R^{m x N_theta} mixes whole projections (Gaussian or Rademacher entries,
    see synth.dense_sketch_matrix).  Kept on the device as float32."""

    def __init__(self, geom: Geometry, G):
        g = np.ascontiguousarray(np.asarray(G, dtype=np.float32))
        if g.ndim != 2 or g.shape[1] != geom.n_angles:
            raise ValueError(f"G must be [m, {geom.n_angles}]")
        self.geom = geom
        self.m = g.shape[0]
        self.dev = torch.from_numpy(g).to(geom.device)


def sketch_rows_(ds: DenseSketch, y: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """S y: [B, N_theta, L] -> [B, m, L] on the matrix cores (skei_sketch_rows)."""
    _check(y, torch.float32, ds.geom.device, "y")
    y3 = y.unsqueeze(0) if y.dim() == 2 else y
    if y3.dim() != 3 or y3.shape[1] != ds.dev.shape[1]:
        raise ValueError(f"y must be [B, {ds.dev.shape[1]}, L]")
    b, k, L = y3.shape
    o = torch.empty((b, ds.m, L), device=y.device, dtype=torch.float32) if out is None else out
    capi.call("skei_sketch_rows", _ptr(ds.dev), ds.m, k, _ptr(y3), b, L, _ptr(o), _stream())
    return o if y.dim() == 3 else o[0]


def sketch_rows_T_(ds: DenseSketch, r: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """S^T r: [B, m, L] -> [B, N_theta, L] (skei_sketch_rows_T)."""
    _check(r, torch.float32, ds.geom.device, "r")
    r3 = r.unsqueeze(0) if r.dim() == 2 else r
    if r3.dim() != 3 or r3.shape[1] != ds.m:
        raise ValueError(f"r must be [B, {ds.m}, L]")
    b, _, L = r3.shape
    k = ds.dev.shape[1]
    o = torch.empty((b, k, L), device=r.device, dtype=torch.float32) if out is None else out
    capi.call("skei_sketch_rows_T", _ptr(ds.dev), ds.m, k, _ptr(r3), b, L, _ptr(o), _stream())
    return o if r.dim() == 3 else o[0]


def radon_adj_(geom: Geometry, y: torch.Tensor, sk: Sketch, out: torch.Tensor | None = None) -> torch.Tensor:
    y3 = _sino(geom, y, sk.m)
    b = y3.shape[0]
    x = torch.empty((b, geom.n, geom.n), device=geom.device, dtype=torch.float32) if out is None else out
    capi.call("skei_radon_adj", geom.handle, _ptr(y3), b, _ptr(sk.dev), sk.m, _ptr(x), _stream())
    return x if y.dim() == 3 else x[0]


def ramp_(geom: Geometry, p: torch.Tensor) -> torch.Tensor:
    _check(p, torch.float32, geom.device, "p")
    if p.shape[-1] != geom.n_det:
        raise ValueError("last axis must be the detector axis")
    q = torch.empty_like(p)
    capi.call("skei_ramp", geom.handle, _ptr(p), p.numel() // geom.n_det, _ptr(q), _stream())
    return q


def backproject_(geom: Geometry, q: torch.Tensor, sk: Sketch) -> torch.Tensor:
    q3 = _sino(geom, q, sk.m, "q")
    b = q3.shape[0]
    x = torch.empty((b, geom.n, geom.n), device=geom.device, dtype=torch.float32)
    capi.call("skei_backproject", geom.handle, _ptr(q3), b, _ptr(sk.dev), sk.m, _ptr(x), _stream())
    return x if q.dim() == 3 else x[0]


def backproject_T_(geom: Geometry, x: torch.Tensor, sk: Sketch) -> torch.Tensor:
    x3 = _img(geom, x)
    b = x3.shape[0]
    q = torch.empty((b, sk.m, geom.n_det), device=geom.device, dtype=torch.float32)
    capi.call("skei_backproject_T", geom.handle, _ptr(x3), b, _ptr(sk.dev), sk.m, _ptr(q), _stream())
    return q if x.dim() == 3 else q[0]


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _fbp_work(geom: Geometry, b: int, m: int, work: torch.Tensor | None):
    nb = int(capi.query("skei_fbp_workspace_bytes", geom.handle, b, m))
    if work is None:
        return _workspace(nb, geom.device), nb
    if work.device != geom.device or work.numel() * work.element_size() < nb:
        raise ValueError(f"fbp workspace must hold {nb} bytes on {geom.device}")
    return work, work.numel() * work.element_size()


def fbp_(geom: Geometry, y: torch.Tensor, sk: Sketch, out: torch.Tensor | None = None,
         work: torch.Tensor | None = None) -> torch.Tensor:
    y3 = _sino(geom, y, sk.m)
    b = y3.shape[0]
    x = torch.empty((b, geom.n, geom.n), device=geom.device, dtype=torch.float32) if out is None else out
    w, nb = _fbp_work(geom, b, sk.m, work)
    capi.call("skei_fbp", geom.handle, _ptr(y3), b, _ptr(sk.dev), sk.m, _ptr(x), _ptr(w), nb, _stream())
    return x if y.dim() == 3 else x[0]


def fbp_adj_(geom: Geometry, x: torch.Tensor, sk: Sketch, out: torch.Tensor | None = None,
             work: torch.Tensor | None = None) -> torch.Tensor:
    x3 = _img(geom, x)
    b = x3.shape[0]
    y = torch.empty((b, sk.m, geom.n_det), device=geom.device, dtype=torch.float32) if out is None else out
    w, nb = _fbp_work(geom, b, sk.m, work)
    capi.call("skei_fbp_adj", geom.handle, _ptr(x3), b, _ptr(sk.dev), sk.m, _ptr(y), _ptr(w), nb, _stream())
    return y if x.dim() == 3 else y[0]


def cos_sin_tensor(phi_or_cs, device) -> torch.Tensor:
    """[C,2] float32 (cos, sin) on `device` from angles (rad) or an existing [C,2] table."""
    a = np.asarray(phi_or_cs, dtype=np.float64)
    if a.ndim == 2 and a.shape[1] == 2:
        cs = a
    else:
        a = a.reshape(-1)
        cs = np.stack([np.cos(a), np.sin(a)], axis=1)
    return torch.from_numpy(cs.astype(np.float32)).to(device)


def rotate_(x: torch.Tensor, cs: torch.Tensor) -> torch.Tensor:
    _check(x, torch.float32, None, "x")
    _check(cs, torch.float32, x.device, "cos_sin")
    x3 = x.unsqueeze(0) if x.dim() == 2 else x
    b, n = x3.shape[0], x3.shape[-1]
    c = cs.shape[0]
    out = torch.empty((b, c, n, n), device=x.device, dtype=torch.float32)
    capi.call("skei_rotate", _ptr(x3), b, c, n, _ptr(cs), _ptr(out), _stream())
    return out if x.dim() == 3 else out[0]


def rotate_adj_(h: torch.Tensor, cs: torch.Tensor) -> torch.Tensor:
    _check(h, torch.float32, None, "h")
    _check(cs, torch.float32, h.device, "cos_sin")
    h4 = h.unsqueeze(0) if h.dim() == 3 else h
    b, c, n = h4.shape[0], h4.shape[1], h4.shape[-1]
    if c != cs.shape[0]:
        raise ValueError("copies mismatch")
    g = torch.empty((b, n, n), device=h.device, dtype=torch.float32)
    capi.call("skei_rotate_adj", _ptr(h4), b, c, n, _ptr(cs), _ptr(g), _stream())
    return g if h.dim() == 4 else g[0]


def sumsq_diff_(a: torch.Tensor, b: torch.Tensor | None = None) -> torch.Tensor:
    _check(a, torch.float32, None, "a")
    if b is not None:
        _check(b, torch.float32, a.device, "b")
        if b.numel() != a.numel():
            raise ValueError("size mismatch")
    out = torch.empty((), dtype=torch.float64, device=a.device)
    nb = capi.query("skei_sumsq_workspace_bytes", a.numel())
    w = _workspace(nb, a.device)
    capi.call("skei_sumsq_diff", _ptr(a), _ptr(b) if b is not None else None, a.numel(), _ptr(out), _ptr(w), nb,
              _stream())
    return out


# ----------------------------------------------------------------- autograd
class RadonFwd(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, geom, sk):
        ctx.geom, ctx.sk = geom, sk
        return radon_fwd_(geom, x.contiguous(), sk)

    @staticmethod
    def backward(ctx, gy):
        return radon_adj_(ctx.geom, gy.contiguous(), ctx.sk), None, None


class RadonResid(torch.autograd.Function):
    """r = S y - A_S x; y is data (no gradient), so the backward is -A_S^T."""
    @staticmethod
    def forward(ctx, x, y_full, geom, sk):
        ctx.geom, ctx.sk = geom, sk
        return radon_resid_(geom, x.contiguous(), y_full.contiguous(), sk)

    @staticmethod
    def backward(ctx, gr):
        return -radon_adj_(ctx.geom, gr.contiguous(), ctx.sk), None, None, None


class SketchRows(torch.autograd.Function):
    """y -> S y for a dense sketch; the backward is S^T."""
    @staticmethod
    def forward(ctx, y, ds):
        ctx.ds = ds
        return sketch_rows_(ds, y.contiguous())

    @staticmethod
    def backward(ctx, g):
        return sketch_rows_T_(ctx.ds, g.contiguous()), None


class RadonAdj(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, geom, sk):
        ctx.geom, ctx.sk = geom, sk
        return radon_adj_(geom, y.contiguous(), sk)

    @staticmethod
    def backward(ctx, gx):
        return radon_fwd_(ctx.geom, gx.contiguous(), ctx.sk), None, None


class FBP(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, geom, sk):
        ctx.geom, ctx.sk = geom, sk
        return fbp_(geom, y.contiguous(), sk)

    @staticmethod
    def backward(ctx, gx):
        return fbp_adj_(ctx.geom, gx.contiguous(), ctx.sk), None, None


class FBPAdj(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, geom, sk):
        ctx.geom, ctx.sk = geom, sk
        return fbp_adj_(geom, x.contiguous(), sk)

    @staticmethod
    def backward(ctx, gy):
        return fbp_(ctx.geom, gy.contiguous(), ctx.sk), None, None


class Rotate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, cs):
        ctx.save_for_backward(cs)
        return rotate_(x.contiguous(), cs)

    @staticmethod
    def backward(ctx, g):
        (cs,) = ctx.saved_tensors
        return rotate_adj_(g.contiguous(), cs), None


def radon_fwd(x, geom: Geometry, idx=None):
    """A_S x (differentiable)."""
    return RadonFwd.apply(x, geom, _as_sketch(geom, idx))


def radon_resid(x, y_full, geom: Geometry, idx=None):
    """S y - A_S x (differentiable in x; y_full is the whole sinogram)."""
    return RadonResid.apply(x, y_full, geom, _as_sketch(geom, idx))


def sketch_rows(y, ds: DenseSketch):
    """S y for a dense sketch (differentiable)."""
    return SketchRows.apply(y, ds)


def radon_resid_dense(x, y_full, geom: Geometry, ds: DenseSketch):
    """S (y - A x) for a dense sketch (differentiable in x): the residual is
    formed in double by skei_radon_resid before the mixing, so the sketch of
    a residual ~100x smaller than y keeps its digits."""
    return SketchRows.apply(RadonResid.apply(x, y_full, geom, geom.full()), ds)


def radon_fwd_dense(x, geom: Geometry, ds: DenseSketch):
    """The densely sketched operator A_S x = S (A x) (differentiable): every
    angle is projected, then the projections are mixed by G."""
    return SketchRows.apply(RadonFwd.apply(x, geom, geom.full()), ds)


def radon_adj(y, geom: Geometry, idx=None):
    """A_S^T y (differentiable)."""
    return RadonAdj.apply(y, geom, _as_sketch(geom, idx))


def fbp(y, geom: Geometry, idx=None):
    """fbp_S y = (pi/m) B_S H y (differentiable)."""
    return FBP.apply(y, geom, _as_sketch(geom, idx))


def fbp_adj(x, geom: Geometry, idx=None):
    return FBPAdj.apply(x, geom, _as_sketch(geom, idx))


def rotate(x, cs):
    """T_phi x for every copy: [B,N,N] -> [B,C,N,N] (differentiable)."""
    return Rotate.apply(x, cs)


def pi_over_m(m: int) -> float:
    return math.pi / m

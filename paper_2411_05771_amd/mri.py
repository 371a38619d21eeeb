"""Multicoil MRI with coil sketches (Sec. 3.4, Eq. (e:mri), Algorithm 3) on
the HIP library (include/skei_mri.h): argument marshalling only -- the DFTs,
coil products, coil mixing, covariance and weights run in the library's
kernels, the PCA eigensolver in its host code.

- ``MRIOperator(maps, mask)``: A = M F C with complex64 coil maps [Nc,N,N]
  and a real mask [N,N] on the device; ``fwd_`` / ``adj_`` / ``pinv_`` and
  the differentiable ``mri_fwd`` / ``mri_pinv`` (autograd Functions whose
  backwards are the library's transposes).
- ``classical_sketch``: the coil-subsampling sketch (Mc of Nc coils).
- ``coil_sketch``: Algorithm 3's initialisation -- coil covariance of the
  measured k-space, PCA to L virtual coils (the maps combined the same way,
  the maps being known), then S_c = [[I_R, 0], [0, S_low]] with Rademacher
  S_low on the low-energy coils; returns the sketched operator and data.
- ``mri_ei_loss``: the sketched EI loss of Algorithm 3 with the network taken
  as the identity (x is adapted directly), built from these operators and
  the library's rotations; its gradient comes from autograd.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np
import torch

from . import capi, ops, synth

__all__ = [
    "MRIOperator", "mri_fwd", "mri_pinv", "coil_mix_", "classical_sketch", "coil_sketch", "coil_covariance_",
    "coil_pca", "rotate_complex", "mri_ei_loss", "mri_skei_ttt_loss", "MRIProblem", "make_problem",
    "time_per_iteration", "MRIGraphStep",
]


def _dev_c64(a, device) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.complex64).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).to(device)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


class MRIOperator:
    """A = M F C (Eq. e:mri) for coil maps [Nc,N,N] (complex) and a real mask
    [N,N], on a HIP device."""

    def __init__(self, maps, mask, device=None):
        device = device or (maps.device if isinstance(maps, torch.Tensor) else torch.device("cuda", 0))
        if torch.device(device).type != "cuda":
            raise ValueError("MRIOperator needs a HIP device (no CPU path)")
        self.maps = _dev_c64(maps, device)
        if self.maps.dim() != 3 or self.maps.shape[1] != self.maps.shape[2]:
            raise ValueError("maps must be [Nc, N, N]")
        self.nc, self.n = int(self.maps.shape[0]), int(self.maps.shape[1])
        m = mask if isinstance(mask, torch.Tensor) else torch.from_numpy(np.asarray(mask, dtype=np.float32))
        self.mask = m.to(device=device, dtype=torch.float32).contiguous()
        if tuple(self.mask.shape) != (self.n, self.n):
            raise ValueError("mask must be [N, N]")
        self.device = self.maps.device
        self._w = None

    @property
    def weights(self) -> torch.Tensor:
        """1 / sum_c |C_c|^2 pixelwise (the pseudo-inverse's weights)."""
        if self._w is None:
            self._w = torch.empty((self.n, self.n), device=self.device, dtype=torch.float32)
            capi.call("skei_coil_weights", _ptr(self.maps), self.nc, self.n, _ptr(self._w), ops._stream())
        return self._w

    def _img(self, x: torch.Tensor) -> torch.Tensor:
        if x.dtype != torch.complex64 or x.device != self.device:
            raise TypeError("images must be complex64 on the operator's device")
        if tuple(x.shape[-2:]) != (self.n, self.n):
            raise ValueError("image size mismatch")
        return x.contiguous().reshape(-1, self.n, self.n)

    def fwd_(self, x: torch.Tensor, weighted: bool = False) -> torch.Tensor:
        """k = M F(C x) (with weighted=True: M F(C W x)); [B,N,N] -> [B,Nc,N,N]."""
        x3 = self._img(x)
        b = x3.shape[0]
        k = torch.empty((b, self.nc, self.n, self.n), device=self.device, dtype=torch.complex64)
        w = _ptr(self.weights) if weighted else None
        capi.call("skei_mri_fwd", _ptr(self.maps), self.nc, self.n, _ptr(x3), b, _ptr(self.mask), w, _ptr(k),
                  ops._stream())
        return k if x.dim() == 3 else k[0]

    def adj_(self, k: torch.Tensor, weighted: bool = False) -> torch.Tensor:
        """x = A^H k (with weighted=True: D^-1 A^H k); [B,Nc,N,N] -> [B,N,N]."""
        if k.dtype != torch.complex64 or k.device != self.device:
            raise TypeError("k-space must be complex64 on the operator's device")
        k4 = k.contiguous().reshape(-1, self.nc, self.n, self.n)
        b = k4.shape[0]
        x = torch.empty((b, self.n, self.n), device=self.device, dtype=torch.complex64)
        work = torch.empty((b, self.nc, self.n, self.n), device=self.device, dtype=torch.complex64)
        w = _ptr(self.weights) if weighted else None
        capi.call("skei_mri_adj", _ptr(self.maps), self.nc, self.n, _ptr(k4), b, _ptr(self.mask), w, _ptr(x),
                  _ptr(work), ops._stream())
        return x if k.dim() == 4 else x[0]

    def pinv_(self, k: torch.Tensor) -> torch.Tensor:
        """A^dagger k = D^-1 A^H k."""
        return self.adj_(k, weighted=True)


class _Fwd(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, op, weighted):
        ctx.op, ctx.weighted = op, weighted
        return op.fwd_(x, weighted)

    @staticmethod
    def backward(ctx, g):
        # (A W)^H = W A^H
        return ctx.op.adj_(g.contiguous(), ctx.weighted), None, None


class _Adj(torch.autograd.Function):
    @staticmethod
    def forward(ctx, k, op, weighted):
        ctx.op, ctx.weighted = op, weighted
        return op.adj_(k, weighted)

    @staticmethod
    def backward(ctx, g):
        # (W A^H)^H = A W
        return ctx.op.fwd_(g.contiguous(), ctx.weighted), None, None


def mri_fwd(x, op: MRIOperator):
    """A x, differentiable."""
    return _Fwd.apply(x, op, False)


def mri_pinv(k, op: MRIOperator):
    """A^dagger k = D^-1 A^H k, differentiable."""
    return _Adj.apply(k, op, True)


def coil_mix_(G, z: torch.Tensor) -> torch.Tensor:
    """out[b, r] = sum_l G[r, l] z[b, l]: S = G (x) I_d on a coil stack
    [B,L,N,N] (or [L,N,N]) -> [B,M,N,N]."""
    Gd = _dev_c64(G, z.device)
    if Gd.dim() != 2:
        raise ValueError("G must be [M, L]")
    m_out, l_in = int(Gd.shape[0]), int(Gd.shape[1])
    z4 = z.contiguous().reshape(-1, *z.shape[-3:]) if z.dim() == 4 else z.contiguous().unsqueeze(0)
    if z4.dtype != torch.complex64 or z4.shape[1] != l_in:
        raise ValueError("z must be complex64 [B, L, N, N] with L = G.shape[1]")
    b, d = int(z4.shape[0]), int(z4.shape[2] * z4.shape[3])
    out = torch.empty((b, m_out, z4.shape[2], z4.shape[3]), device=z.device, dtype=torch.complex64)
    capi.call("skei_coil_mix", _ptr(Gd), m_out, l_in, _ptr(z4), b, d, _ptr(out), ops._stream())
    return out if z.dim() == 4 else out[0]


def coil_covariance_(k: torch.Tensor) -> np.ndarray:
    """V [Nc,Nc] complex128 (host) of one measurement k [Nc,N,N]."""
    nc = int(k.shape[0])
    V = torch.empty((nc, nc, 2), device=k.device, dtype=torch.float64)
    capi.call("skei_coil_covariance", _ptr(k.contiguous()), nc, int(k.shape[1] * k.shape[2]), _ptr(V), ops._stream())
    Vh = V.cpu().numpy()
    return Vh[..., 0] + 1j * Vh[..., 1]


def coil_pca(V: np.ndarray, L: int):
    """(Q_L [Nc,L], eigenvalues [L]) by the library's host eigensolver."""
    nc = V.shape[0]
    Vi = np.ascontiguousarray(np.stack([V.real, V.imag], axis=-1), dtype=np.float64)
    Q = np.zeros((nc, L, 2))
    w = np.zeros(L)
    capi.call("skei_coil_pca", Vi.ctypes.data_as(ctypes.c_void_p), nc, L, Q.ctypes.data_as(ctypes.c_void_p),
              w.ctypes.data_as(ctypes.c_void_p))
    return Q[..., 0] + 1j * Q[..., 1], w


def classical_sketch(op: MRIOperator, y: torch.Tensor, coils):
    """The classical coil-subsampling sketch: the operator on coils `coils`
    and the matching k-space [B,Mc,N,N]."""
    coils = np.asarray(coils, dtype=np.int64)
    G = np.zeros((coils.size, op.nc))
    G[np.arange(coils.size), coils] = 1.0
    maps_s = coil_mix_(G, op.maps)
    return MRIOperator(maps_s, op.mask), coil_mix_(G, y)


def coil_sketch(op: MRIOperator, y: torch.Tensor, L: int, R: int, mc: int, seed: int = synth.SEED_MRI):
    """Algorithm 3's coil sketch from one measurement y [1,Nc,N,N]:
    PCA to L virtual coils, R of them kept, the other L - R mixed into
    mc - R by Rademacher signs.  Returns (sketched operator, sketched data,
    info with Q, eigenvalues and S_c)."""
    if not (1 <= R <= L <= op.nc and R <= mc and (mc > R) == (L > R)):
        raise ValueError("need 1 <= R <= L <= Nc, R <= Mc, and Mc > R exactly when L > R")
    V = coil_covariance_(y[0] if y.dim() == 4 else y)
    Q, w = coil_pca(V, L)
    S_c = np.zeros((mc, L))
    S_c[:R, :R] = np.eye(R)
    if L > R:
        S_c[R:, R:] = synth.rademacher_signs(mc - R, L - R, seed)
    Gq = Q.T                                          # virtual coil l = sum_i Q[i, l] coil i
    virt_maps = coil_mix_(Gq, op.maps)
    virt_y = coil_mix_(Gq, y)
    maps_s = coil_mix_(S_c, virt_maps)
    return MRIOperator(maps_s, op.mask), coil_mix_(S_c, virt_y), {"Q": Q, "eigenvalues": w, "S_c": S_c}


def rotate_complex(x: torch.Tensor, cs: torch.Tensor) -> torch.Tensor:
    """T_c x for complex x [B,N,N]: the library's bilinear rotation of the
    real and imaginary parts; -> [B,C,N,N] complex (differentiable)."""
    return torch.complex(ops.rotate(x.real.contiguous(), cs), ops.rotate(x.imag.contiguous(), cs))


class _SumSq(torch.autograd.Function):
    """||r||^2 of a complex tensor (its real and imaginary parts), reduced in
    double by the library in a fixed order (no atomics, no memset: the form
    that HIP graph capture keeps correct on every replay)."""

    @staticmethod
    def forward(ctx, r):
        rr = torch.view_as_real(r.contiguous()).reshape(-1)
        ctx.save_for_backward(rr)
        ctx.shape = r.shape
        return ops.sumsq_diff_(rr)

    @staticmethod
    def backward(ctx, g):
        (rr,) = ctx.saved_tensors
        return torch.view_as_complex((rr * (2.0 * g).float()).reshape(-1, 2)).reshape(ctx.shape)


def _sumsq(r, library: bool):
    if library:
        return _SumSq.apply(r)
    return (torch.view_as_real(r).double() ** 2).sum()


def mri_ei_loss(x: torch.Tensor, y: torch.Tensor, op: MRIOperator, cs: torch.Tensor, lam: float = 1.0,
                library_sums: bool = False):
    """The sketched EI loss of Algorithm 3 with the network taken as the
    identity: sum_b ||y_b - A x_b||^2 + (lam / C) sum_{b,c} ||T_c x_b -
    A^dagger A T_c x_b||^2, for the (sketched) operator `op` and data y.
    Returns (loss, l_MC, l_EI) as float64 scalars; differentiable in x."""
    x3 = x if x.dim() == 3 else x.unsqueeze(0)
    y4 = y if y.dim() == 4 else y.unsqueeze(0)
    r_mc = y4 - mri_fwd(x3, op)
    l_mc = _sumsq(r_mc, library_sums)
    z = rotate_complex(x3, cs)                                   # [B,C,N,N]
    b, c = z.shape[0], z.shape[1]
    zf = z.reshape(b * c, op.n, op.n)
    r = zf - mri_pinv(mri_fwd(zf, op), op)
    l_ei = _sumsq(r, library_sums)
    return l_mc + (lam / c) * l_ei, l_mc, l_ei


def _as_channels(z: torch.Tensor) -> torch.Tensor:
    """complex [B,N,N] -> real [B,2,N,N] (real and imaginary channels)."""
    return torch.view_as_real(z).permute(0, 3, 1, 2).contiguous()


def _as_complex(h: torch.Tensor) -> torch.Tensor:
    """real [B,2,N,N] -> complex [B,N,N]."""
    return torch.view_as_complex(h.permute(0, 2, 3, 1).contiguous())


def mri_skei_ttt_loss(net, x_in: torch.Tensor, y: torch.Tensor, op: MRIOperator, cs: torch.Tensor,
                      lam: float = 1.0):
    """Algorithm 3's loss with a network F (real/imaginary channels):
    x = F(A^dagger y~); ||y_S - A_S x||^2 + lam ||T x - F(A_S^dagger A_S T x)||^2
    (one transformation per iteration, averaged over the rows of cs).
    x_in: the fixed zero-filled start A^dagger y~ [1,N,N] complex."""
    x = _as_complex(net(_as_channels(x_in)))
    y4 = y if y.dim() == 4 else y.unsqueeze(0)
    r_mc = y4 - mri_fwd(x, op)
    l_mc = (torch.view_as_real(r_mc).double() ** 2).sum()
    z = rotate_complex(x, cs)
    b, c = z.shape[0], z.shape[1]
    zf = z.reshape(b * c, op.n, op.n)
    w = _as_complex(net(_as_channels(mri_pinv(mri_fwd(zf, op), op))))
    l_ei = (torch.view_as_real(zf - w).double() ** 2).sum()
    return l_mc + (lam / c) * l_ei, l_mc, l_ei


class MRIProblem:
    """A synthetic multicoil acquisition: ground truth, maps, mask, measured
    k-space y = A x + noise, and the zero-filled start A^dagger y."""

    def __init__(self, n: int = 128, nc: int = 15, accel: int = 4, noise: float = 0.005, seed: int = synth.SEED_MRI,
                 device=None):
        device = device or torch.device("cuda", 0)
        self.x_true = synth.complex_phantom(n, synth.SEED_PHANTOM + seed % 1000)
        self.maps_np = synth.coil_maps(nc, n, seed)
        self.mask_np = synth.cartesian_mask(n, accel, seed=seed)
        self.op = MRIOperator(self.maps_np, self.mask_np, device)
        k = self.op.fwd_(_dev_c64(self.x_true[None], device))
        scale = float(torch.abs(k).max())
        nz = _dev_c64(synth.complex_noise(k.shape, seed + 11), device)
        self.y = (k + noise * scale * nz) * self.op.mask   # noise only on acquired samples
        self.x0 = self.op.pinv_(self.y)                    # zero-filled A^dagger y


def make_problem(**kw) -> MRIProblem:
    return MRIProblem(**kw)


def time_per_iteration(step, iters: int = 20, warmup: int = 3) -> float:
    """Mean wall time (s) of `step()`, device-synchronised."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / iters


class MRIGraphStep:
    """One EI iteration of Algorithm 3 with the network taken as the
    identity -- loss, backward, Adam step on the image -- captured once in a
    HIP graph and replayed.  The operator and data stay fixed (the full
    operator or one coil sketch); each replay takes the rotation written
    into a static (cos, sin) buffer beforehand.  Every kernel of the
    iteration is one of the library's or an elementwise PyTorch kernel, and
    the sums are the library's fixed-order reductions, so the graph holds no
    memset node.  x is updated in place."""

    def __init__(self, x0: torch.Tensor, y: torch.Tensor, op: MRIOperator, lam: float = 1.0, lr: float = 5e-4,
                 warmup: int = 3, select: int = 0):
        """select > 0: the classical sketch, a new subset of `select` coils
        per replay -- the selection matrix is a static device buffer (set by
        step), and the sketched maps, data and weights are formed inside the
        graph by the library's coil mixing."""
        self.x = x0.detach().clone().requires_grad_(True)
        self.y, self.op, self.lam = y, op, lam
        self.cs = torch.zeros((1, 2), device=x0.device, dtype=torch.float32)
        self.cs[0, 0] = 1.0
        self.select = int(select)
        if self.select:
            G = np.zeros((self.select, op.nc))
            G[np.arange(self.select), np.arange(self.select)] = 1.0
            self.G = _dev_c64(G, x0.device)
        self.opt = torch.optim.Adam([self.x], lr=lr, capturable=True)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(warmup):
                self._iteration()
        torch.cuda.current_stream().wait_stream(side)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.loss = self._iteration()
        self.reset(x0)

    def reset(self, x0: torch.Tensor):
        """Back to x0 with fresh Adam moments (the warm-up iterations moved
        them); in place, so the captured graph keeps its addresses."""
        with torch.no_grad():
            self.x.copy_(x0)
            for st in self.opt.state.values():
                for v in st.values():
                    if torch.is_tensor(v):
                        v.zero_()

    def _iteration(self):
        self.opt.zero_grad(set_to_none=True)
        if self.select:
            op = MRIOperator(coil_mix_(self.G, self.op.maps), self.op.mask)
            op.weights   # formed inside the graph from this replay's maps
            y = coil_mix_(self.G, self.y)
        else:
            op, y = self.op, self.y
        loss, _, _ = mri_ei_loss(self.x, y, op, self.cs, self.lam, library_sums=True)
        loss.backward()
        self.opt.step()
        return loss.detach()

    def step(self, cos_sin: torch.Tensor, coils=None):
        """One iteration with the rotation cos_sin [1, 2] (and, for the
        classical sketch, the coil subset `coils`); returns the loss (device
        scalar, valid once the stream reaches it)."""
        self.cs.copy_(cos_sin)
        if self.select:
            if coils is None or len(coils) != self.select:
                raise ValueError(f"pass {self.select} coils")
            G = np.zeros((self.select, self.op.nc), dtype=np.complex64)
            G[np.arange(self.select), np.asarray(coils)] = 1.0
            self.G.copy_(torch.from_numpy(G))
        self.graph.replay()
        return self.loss


"""Sketched equivariant test-time training (SkEI-TTT, Algorithm 2).

A pretrained reconstruction network F_theta is adapted to one measurement
y~ by minimising the sketched TTT loss of Eq. (skeilossttt): per iteration,
with a sampled sketch S_k and transformation T_i,

    x     = F_theta(A^dagger y~)                     (A^dagger = FBP, Sec. 4.1.1)
    l_MC  = || S_k y~ - A_{S_k} x ||^2               (sketched MC loss)
    z     = T_i x
    l_EI  = || z - F_theta( fbp_{S_k}(A_{S_k} z) ) ||^2   (sketched EI regularisation)
    theta <- Adam step on grad_theta (l_MC + lambda l_EI)

updating either every parameter or only the BatchNorm affine parameters
(Sec. 3.3, "BN-NA").  The sketches are the interleaved angle subsets
S_k = {k, k+N, ...} (Sec. 4.2.1), one drawn uniformly per iteration; the
transformations are rotations by whole degrees 1..360 (Sec. 4.1.3).

Every CT operator (the residual S y - A_S x, A_S, fbp_S, T and, in the
backward pass, their hand-written transposes) is a call into the HIP
library through the autograd Functions of ``ops``.  The network is a plain
PyTorch module: a residual U-Net with BatchNorm (Sec. 4.1.3 uses the U-Net
of Ronneberger et al. in its residual form); its convolutions are PyTorch's.
"""
from __future__ import annotations

import time

import numpy as np
import torch
import torch.nn as nn

from . import ops, synth


class _Block(nn.Module):
    def __init__(self, cin, cout):
        super().__init__()
        self.body = nn.Sequential(
            nn.Conv2d(cin, cout, 3, padding=1, bias=False), nn.BatchNorm2d(cout), nn.ReLU(inplace=True),
            nn.Conv2d(cout, cout, 3, padding=1, bias=False), nn.BatchNorm2d(cout), nn.ReLU(inplace=True))

    def forward(self, x):
        return self.body(x)


class ResUNet(nn.Module):
    """A residual U-Net with BatchNorm: F(x) = x + U(x) for images of
    `channels` channels (1 for CT, 2 -- real and imaginary parts -- for MRI)
    whose side is a multiple of 2^(depth-1)."""

    def __init__(self, width: int = 32, depth: int = 4, channels: int = 1):
        super().__init__()
        ch = [width * 2 ** i for i in range(depth)]
        self.down = nn.ModuleList([_Block(channels if i == 0 else ch[i - 1], ch[i]) for i in range(depth)])
        self.up = nn.ModuleList([nn.ConvTranspose2d(ch[i], ch[i - 1], 2, stride=2) for i in range(depth - 1, 0, -1)])
        self.dec = nn.ModuleList([_Block(2 * ch[i - 1], ch[i - 1]) for i in range(depth - 1, 0, -1)])
        self.out = nn.Conv2d(ch[0], channels, 1)
        self.pool = nn.MaxPool2d(2)

    def forward(self, x):
        skips = []
        h = x
        for i, blk in enumerate(self.down):
            h = blk(h if i == 0 else self.pool(h))
            skips.append(h)
        for up, dec, skip in zip(self.up, self.dec, reversed(skips[:-1])):
            h = dec(torch.cat([up(h), skip], dim=1))
        return x + self.out(h)


def bn_parameters(net: nn.Module):
    """The BatchNorm affine parameters (scale and shift) of a network."""
    return [p for m in net.modules() if isinstance(m, nn.BatchNorm2d) for p in (m.weight, m.bias)]


def rotation_table(device) -> torch.Tensor:
    """(cos, sin) of the rotations by 1..360 degrees, [360, 2] float32."""
    phi = np.deg2rad(np.arange(1, 361, dtype=np.float64))
    return torch.from_numpy(synth.cos_sin(phi).astype(np.float32)).to(device)


def skei_ttt_loss(net, x_in, y, geom: ops.Geometry, sketch, cs, lam: float = 1.0):
    """The sketched TTT loss of one iteration and its parts.
    x_in: A^dagger y~ as [1, N, N]; y: the whole measured sinogram
    [1, N_theta, N_det]; sketch: the angle list of S_k; cs: [1, 2] (cos, sin)
    of T_i.  Returns (loss, l_MC, l_EI) as float64 scalars."""
    sk = ops._as_sketch(geom, sketch)
    x = net(x_in.unsqueeze(1)).squeeze(1)                     # F(A^dagger y~), [1, N, N]
    l_mc = (ops.radon_resid(x, y, geom, sk).double() ** 2).sum()
    z = ops.rotate(x, cs).reshape(x.shape)                     # T_i x
    w = net(ops.fbp(ops.radon_fwd(z, geom, sk), geom, sk).unsqueeze(1)).squeeze(1)
    l_ei = ((z - w).double() ** 2).sum()
    return l_mc + lam * l_ei, l_mc, l_ei


class SkEITTT:
    """Algorithm 2 for one measurement.

    y: [N_theta, N_det] or [1, N_theta, N_det] device float32 (the whole scan);
    splits: N of the interleaved sketches (1 = every angle); mode "full"
    adapts every parameter, "bn" only the BatchNorm affine parameters; Adam
    with learning rate 5e-4 (Sec. 4.1.3)."""

    def __init__(self, net: nn.Module, geom: ops.Geometry, y: torch.Tensor, splits: int = 1, mode: str = "full",
                 lam: float = 1.0, lr: float = 5e-4, seed: int = synth.SEED_SKETCH):
        if mode not in ("full", "bn"):
            raise ValueError("mode is 'full' or 'bn'")
        if geom.n_angles % splits:
            raise ValueError("the interleaved sketches need N_theta divisible by the split count")
        self.net, self.geom, self.lam = net, geom, float(lam)
        self.y = y if y.dim() == 3 else y.unsqueeze(0)
        self.x_in = ops.fbp_(geom, self.y, geom.full()).contiguous()     # A^dagger y~ (fixed)
        self.sketches = [geom.sketch(synth.interleaved_sketch(geom.n_angles, splits, k)) for k in range(splits)]
        self.params = list(net.parameters()) if mode == "full" else bn_parameters(net)
        if mode == "bn":
            for p in net.parameters():
                p.requires_grad_(False)
            for p in self.params:
                p.requires_grad_(True)
        self.opt = torch.optim.Adam(self.params, lr=lr)
        self.rot = rotation_table(self.y.device)
        self.rng = synth.rng(seed)
        self.losses = []

    def step(self):
        k = int(self.rng.integers(len(self.sketches)))
        i = int(self.rng.integers(360))
        self.net.train()
        self.opt.zero_grad(set_to_none=True)
        loss, _, _ = skei_ttt_loss(self.net, self.x_in, self.y, self.geom, self.sketches[k], self.rot[i:i + 1],
                                   self.lam)
        loss.backward()
        self.opt.step()
        self.losses.append(loss.detach())
        return loss

    def run(self, iters: int):
        for _ in range(iters):
            self.step()
        return self

    @torch.no_grad()
    def reconstruct(self):
        """The adapted reconstruction F_theta(A^dagger y~)."""
        self.net.eval()
        return self.net(self.x_in.unsqueeze(1)).squeeze(1)


def time_per_iteration(ttt: SkEITTT, iters: int, warmup: int = 3) -> float:
    """Mean wall time (s) of one TTT iteration, device-synchronised."""
    ttt.run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ttt.run(iters)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / iters


def network_size(net: nn.Module) -> dict:
    return {"parameters": sum(p.numel() for p in net.parameters()),
            "bn_parameters": sum(p.numel() for p in bn_parameters(net))}


__all__ = ["ResUNet", "bn_parameters", "rotation_table", "skei_ttt_loss", "SkEITTT", "time_per_iteration",
           "network_size"]

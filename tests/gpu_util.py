"""Helpers shared by the GPU parity tests (host-side comparisons only)."""
import numpy as np
import torch


def dev():
    return torch.device("cuda", 0)


def to_dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev(), dtype=dtype)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def relerr(got, want):
    """Relative max-norm error ||got - want||_inf / ||want||_inf."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return float(np.max(np.abs(got - want)) / np.max(np.abs(want)))


def adjoint_gap(ax, y, x, aty):
    """|<Ax,y> - <x,A^T y>| / |<Ax,y>| with inner products in float64 on the host."""
    lhs = float(np.vdot(np.asarray(ax, np.float64).ravel(), np.asarray(y, np.float64).ravel()))
    rhs = float(np.vdot(np.asarray(x, np.float64).ravel(), np.asarray(aty, np.float64).ravel()))
    return abs(lhs - rhs) / abs(lhs)


def f32(a):
    """Round to float32 and back: the exact values both sides receive."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)

"""Seeded synthetic inputs shared by the HIP path's tests/benchmark and the oracle.

This module holds none of the method's arithmetic: it only draws phantoms,
angle lists, rotation angles and noise with numpy's PCG64 generator.  The
paper's CT100 images (Sec. 4.1.1) are not available; random ellipse phantoms
of the same kind of piecewise-constant structure stand in for them.

Seeds used across the repository: phantoms 1000+i, sketches 2000,
rotations 3000, noise 4000, arrivals 5000.
"""
from __future__ import annotations

import math

import numpy as np

SEED_PHANTOM = 1000
SEED_SKETCH = 2000
SEED_ROTATION = 3000
SEED_NOISE = 4000
SEED_ARRIVALS = 5000


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def ellipse_params(seed: int, n_min: int = 5, n_max: int = 10) -> np.ndarray:
    """Draw 5-10 ellipses: rows (cx, cy, a, b, alpha, intensity).

    Centres uniform in the disk of radius 0.8 (normalised [-1,1]^2 frame),
    semi-axes U(0.05, 0.4), orientation U[0, pi), intensity U(0.1, 1).
    """
    g = rng(seed)
    k = int(g.integers(n_min, n_max + 1))
    r = 0.8 * np.sqrt(g.uniform(0.0, 1.0, k))
    t = g.uniform(0.0, 2.0 * math.pi, k)
    cx, cy = r * np.cos(t), r * np.sin(t)
    a = g.uniform(0.05, 0.4, k)
    b = g.uniform(0.05, 0.4, k)
    alpha = g.uniform(0.0, math.pi, k)
    inten = g.uniform(0.1, 1.0, k)
    return np.stack([cx, cy, a, b, alpha, inten], axis=1)


def ellipse_phantom(n: int, seed: int, dtype=np.float32) -> np.ndarray:
    """Point-sample an ellipse phantom at pixel centres; overlaps add.

    Pixel (i, j) sits at normalised ((j - (n-1)/2) / (n/2), (i - (n-1)/2) / (n/2)).
    """
    e = ellipse_params(seed)
    c = (n - 1) / 2.0
    coords = (np.arange(n, dtype=np.float64) - c) / (n / 2.0)
    X, Y = np.meshgrid(coords, coords)   # X varies along columns (j), Y along rows (i)
    img = np.zeros((n, n), dtype=np.float64)
    for cx, cy, a, b, alpha, inten in e:
        ca, sa = math.cos(alpha), math.sin(alpha)
        dx, dy = X - cx, Y - cy
        xr = ca * dx + sa * dy
        yr = -sa * dx + ca * dy
        img[(xr / a) ** 2 + (yr / b) ** 2 <= 1.0] += inten
    return img.astype(dtype)


def phantom_batch(n: int, batch: int, first: int = 0, dtype=np.float32) -> np.ndarray:
    return np.stack([ellipse_phantom(n, SEED_PHANTOM + first + i, dtype) for i in range(batch)])


def interleaved_sketch(n_angles: int, n_splits: int, k: int) -> np.ndarray:
    """S_k of the N-way interleaved split: angles k, k+N, k+2N, ... (int32)."""
    if not 0 <= k < n_splits:
        raise ValueError("k out of range")
    return np.arange(k, n_angles, n_splits, dtype=np.int32)


def random_sketch(n_angles: int, m: int, seed: int = SEED_SKETCH) -> np.ndarray:
    """A seeded random subset of m distinct angles, ascending (int32)."""
    g = rng(seed)
    return np.sort(g.choice(n_angles, size=m, replace=False)).astype(np.int32)


def rotation_angles(copies: int, seed: int = SEED_ROTATION) -> np.ndarray:
    """phi ~ U[0, 2 pi), float64."""
    return rng(seed).uniform(0.0, 2.0 * math.pi, copies)


def cos_sin(phi) -> np.ndarray:
    """[C,2] table of (cos phi, sin phi) in float64."""
    phi = np.asarray(phi, dtype=np.float64).reshape(-1)
    return np.stack([np.cos(phi), np.sin(phi)], axis=1)


def std_noise(shape, seed: int = SEED_NOISE) -> np.ndarray:
    """Standard normal draws (float64) to be scaled by the caller."""
    return rng(seed).standard_normal(shape)


def add_relative_noise(y_clean: np.ndarray, z: np.ndarray, rel: float = 0.01) -> np.ndarray:
    """y = y_clean + rel * max(y_clean) * z  (sigma = 0.01 * max)."""
    return y_clean + rel * float(np.max(y_clean)) * z


def uniform(shape, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    return rng(seed).uniform(lo, hi, shape)


SEED_PROBLEMS = 6000


def uneven_problems(count: int = 64, sizes=(128, 256, 512), angles=(90, 720), ratios=(2, 4, 8), copies: int = 8,
                    seed: int = SEED_PROBLEMS) -> list[dict]:
    """A seeded list of uneven EI problems (the batched-plan workload):
    N drawn from `sizes`, N_theta ~ U{angles[0]..angles[1]},
    N_det = ceil(sqrt(2) N) + 1, sketch size m = N_theta // ratio with ratio
    drawn from `ratios` (a random subset, ascending), `copies` rotations.
    Each entry also carries its own seeds for the phantom, sketch, rotations
    and noise."""
    g = rng(seed)
    out = []
    for i in range(count):
        n = int(g.choice(sizes))
        na = int(g.integers(angles[0], angles[1] + 1))
        ratio = int(g.choice(ratios))
        out.append(dict(n=n, n_angles=na, n_det=int(np.ceil(np.sqrt(2.0) * n)) + 1, ratio=ratio,
                        m=max(1, na // ratio), copies=copies, phantom_seed=SEED_PHANTOM + 100 * i,
                        sketch_seed=SEED_SKETCH + 100 * i, rotation_seed=SEED_ROTATION + 100 * i,
                        noise_seed=SEED_NOISE + 100 * i))
    return out


def poisson_jobs(count: int, rate: float, sizes=(256, 512, 1024), angles=(180, 1440), ratios=(2, 4, 8),
                 copies: int = 16, iters: int = 50, seed: int = SEED_ARRIVALS) -> list[dict]:
    """A seeded stream of test-time-adaptation jobs: Poisson arrivals at
    `rate` jobs per second (exponential gaps, first job at t = 0), N drawn
    from `sizes`, N_theta ~ U{angles}, N_det = ceil(sqrt(2) N), sketch ratio
    from `ratios` (interleaved subsets of N_theta // ratio angles), `copies`
    rotations and `iters` iterations each, with per-job seeds."""
    g = rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        if i > 0:
            t += float(g.exponential(1.0 / rate))
        n = int(g.choice(sizes))
        na = int(g.integers(angles[0], angles[1] + 1))
        ratio = int(g.choice(ratios))
        out.append(dict(job=i, arrival=t, n=n, n_angles=na, n_det=int(np.ceil(np.sqrt(2.0) * n)), ratio=ratio,
                        m=max(1, na // ratio), copies=copies, iters=iters, phantom_seed=SEED_PHANTOM + 7919 * (i + 1),
                        rotation_seed=SEED_ROTATION + 7919 * (i + 1), noise_seed=SEED_NOISE + 7919 * (i + 1)))
    return out


def dense_sketch_matrix(m: int, n_rows: int, kind: str = "gaussian", seed: int = SEED_SKETCH) -> np.ndarray:
    """A dense sketch G in R^{m x n_rows} (float64): i.i.d. N(0, 1/m) entries
    ("gaussian") or +-1/sqrt(m) with equal probability ("rademacher"), so
    that E[G^T G] = I.  Seeded; passed to both the library and the oracle."""
    g = rng(seed)
    if kind == "gaussian":
        return g.standard_normal((m, n_rows)) / np.sqrt(m)
    if kind == "rademacher":
        return np.where(g.integers(0, 2, size=(m, n_rows)) == 1, 1.0, -1.0) / np.sqrt(m)
    raise ValueError("kind is 'gaussian' or 'rademacher'")


# ---------------------------------------------------------------- multicoil MRI
SEED_MRI = 7000


def coil_maps(nc: int, n: int, seed: int = SEED_MRI) -> np.ndarray:
    """Smooth synthetic coil sensitivities [nc, n, n] complex128: Gaussian
    profiles centred on a ring around the field of view (radius 0.6 n, width
    0.35 n, small random jitter), each with a smooth linear phase, then
    normalised so that sum_c |C_c|^2 = 1 at every pixel.  They stand in for
    the ESPIRiT maps of measured data."""
    g = rng(seed)
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    c0 = 0.5 * (n - 1)
    maps = np.empty((nc, n, n), dtype=np.complex128)
    for c in range(nc):
        th = 2.0 * math.pi * c / nc + g.uniform(-0.1, 0.1)
        cx, cy = c0 + 0.6 * n * math.cos(th), c0 + 0.6 * n * math.sin(th)
        sig = 0.35 * n * g.uniform(0.9, 1.1)
        mag = np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2.0 * sig * sig))
        ph = g.uniform(-math.pi, math.pi) + (g.uniform(-1.0, 1.0) * xx + g.uniform(-1.0, 1.0) * yy) * math.pi / n
        maps[c] = mag * np.exp(1j * ph)
    return maps / np.sqrt(np.sum(np.abs(maps) ** 2, axis=0))[None]


def complex_phantom(n: int, seed: int) -> np.ndarray:
    """An ellipse phantom with a smooth random phase, [n, n] complex128."""
    g = rng(seed + 1)
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64) / n
    ph = g.uniform(-1.0, 1.0) * xx + g.uniform(-1.0, 1.0) * yy + g.uniform(-0.5, 0.5) * xx * yy
    return ellipse_phantom(n, seed, dtype=np.float64) * np.exp(1j * math.pi * ph)


def cartesian_mask(n: int, accel: int = 4, center_frac: float = 0.08, seed: int = SEED_MRI) -> np.ndarray:
    """Cartesian undersampling of the phase-encode (row) direction at
    acceleration `accel` (n / accel rows kept): every row within
    center_frac * n of the zero frequency (the rows near index 0 and n - 1
    of the unshifted DFT grid), the rest drawn at random; [n, n] float64 0/1."""
    g = rng(seed + 2)
    keep = max(1, n // accel)
    nc = max(1, min(keep, int(round(center_frac * n))))
    freq = np.minimum(np.arange(n), n - np.arange(n))      # |frequency| of each row
    centre = np.argsort(freq, kind="stable")[:nc]
    rest = np.setdiff1d(np.arange(n), centre)
    rows = np.concatenate([centre, g.choice(rest, size=keep - nc, replace=False)])
    mask = np.zeros((n, n))
    mask[rows] = 1.0
    return mask


def rademacher_signs(rows: int, cols: int, seed: int = SEED_MRI) -> np.ndarray:
    """i.i.d. +-1 entries with equal probability, [rows, cols] float64."""
    return np.where(rng(seed + 3).integers(0, 2, size=(rows, cols)) == 1, 1.0, -1.0)


def complex_noise(shape, seed: int) -> np.ndarray:
    """Standard complex Gaussian noise (independent N(0, 1/2) parts)."""
    g = rng(seed)
    return (g.standard_normal(shape) + 1j * g.standard_normal(shape)) / math.sqrt(2.0)

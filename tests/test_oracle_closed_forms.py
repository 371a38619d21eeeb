"""Pins P3-P6, P8-P10: the oracle against closed forms, symmetries and special cases.

None of these re-types the oracle's formulas: they compare with analytic line
integrals (Gaussian, disk), with plain column/row sums, with numpy's exact
90-degree rotation, and with the reconstruction property of FBP.
"""
import math

import numpy as np
import pytest


def gaussian_image(n, x0, y0, sigma):
    c = (n - 1) / 2.0
    X, Y = np.meshgrid(np.arange(n) - c, np.arange(n) - c)
    return np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / (2 * sigma ** 2))


def gaussian_sinogram(n_angles, n_det, x0, y0, sigma):
    """Exact line integrals of the continuous Gaussian: sqrt(2 pi) sigma exp(-(s - s0)^2 / 2 sigma^2)."""
    s = np.arange(n_det) - (n_det - 1) / 2.0
    th = math.pi * np.arange(n_angles) / n_angles
    s0 = x0 * np.cos(th) + y0 * np.sin(th)
    return math.sqrt(2 * math.pi) * sigma * np.exp(-(s[None, :] - s0[:, None]) ** 2 / (2 * sigma ** 2))


# ---------------------------------------------------------------- P3 / P4
@pytest.mark.parametrize("n_det", [91, 90])
def test_axis_angles_give_column_and_row_sums(orc, n_det):
    n, n_angles = 64, 60
    x = np.random.default_rng(1).uniform(0, 1, (n, n))
    y = orc.radon_fwd(x, n_angles, n_det, np.array([0, 30], dtype=np.int32))
    col, row = x.sum(axis=0), x.sum(axis=1)
    off = (n_det - n) // 2
    if (n_det - n) % 2:          # detector centres fall half-way between pixel centres
        pad = np.concatenate([[0.0], col, [0.0]])
        want0 = np.zeros(n_det)
        want0[off:off + n + 1] = 0.5 * (pad[:-1] + pad[1:])
        padr = np.concatenate([[0.0], row, [0.0]])
        want90 = np.zeros(n_det)
        want90[off:off + n + 1] = 0.5 * (padr[:-1] + padr[1:])
    else:
        want0 = np.zeros(n_det)
        want0[off:off + n] = col
        want90 = np.zeros(n_det)
        want90[off:off + n] = row
    assert np.max(np.abs(y[0] - want0)) < 1e-12
    assert np.max(np.abs(y[1] - want90)) < 1e-12 * np.max(want90)


def test_mass_conservation(orc):
    """Every projection sums to the image sum: exactly at 0 and 90 degrees,
    and to within the interpolation error for a smooth image elsewhere."""
    n, n_angles, n_det = 64, 60, 91
    x = np.random.default_rng(2).uniform(0, 1, (n, n))
    y = orc.radon_fwd(x, n_angles, n_det, np.array([0, 30], dtype=np.int32))
    assert np.max(np.abs(y.sum(axis=1) - x.sum())) < 1e-10
    g = gaussian_image(n, 2.3, -1.7, 6.0)
    yg = orc.radon_fwd(g, n_angles, n_det)
    rel = np.abs(yg.sum(axis=1) - g.sum()) / g.sum()
    assert rel.max() < 1e-4
    # a point-sampled disk has edges, so its per-pixel interpolation weights
    # (which sum to 0.828 .. 1.414 at 45 degrees) no longer average out exactly
    c = (n - 1) / 2.0
    X, Y = np.meshgrid(np.arange(n) - c, np.arange(n) - c)
    disk = (X ** 2 + Y ** 2 <= 20.0 ** 2).astype(float)
    yd = orc.radon_fwd(disk, n_angles, n_det)
    assert np.abs(yd.sum(axis=1) / disk.sum() - 1).max() < 2e-3


# ---------------------------------------------------------------- P5
def test_gaussian_sinogram_converges_to_line_integrals(orc):
    n, n_angles, n_det = 128, 36, 183
    errs = []
    for sigma in (2.0, 4.0, 8.0):
        x0, y0 = 7.3, -11.6          # off-centre: pins the s = X cos + Y sin orientation
        y = orc.radon_fwd(gaussian_image(n, x0, y0, sigma), n_angles, n_det)
        want = gaussian_sinogram(n_angles, n_det, x0, y0, sigma)
        errs.append(np.max(np.abs(y - want)) / np.max(want))
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1]
    assert errs[2] < 2e-3


def test_disk_chord_lengths(orc):
    """Point-sampled disk of radius r: inner rays approach 2 sqrt(r^2 - s^2)."""
    n, n_angles, n_det = 128, 24, 183
    c = (n - 1) / 2.0
    X, Y = np.meshgrid(np.arange(n) - c, np.arange(n) - c)
    s = np.arange(n_det) - (n_det - 1) / 2.0
    errs = []
    for r in (12.0, 24.0, 48.0):
        disk = (X ** 2 + Y ** 2 <= r * r).astype(float)
        y = orc.radon_fwd(disk, n_angles, n_det)
        inner = np.abs(s) < 0.8 * r
        want = 2 * np.sqrt(r * r - s[inner] ** 2)
        errs.append(np.max(np.abs(y[:, inner] - want[None, :]) / want[None, :]))
    assert errs[2] < errs[0]
    assert errs[2] < 0.03


def test_ellipse_projection_matches_analytic_formula(orc):
    """Projection of a rotated, shifted ellipse (Kak & Slaney ch. 3):
    p(theta, t) = 2 rho a b / a2 * sqrt(a2 - t'^2), a2 = a^2 cos^2(theta-alpha) + b^2 sin^2(theta-alpha),
    t' = t - (x0 cos theta + y0 sin theta)."""
    n, n_angles, n_det = 256, 12, 365
    c = (n - 1) / 2.0
    X, Y = np.meshgrid(np.arange(n) - c, np.arange(n) - c)
    x0, y0, a, b, alpha, rho = 20.0, -13.0, 70.0, 35.0, 0.6, 0.8
    xr = math.cos(alpha) * (X - x0) + math.sin(alpha) * (Y - y0)
    yr = -math.sin(alpha) * (X - x0) + math.cos(alpha) * (Y - y0)
    img = rho * ((xr / a) ** 2 + (yr / b) ** 2 <= 1.0)
    y = orc.radon_fwd(img, n_angles, n_det)
    s = np.arange(n_det) - (n_det - 1) / 2.0
    for ai in range(n_angles):
        th = math.pi * ai / n_angles
        a2 = (a * math.cos(th - alpha)) ** 2 + (b * math.sin(th - alpha)) ** 2
        t = s - (x0 * math.cos(th) + y0 * math.sin(th))
        inner = t ** 2 < 0.6 * a2
        want = 2 * rho * a * b / a2 * np.sqrt(a2 - t[inner] ** 2)
        assert np.max(np.abs(y[ai, inner] - want) / want) < 0.02


# ---------------------------------------------------------------- P6
def test_quarter_turn_symmetry(orc):
    """A x at theta + pi/2 equals A of the image turned by 90 degrees at theta."""
    n, n_angles, n_det = 48, 40, 69
    x = np.random.default_rng(3).uniform(0, 1, (n, n))
    first = np.arange(n_angles // 2, dtype=np.int32)
    y_hi = orc.radon_fwd(x, n_angles, n_det, first + n_angles // 2)
    y_rot = orc.radon_fwd(np.rot90(x, 1), n_angles, n_det, first)
    assert np.max(np.abs(y_hi - y_rot)) < 1e-12 * np.max(np.abs(y_hi))


def test_rotation_commutes_with_projection_at_quarter_turn(orc):
    """A(T_phi x)(theta) = A x(theta - phi) for phi = pi/2 (T is then an exact permutation)."""
    n, n_angles, n_det = 48, 40, 69
    x = np.random.default_rng(4).uniform(0, 1, (n, n))
    tx = orc.rotate(x, np.array([[0.0, 1.0]]))[0]
    upper = np.arange(n_angles // 2, n_angles, dtype=np.int32)
    lhs = orc.radon_fwd(tx, n_angles, n_det, upper)
    rhs = orc.radon_fwd(x, n_angles, n_det, upper - n_angles // 2)
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(rhs))


# ---------------------------------------------------------------- P9
def test_fbp_reconstructs_smooth_image(orc):
    n, n_angles, n_det = 64, 180, 91
    g = gaussian_image(n, 4.0, -3.0, 6.0)
    rec = orc.fbp(orc.radon_fwd(g, n_angles, n_det), n, n_angles)
    c = (n - 1) / 2.0
    X, Y = np.meshgrid(np.arange(n) - c, np.arange(n) - c)
    inside = X ** 2 + Y ** 2 < 24 ** 2
    err = np.max(np.abs(rec - g)[inside])
    assert err < 0.02            # pins the pi/m scale and the ramp normalisation
    # sketched FBP of the sketched sinogram is still a reconstruction
    idx = np.arange(0, n_angles, 4, dtype=np.int32)
    rec_s = orc.fbp(orc.radon_fwd(g, n_angles, n_det, idx), n, n_angles, idx)
    assert np.max(np.abs(rec_s - g)[inside]) < 0.05


# ---------------------------------------------------------------- P10
def test_rotation_special_cases(orc):
    n = 32
    x = np.random.default_rng(6).uniform(0, 1, (n, n))
    out = orc.rotate(x, np.array([[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0]]))
    assert np.array_equal(out[0], x)
    assert np.array_equal(out[1], np.rot90(x, -1))
    assert np.array_equal(out[2], np.rot90(x, 2))


def test_rotation_moves_blob_centre(orc):
    n, phi = 96, 0.9
    q0 = np.array([14.0, -9.0])
    x = gaussian_image(n, q0[0], q0[1], 3.0)
    out = orc.rotate(x, np.array([[math.cos(phi), math.sin(phi)]]))[0]
    c = (n - 1) / 2.0
    X, Y = np.meshgrid(np.arange(n) - c, np.arange(n) - c)
    got = np.array([(out * X).sum(), (out * Y).sum()]) / out.sum()
    want = np.array([math.cos(phi) * q0[0] - math.sin(phi) * q0[1], math.sin(phi) * q0[0] + math.cos(phi) * q0[1]])
    assert np.max(np.abs(got - want)) < 0.05

"""Pins P2, P7, P11, P12: adjoint identities, sketch consistency, gradient by
central finite differences, and linearity -- at sizes beyond the dense tests."""
import math

import numpy as np
import pytest

from paper_2411_05771_amd import synth

N, NA, ND = 64, 60, 91


def rel_gap(a, b):
    return abs(a - b) / abs(a)


def test_adjoint_identities(orc):
    g = np.random.default_rng(10)
    x = g.uniform(0, 1, (2, N, N))
    y = g.uniform(0, 1, (2, NA, ND))
    idx = synth.random_sketch(NA, 15, seed=7)
    ys = y[:, :15]
    assert rel_gap(np.vdot(orc.radon_fwd(x, NA, ND), y), np.vdot(x, orc.radon_adj(y, N, NA))) < 1e-12
    assert rel_gap(np.vdot(orc.radon_fwd(x, NA, ND, idx), ys), np.vdot(x, orc.radon_adj(ys, N, NA, idx))) < 1e-12
    assert rel_gap(np.vdot(orc.backproject(y, N, NA), x), np.vdot(y, orc.backproject_T(x, NA, ND))) < 1e-12
    assert rel_gap(np.vdot(orc.ramp(y), y[::-1]), np.vdot(y, orc.ramp(y[::-1]))) < 1e-12
    assert rel_gap(np.vdot(orc.fbp(ys, N, NA, idx), x), np.vdot(ys, orc.fbp_adj(x, NA, ND, idx))) < 1e-12
    cs = synth.cos_sin(synth.rotation_angles(3))
    h = g.uniform(0, 1, (2, 3, N, N))
    assert rel_gap(np.vdot(orc.rotate(x, cs), h), np.vdot(x, orc.rotate_adj(h, cs))) < 1e-12


def test_sketch_is_row_selection(orc):
    x = synth.ellipse_phantom(N, 1000).astype(np.float64)
    full = orc.radon_fwd(x, NA, ND)
    idx = synth.interleaved_sketch(NA, 4, 0)
    assert np.array_equal(orc.radon_fwd(x, NA, ND, idx), full[idx])
    ys = np.random.default_rng(11).uniform(0, 1, (idx.size, ND))
    zero_filled = np.zeros((NA, ND))
    zero_filled[idx] = ys
    assert np.max(np.abs(orc.radon_adj(ys, N, NA, idx) - orc.radon_adj(zero_filled, N, NA))) < 1e-12


def test_linearity(orc):
    g = np.random.default_rng(12)
    x, z = g.uniform(0, 1, (2, N, N))
    a, b = 0.7, -1.3
    lhs = orc.radon_fwd(a * x + b * z, NA, ND)
    rhs = a * orc.radon_fwd(x, NA, ND) + b * orc.radon_fwd(z, NA, ND)
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(lhs))


@pytest.mark.parametrize("mc", ["full", "sketch"])
def test_gradient_central_differences(orc, mc):
    """16 seeded unit directions, h = 1e-4; the loss is quadratic so central
    differences are exact up to rounding."""
    n, na, nd = 16, 12, 23
    x = synth.ellipse_phantom(n, 1001).astype(np.float64)
    y = orc.radon_fwd(synth.ellipse_phantom(n, 1002).astype(np.float64), na, nd)
    idx = np.array([0, 4, 7, 9], dtype=np.int32)
    cs = synth.cos_sin(synth.rotation_angles(3, seed=21))
    mc_idx = idx if mc == "sketch" else None
    loss, grad = orc.ei_loss_grad(x, y, na, idx, cs, 0.8, mc_idx)
    g = np.random.default_rng(13)
    h = 1e-4
    for _ in range(16):
        v = g.standard_normal((n, n))
        v /= np.linalg.norm(v)
        lp, _ = orc.ei_loss_grad(x + h * v, y, na, idx, cs, 0.8, mc_idx, want_grad=False)
        lm, _ = orc.ei_loss_grad(x - h * v, y, na, idx, cs, 0.8, mc_idx, want_grad=False)
        fd = (lp - lm) / (2 * h)
        an = float(np.vdot(grad, v))
        assert abs(fd - an) <= 1e-8 * max(abs(an), 1e-3 * np.linalg.norm(grad))


def test_batch_is_independent_images(orc):
    n, na, nd = 16, 12, 23
    xb = synth.phantom_batch(n, 3).astype(np.float64)
    yb = orc.radon_fwd(synth.phantom_batch(n, 3, first=10).astype(np.float64), na, nd)
    idx = np.array([1, 5, 8], dtype=np.int32)
    cs = synth.cos_sin([0.3, 2.0])
    lb, gb = orc.ei_loss_grad(xb, yb, na, idx, cs, 1.0)
    parts = [orc.ei_loss_grad(xb[i], yb[i], na, idx, cs, 1.0) for i in range(3)]
    assert abs(lb - sum(p[0] for p in parts)) < 1e-12 * lb
    for i in range(3):
        assert np.max(np.abs(gb[i] - parts[i][1])) < 1e-12 * np.max(np.abs(gb[i]))

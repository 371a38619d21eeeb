"""Pin P1: the oracle's loops equal dense matrices built from closed-form entries.

Tiny problems (8x8 images, 13 detectors, 8 and 12 angles so that the 45 and
135 degree branch ties are included).  Any dropped term, wrong sign, wrong
index or transposed operand in a loop changes some matrix entry.
"""
import math

import numpy as np
import pytest

import dense_ref as D

N, NDET = 8, 13


def columns(op, d):
    """Matrix of a linear map by applying it to the canonical basis."""
    return np.stack([op(e) for e in np.eye(d)], axis=1)


@pytest.mark.parametrize("n_angles", [8, 12])
def test_joseph_forward_and_adjoint_match_closed_form(orc, n_angles):
    A = D.joseph_matrix(N, n_angles, NDET)
    fwd = columns(lambda e: orc.radon_fwd(e.reshape(N, N), n_angles, NDET).reshape(-1), N * N)
    adj = columns(lambda e: orc.radon_adj(e.reshape(n_angles, NDET), N, n_angles).reshape(-1), n_angles * NDET)
    assert np.max(np.abs(fwd - A)) < 1e-13
    assert np.max(np.abs(adj - A.T)) < 1e-13


def test_joseph_sketch_rows_match_closed_form(orc):
    idx = np.array([5, 1, 1, 9], dtype=np.int32)          # any order, duplicates allowed
    A = D.joseph_matrix(N, 12, NDET, idx)
    fwd = columns(lambda e: orc.radon_fwd(e.reshape(N, N), 12, NDET, idx).reshape(-1), N * N)
    adj = columns(lambda e: orc.radon_adj(e.reshape(len(idx), NDET), N, 12, idx).reshape(-1), len(idx) * NDET)
    assert np.max(np.abs(fwd - A)) < 1e-13
    assert np.max(np.abs(adj - A.T)) < 1e-13


@pytest.mark.parametrize("n_angles", [8, 12])
def test_backprojection_and_transpose_match_closed_form(orc, n_angles):
    B = D.backprojection_matrix(N, n_angles, NDET)
    bp = columns(lambda e: orc.backproject(e.reshape(n_angles, NDET), N, n_angles).reshape(-1), n_angles * NDET)
    bpT = columns(lambda e: orc.backproject_T(e.reshape(N, N), n_angles, NDET).reshape(-1), N * N)
    assert np.max(np.abs(bp - B)) < 1e-13
    assert np.max(np.abs(bpT - B.T)) < 1e-13


@pytest.mark.parametrize("n_det", [13, 14, 31])
def test_ramp_matches_quadrature_toeplitz(orc, n_det):
    H = D.ramp_matrix(n_det)
    got = columns(lambda e: orc.ramp(e[None]).reshape(-1), n_det)
    assert np.max(np.abs(got - H)) < 1e-12


def test_fbp_matches_dense_composition(orc):
    n_angles, idx = 12, np.array([0, 3, 7, 10], dtype=np.int32)
    F = (math.pi / len(idx)) * D.backprojection_matrix(N, n_angles, NDET, idx) @ np.kron(np.eye(len(idx)), D.ramp_matrix(NDET))
    got = columns(lambda e: orc.fbp(e.reshape(len(idx), NDET), N, n_angles, idx).reshape(-1), len(idx) * NDET)
    gotT = columns(lambda e: orc.fbp_adj(e.reshape(N, N), n_angles, NDET, idx).reshape(-1), N * N)
    assert np.max(np.abs(got - F)) < 1e-12
    assert np.max(np.abs(gotT - F.T)) < 1e-12


@pytest.mark.parametrize("phi", [0.0, 0.3, 1.1, math.pi / 2, 2.5, 4.0, 5.9])
def test_rotation_and_transpose_match_closed_form(orc, phi):
    c, s = math.cos(phi), math.sin(phi)
    T = D.rotation_matrix(N, c, s)
    cs = np.array([[c, s]])
    rot = columns(lambda e: orc.rotate(e.reshape(N, N), cs)[0].reshape(-1), N * N)
    rotT = columns(lambda e: orc.rotate_adj(e.reshape(1, N, N), cs).reshape(-1), N * N)
    assert np.max(np.abs(rot - T)) < 1e-13
    assert np.max(np.abs(rotT - T.T)) < 1e-13


def test_rotation_adjoint_sums_over_copies(orc):
    phis = [0.2, 1.7, 3.3]
    cs = np.array([[math.cos(p), math.sin(p)] for p in phis])
    h = np.random.default_rng(0).standard_normal((3, N, N))
    want = sum(D.rotation_matrix(N, c, s).T @ h[i].reshape(-1) for i, (c, s) in enumerate(cs))
    assert np.max(np.abs(orc.rotate_adj(h, cs).reshape(-1) - want)) < 1e-12


@pytest.mark.parametrize("lam,mc", [(1.0, None), (0.0, None), (0.7, "sketch")])
def test_ei_loss_and_gradient_match_matrix_algebra(orc, lam, mc):
    n, n_angles, n_det = 8, 12, 13
    g = np.random.default_rng(5)
    x = g.uniform(0, 1, (n, n))
    y = g.uniform(0, 3, (n_angles, n_det))
    idx = np.array([1, 4, 6, 11], dtype=np.int32)
    mc_idx = idx if mc == "sketch" else None
    cs = np.array([[math.cos(p), math.sin(p)] for p in (0.4, 2.2, 5.0)])
    want_l, want_g = D.ei_loss_grad_dense(x, y, n_angles, idx, cs, lam, mc_idx)
    got_l, got_g = orc.ei_loss_grad(x, y, n_angles, idx, cs, lam, mc_idx)
    assert abs(got_l - want_l) <= 1e-12 * abs(want_l)
    assert np.max(np.abs(got_g - want_g)) <= 1e-12 * np.max(np.abs(want_g))

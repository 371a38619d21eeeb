"""Dense measurement-space sketches on the matrix cores (skei_sketch_rows /
skei_sketch_rows_T, S = G (x) I) against the FP64 oracle: relative max-norm
error <= 1e-5 for Gaussian and Rademacher G at the EI-step shape (90 x 360
mixes of 363-detector rows, 16 images), a ragged shape (tiles partly
filled), one-row and one-column G, and a 1440-angle scan; adjoint gaps
|<S y, r> - <y, S^T r>| / (||S y|| ||r||) <= 1e-6 (the sketches are signed); a 0/1 selector G gives bitwise the rows of the angle-subsampled
operator; the autograd backward is S^T; and the densely sketched MC
residual S (y - A x) with its gradient."""
import numpy as np
import pytest
import torch

from gpu_util import f32, host, relerr, to_dev
from paper_2411_05771_amd import synth

pytestmark = pytest.mark.gpu

SHAPES = [  # (m, n_rows, row_len, batch, kind)
    (90, 360, 363, 16, "gaussian"),
    (90, 360, 363, 16, "rademacher"),
    (7, 13, 50, 3, "gaussian"),
    (1, 60, 91, 2, "rademacher"),
    (45, 1, 70, 1, "gaussian"),
    (180, 1440, 1449, 1, "gaussian"),
]


@pytest.mark.parametrize("m,k,L,b,kind", SHAPES)
def test_sketch_rows_parity_and_adjoint(skei, orc, m, k, L, b, kind):
    G = f32(synth.dense_sketch_matrix(m, k, kind, 77))

    class _G:   # a DenseSketch without a geometry of that angle count
        pass
    ds = _G()
    ds.m, ds.dev = m, to_dev(G)
    ds.geom = type("g", (), {"device": ds.dev.device})()
    y = f32(np.random.default_rng(5).uniform(0, 1, (b, k, L)))
    r = f32(np.random.default_rng(6).uniform(0, 1, (b, m, L)))
    sy = host(skei.sketch_rows_(ds, to_dev(y)))
    st = host(skei.sketch_rows_T_(ds, to_dev(r)))
    e, et = relerr(sy, orc.sketch_rows(G, y)), relerr(st, orc.sketch_rows_T(G, r))
    # G has random signs, so <S y, r> is a random-sign sum ~sqrt(m k) smaller
    # than its terms even for nonnegative y, r: the gap is scaled by the
    # Cauchy-Schwarz bound ||S y|| ||r|| instead of |<S y, r>|
    lhs, rhs = float(np.vdot(sy, r)), float(np.vdot(y, st))
    gap = abs(lhs - rhs) / (np.linalg.norm(sy) * np.linalg.norm(r))
    print(f"\n[dense] m={m} k={k} L={L} b={b} {kind}: S {e:.2e} S^T {et:.2e} adjoint gap {gap:.1e}", flush=True)
    assert e <= 1e-5 and et <= 1e-5 and gap <= 1e-6


def test_selector_reproduces_angle_subsampling_bitwise(skei):
    n, na, nd = 64, 60, 91
    geom = skei.Geometry(n, na, nd)
    idx = synth.interleaved_sketch(na, 4, 1)
    G = np.zeros((idx.size, na))
    G[np.arange(idx.size), idx] = 1.0
    ds = skei.DenseSketch(geom, G)
    x = to_dev(np.stack([synth.ellipse_phantom(n, synth.SEED_PHANTOM + i) for i in range(2)]))
    dense = skei.radon_fwd_dense(x, geom, ds)
    sub = skei.radon_fwd_(geom, x, geom.sketch(idx))
    assert torch.equal(dense, sub)


def test_dense_mc_residual_and_autograd_against_oracle(skei, orc):
    n, na, nd, m = 128, 180, 182, 45
    geom = skei.Geometry(n, na, nd)
    G = f32(synth.dense_sketch_matrix(m, na, "gaussian", 3))
    ds = skei.DenseSketch(geom, G)
    xt = synth.ellipse_phantom(n, synth.SEED_PHANTOM + 9).astype(np.float64)[None]
    yc = orc.radon_fwd(xt, na, nd)
    y = f32(synth.add_relative_noise(yc, synth.std_noise(yc.shape, synth.SEED_NOISE + 9)))
    x0 = f32(orc.fbp(y, n, na))
    # loss = || S (y - A x) ||^2 and its gradient -2 A^T S^T S (y - A x)
    x = to_dev(x0).requires_grad_(True)
    r = skei.radon_resid_dense(x, to_dev(y), geom, ds)
    loss = (r.double() ** 2).sum()
    loss.backward()
    r_o = orc.sketch_rows(G, y) - orc.sketch_rows(G, orc.radon_fwd(x0, na, nd))
    g_o = -2.0 * orc.radon_adj(orc.sketch_rows_T(G, r_o), n, na)
    e_r, e_g = relerr(host(r), r_o), relerr(host(x.grad), g_o)
    e_l = abs(float(loss) - float(np.sum(r_o ** 2))) / float(np.sum(r_o ** 2))
    print(f"\n[dense] MC residual {e_r:.2e} loss {e_l:.2e} grad {e_g:.2e}", flush=True)
    assert e_r <= 1e-5 and e_l <= 1e-5 and e_g <= 1e-5

"""Pins of the oracle's dense measurement-space sketch S = G (x) I (Sec. 2.3:
Gaussian and Rademacher sketches) against things other than itself:
a 0/1 selector G reduces to angle subsampling (the row selection the paper's
interleaved sketches use); integer +-1 matrices on integer sinograms against
a brute-force triple loop (exact); the adjoint identity; and the sketch
generator's E[G^T G] = I (exact on the diagonal for Rademacher, Monte-Carlo
for Gaussian)."""
import numpy as np

import oracle
from paper_2411_05771_amd import synth


def test_selector_is_row_subsampling():
    rng = np.random.default_rng(1)
    y = rng.standard_normal((3, 12, 7))
    idx = np.array([4, 0, 9, 9])
    G = np.zeros((idx.size, 12))
    G[np.arange(idx.size), idx] = 1.0
    assert np.array_equal(oracle.sketch_rows(G, y), y[:, idx])
    r = rng.standard_normal((3, idx.size, 7))
    want = np.zeros_like(y)
    for i, a in enumerate(idx):
        want[:, a] += r[:, i]
    assert np.allclose(oracle.sketch_rows_T(G, r), want, rtol=0, atol=1e-15)


def test_integer_products_equal_brute_force():
    rng = np.random.default_rng(2)
    m, k, L, B = 3, 5, 4, 2
    G = rng.choice([-1.0, 1.0], size=(m, k))
    y = rng.integers(-9, 10, size=(B, k, L)).astype(np.float64)
    want = np.zeros((B, m, L))
    for b in range(B):
        for i in range(m):
            for c in range(L):
                s = 0.0
                for a in range(k):
                    s += G[i][a] * y[b][a][c]
                want[b][i][c] = s
    assert np.array_equal(oracle.sketch_rows(G, y), want)
    r = rng.integers(-9, 10, size=(B, m, L)).astype(np.float64)
    want_t = np.zeros((B, k, L))
    for b in range(B):
        for a in range(k):
            for c in range(L):
                want_t[b][a][c] = sum(G[i][a] * r[b][i][c] for i in range(m))
    assert np.array_equal(oracle.sketch_rows_T(G, r), want_t)


def test_adjoint_identity():
    rng = np.random.default_rng(3)
    G = synth.dense_sketch_matrix(9, 30, "gaussian", 11)
    y = rng.standard_normal((2, 30, 17))
    r = rng.standard_normal((2, 9, 17))
    lhs = np.vdot(oracle.sketch_rows(G, y), r)
    rhs = np.vdot(y, oracle.sketch_rows_T(G, r))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_generator_is_isotropic():
    # Rademacher: every column has unit norm exactly
    G = synth.dense_sketch_matrix(16, 40, "rademacher", 5)
    assert np.allclose(np.sum(G * G, axis=0), 1.0, rtol=0, atol=1e-15)
    assert set(np.unique(np.abs(G) * 4)) == {1.0}
    # Gaussian: the mean of G^T G over independent draws approaches I
    m, n, draws = 8, 6, 4000
    acc = np.zeros((n, n))
    for s in range(draws):
        G = synth.dense_sketch_matrix(m, n, "gaussian", 10000 + s)
        acc += G.T @ G
    acc /= draws
    # each entry's standard error is about sqrt(2/(m draws)) on the diagonal, sqrt(1/(m draws)) off it
    assert np.max(np.abs(acc - np.eye(n))) < 5 * np.sqrt(2.0 / (m * draws))

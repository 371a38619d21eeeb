"""skei_coil_pca, the host Hermitian Jacobi eigensolver behind the PCA coil
compression of Algorithm 3, against the FP64 oracle (numpy's eigh, with the
same phase convention) on random Hermitian and coil-covariance matrices up
to the 64-coil limit; plus the argument checks.  Host call: runs without a
GPU."""
import ctypes

import numpy as np
import pytest

from oracle import mri as omri
from paper_2411_05771_amd import capi


def pca(V, L):
    nc = V.shape[0]
    Vi = np.ascontiguousarray(np.stack([V.real, V.imag], axis=-1))
    Q = np.zeros((nc, L, 2))
    w = np.zeros(L)
    rc = capi.lib().skei_coil_pca(Vi.ctypes.data_as(ctypes.c_void_p), nc, L, Q.ctypes.data_as(ctypes.c_void_p),
                                  w.ctypes.data_as(ctypes.c_void_p))
    assert rc == 0
    return Q[..., 0] + 1j * Q[..., 1], w


@pytest.mark.parametrize("nc,L,seed", [(1, 1, 0), (2, 1, 1), (5, 3, 2), (15, 15, 3), (15, 8, 4), (32, 10, 5),
                                       (64, 64, 6)])
def test_matches_oracle_eigenvectors(hiplib, orc, nc, L, seed):
    rng = np.random.default_rng(seed)
    k = (rng.standard_normal((nc, 24, 24)) + 1j * rng.standard_normal((nc, 24, 24))) \
        * rng.uniform(0.2, 3.0, nc)[:, None, None]
    mix = rng.standard_normal((nc, nc)) + 1j * rng.standard_normal((nc, nc))
    k = np.einsum("ij,jpq->ipq", mix, k)     # correlated coils
    V = omri.coil_covariance(k)
    Q, w = pca(V, L)
    Qo, wo = omri.pca_coils(V, L)
    assert np.max(np.abs(w - wo)) <= 1e-12 * wo[0]
    # eigenvalue gaps of random matrices keep the eigenvectors well separated
    assert np.max(np.abs(Q - Qo)) < 1e-9, np.max(np.abs(Q - Qo))
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(L))) < 1e-12


def test_diagonal_and_degenerate_inputs(hiplib, orc):
    V = np.diag([1.0, 5.0, 3.0]).astype(complex)
    Q, w = pca(V, 3)
    assert np.allclose(w, [5.0, 3.0, 1.0])
    assert np.allclose(np.abs(Q), np.eye(3)[:, [1, 2, 0]])
    Z = np.zeros((4, 4), complex)   # all-zero covariance: any orthonormal basis, eigenvalues 0
    Q, w = pca(Z, 2)
    assert np.all(w == 0.0) and np.allclose(Q.conj().T @ Q, np.eye(2))


def test_rejects_bad_arguments(hiplib):
    V = np.eye(3, dtype=np.float64).repeat(2, axis=1)
    Q, w = np.zeros(18), np.zeros(3)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    assert capi.lib().skei_coil_pca(p(V), 3, 4, p(Q), p(w)) == -1
    assert capi.lib().skei_coil_pca(p(V), 3, 0, p(Q), p(w)) == -1
    assert capi.lib().skei_coil_pca(None, 3, 1, p(Q), p(w)) == -1
    assert capi.lib().skei_coil_pca(p(V), 65, 1, p(Q), p(w)) == -4

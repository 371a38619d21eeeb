"""Pins of the FP64 multicoil MRI oracle (Sec. 3.4, Eq. (e:mri), Algorithm 3)
to things other than itself:

- the DFT against the textbook sum, written as explicit loops on an 8 x 8
  grid (scaling and sign), Parseval, and a delta -> constant;
- A against a dense matrix assembled block by block from the definition
  M (I (x) F~) [diag(C_1); ...; diag(C_Nc)] on a 4 x 4, 3-coil case;
- the adjoint identity <A x, k> = <x, A^H k>;
- with every sample kept, A^H A = D (F~ unitary), so A^dagger A = I where the
  maps do not all vanish;
- the classical sketch equals coil selection, of the maps or of the data;
- PCA: the covariance against explicit per-entry sums, the eigen-relation,
  orthonormality, the phase convention, a rank-one closed form (coils
  a_i s: top eigenvector conj(a) / ||a||, eigenvalue ||a||^2 var(s)), and the
  compressed coils' covariance diag(eigenvalues);
- compression commutes with the forward model (virtual maps), and the coil
  sketch with R = L is the identity;
- the EI loss and gradient against central finite differences along random
  real and imaginary directions, the gradient's MC part against the plain
  -2 A^H (y - A x), and the EI term vanishing with a full mask."""
import numpy as np
import pytest

from oracle import mri, oracle

pytestmark = pytest.mark.usefixtures("orc")


def crand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_dft_is_the_textbook_sum():
    rng = np.random.default_rng(1)
    n = 8
    z = crand(rng, n, n)
    ref = np.zeros((n, n), complex)
    for u in range(n):
        for v in range(n):
            s = 0j
            for p in range(n):
                for q in range(n):
                    s += z[p, q] * np.exp(-2j * np.pi * (u * p + v * q) / n)
            ref[u, v] = s / n
    assert np.max(np.abs(mri.dft2(z) - ref)) < 1e-12
    assert abs(np.linalg.norm(mri.dft2(z)) - np.linalg.norm(z)) < 1e-12
    assert np.max(np.abs(mri.idft2(mri.dft2(z)) - z)) < 1e-12
    d = np.zeros((n, n))
    d[0, 0] = 1.0
    assert np.max(np.abs(mri.dft2(d) - 1.0 / n)) < 1e-15


def dense_A(maps, mask):
    nc, n, _ = maps.shape
    d = n * n
    W = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n) / np.sqrt(n)
    F1 = np.kron(W, W)                       # row-major vec of W z W^T
    A = np.zeros((nc * d, d), complex)
    for c in range(nc):
        A[c * d:(c + 1) * d] = np.diag(mask.ravel()) @ F1 @ np.diag(maps[c].ravel())
    return A


def test_forward_and_adjoint_match_the_dense_definition():
    rng = np.random.default_rng(2)
    nc, n = 3, 4
    maps = crand(rng, nc, n, n)
    mask = (rng.uniform(size=(n, n)) < 0.5).astype(float)
    A = dense_A(maps, mask)
    x = crand(rng, 2, n, n)
    k = mri.mri_fwd(x, maps, mask)
    for b in range(2):
        assert np.max(np.abs(k[b].ravel() - A @ x[b].ravel())) < 1e-12
    kk = crand(rng, 2, nc, n, n)
    xa = mri.mri_adj(kk, maps, mask)
    for b in range(2):
        assert np.max(np.abs(xa[b].ravel() - A.conj().T @ kk[b].ravel())) < 1e-12


def test_adjoint_identity_and_full_mask_inverse():
    rng = np.random.default_rng(3)
    nc, n = 4, 16
    maps = crand(rng, nc, n, n)
    mask = (rng.uniform(size=(n, n)) < 0.3).astype(float)
    x, k = crand(rng, 1, n, n), crand(rng, 1, nc, n, n)
    lhs = np.vdot(mri.mri_fwd(x, maps, mask), k)
    rhs = np.vdot(x, mri.mri_adj(k, maps, mask))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    full = np.ones((n, n))
    assert np.max(np.abs(mri.mri_pinv(mri.mri_fwd(x, maps, full), maps, full) - x)) < 1e-12
    D = np.sum(np.abs(maps) ** 2, axis=0)
    assert np.max(np.abs(mri.mri_adj(mri.mri_fwd(x, maps, full), maps, full) - D * x)) < 1e-11


def test_classical_sketch_is_coil_selection():
    rng = np.random.default_rng(4)
    nc, n = 6, 8
    maps = crand(rng, nc, n, n)
    mask = (rng.uniform(size=(n, n)) < 0.5).astype(float)
    x = crand(rng, 2, n, n)
    coils = [4, 1, 5]
    G = mri.selection_matrix(coils, nc)
    assert np.array_equal(G.sum(axis=1), np.ones(3))
    k = mri.mri_fwd(x, maps, mask)
    assert np.array_equal(mri.coil_mix(G, k), k[:, coils])
    assert np.max(np.abs(mri.mri_fwd(x, mri.coil_mix(G, maps), mask) - k[:, coils])) < 1e-13


def test_covariance_entries_and_pca():
    rng = np.random.default_rng(5)
    nc, n = 5, 6
    k = crand(rng, nc, n, n) * np.arange(1, nc + 1)[:, None, None]
    V = mri.coil_covariance(k)
    d = n * n
    for i in range(nc):
        for j in range(nc):
            mi, mj = k[i].sum() / d, k[j].sum() / d
            s = 0j
            for p in range(n):
                for q in range(n):
                    s += np.conj(k[i, p, q] - mi) * (k[j, p, q] - mj)
            assert abs(V[i, j] - s / (d - 1)) < 1e-12 * abs(s)
    assert np.max(np.abs(V - V.conj().T)) < 1e-13
    Q, w = mri.pca_coils(V, 3)
    assert np.all(np.diff(w) <= 0)
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(3))) < 1e-12
    assert np.max(np.abs(V @ Q - Q * w)) < 1e-10 * w[0]
    for j in range(3):
        i = int(np.argmax(np.abs(Q[:, j])))
        assert abs(Q[i, j].imag) < 1e-15 and Q[i, j].real > 0
    # the compressed coils are uncorrelated with variances w
    kt = mri.coil_mix(Q.T, k)
    assert np.max(np.abs(mri.coil_covariance(kt) - np.diag(w))) < 1e-10 * w[0]


def test_pca_rank_one_closed_form():
    rng = np.random.default_rng(6)
    nc, n = 4, 8
    a = crand(rng, nc)
    s = crand(rng, n, n)
    k = a[:, None, None] * s[None]
    V = mri.coil_covariance(k)
    Q, w = mri.pca_coils(V, 1)
    sb = s.ravel() - s.mean()
    var = np.vdot(sb, sb).real / (n * n - 1)
    assert abs(w[0] - np.vdot(a, a).real * var) < 1e-12 * w[0]
    q = np.conj(a) / np.linalg.norm(a)
    i = int(np.argmax(np.abs(q)))
    q = q * np.conj(q[i]) / abs(q[i])
    assert np.max(np.abs(Q[:, 0] - q)) < 1e-12


def test_compression_commutes_and_identity_sketch():
    rng = np.random.default_rng(7)
    nc, n, L = 6, 8, 4
    maps = crand(rng, nc, n, n)
    mask = (rng.uniform(size=(n, n)) < 0.5).astype(float)
    x = crand(rng, 1, n, n)
    k = mri.mri_fwd(x, maps, mask)
    Q, _ = mri.pca_coils(mri.coil_covariance(k[0]), L)
    virt = mri.coil_mix(Q.T, maps)
    assert np.max(np.abs(mri.coil_mix(Q.T, k) - mri.mri_fwd(x, virt, mask))) < 1e-12
    S = mri.coil_sketch_matrix(L, L, np.zeros((0, 0)))
    assert np.array_equal(S, np.eye(L))
    S2 = mri.coil_sketch_matrix(L, 2, np.array([[1.0, -1.0], [-1.0, -1.0], [1.0, 1.0]]))
    assert S2.shape == (5, 4) and np.array_equal(S2[:2, :2], np.eye(2)) and not S2[:2, 2:].any()


def test_ei_loss_and_gradient():
    rng = np.random.default_rng(8)
    nc, n, C = 3, 8, 2
    maps = crand(rng, nc, n, n) * 0.5
    mask = (rng.uniform(size=(n, n)) < 0.5).astype(float)
    x = crand(rng, 1, n, n)
    y = mri.mri_fwd(crand(rng, 1, n, n), maps, mask)
    phi = np.array([0.3, 1.9])
    cs = np.stack([np.cos(phi), np.sin(phi)], axis=1)
    loss, g = mri.mri_ei_loss_grad(x, y, maps, mask, cs, lam=0.7)
    for t in range(6):
        dx = crand(rng, 1, n, n) if t % 2 else rng.standard_normal((1, n, n)) * 1j
        h = 1e-6
        lp, _ = mri.mri_ei_loss_grad(x + h * dx, y, maps, mask, cs, lam=0.7)
        lm, _ = mri.mri_ei_loss_grad(x - h * dx, y, maps, mask, cs, lam=0.7)
        fd = (lp - lm) / (2 * h)
        an = float(np.sum(g.real * dx.real + g.imag * dx.imag))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (t, fd, an)
    l0, g0 = mri.mri_ei_loss_grad(x, y, maps, mask, cs, lam=0.0)
    r = y - mri.mri_fwd(x, maps, mask)
    assert abs(l0 - np.sum(np.abs(r) ** 2)) < 1e-10 * l0
    assert np.max(np.abs(g0 + 2 * mri.mri_adj(r, maps, mask))) < 1e-10
    full = np.ones((n, n))
    yf = mri.mri_fwd(x, maps, full)
    lf, _ = mri.mri_ei_loss_grad(x, yf, maps, full, cs, lam=1.0)
    assert lf < 1e-20   # A x = y and P = I: both terms vanish


def test_rotation_of_complex_images_is_per_part():
    rng = np.random.default_rng(9)
    z = crand(rng, 8, 8)
    cs = np.array([[np.cos(0.4), np.sin(0.4)]])
    out = mri._rot(z, cs)
    assert np.array_equal(out.real, oracle.rotate(z.real, cs))
    assert np.array_equal(out.imag, oracle.rotate(z.imag, cs))

"""FP64 oracle of the multicoil MRI operator and its coil sketches (Sec. 3.4:
the forward model of Eq. (e:mri), the classical coil-subsampling sketch, PCA
coil compression and the coil sketch of Algorithm 3).

TEST INFRASTRUCTURE ONLY: imported by the tests and by the benchmark's
CPU-baseline leg, never by the product package.  Plain numpy in complex128;
the DFT and the Hermitian eigensolver are library primitives used as single
steps.

Conventions (the readings this oracle fixes):
- an image x is complex [B, N, N]; coil maps C are complex [Nc, N, N];
  k-space is complex [B, Nc, N, N]; the sampling mask M is a 0/1 array
  [N, N] (the diagonal of M), shared by every coil;
- the DFT F~ is the orthonormal 2-D DFT with no shift,
      (F~ z)[u, v] = (1/N) sum_{p,q} z[p, q] exp(-2 pi i (u p + v q) / N);
- A x = M F (C x): k[b, c] = M * F~(C_c * x[b])                 (Eq. e:mri);
- A^H k = sum_c conj(C_c) * F~^H(M * k[b, c]);
- the pseudo-inverse used for A^dagger is the coil-weighted adjoint
  D^-1 A^H with D = sum_c |C_c|^2 pixelwise (the least-squares inverse of
  the coil stage; with M = I it is exact);
- coil sketches act on the coil index only: (S z)[r] = sum_l G[r, l] z[l]
  (S = G (x) I_d).  Classical: G selects Mc of the Nc coils.  Coil sketch:
  G = S_c = [[I_R, 0], [0, S_low]] on PCA virtual coils, S_low of +-1;
- PCA: each coil's k-space is centred over its d = N^2 samples,
  V[i, j] = kbar_i^H kbar_j / (d - 1); Q_L holds the L dominant
  eigenvectors, each scaled so that its entry of largest modulus (the first
  such) is real and positive; virtual coils k~ = k Q_L, and, the maps being
  known, the virtual maps are the same combination C~_l = sum_i Q[i, l] C_i
  (by linearity of Eq. (e:mri) in the coil index).
"""
from __future__ import annotations

import numpy as np

from . import oracle

__all__ = [
    "dft2", "idft2", "mri_fwd", "mri_adj", "coil_weights", "mri_pinv", "selection_matrix", "coil_mix",
    "coil_covariance", "pca_coils", "coil_sketch_matrix", "mri_ei_loss_grad",
]


def _c(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def dft2(z):
    """Orthonormal 2-D DFT over the last two axes."""
    return np.fft.fft2(_c(z), norm="ortho")


def idft2(z):
    """Inverse (= adjoint) of dft2."""
    return np.fft.ifft2(_c(z), norm="ortho")


def mri_fwd(x, maps, mask):
    """k[b, c] = M * F~(C_c x[b])  (Eq. e:mri).  x [B,N,N] -> [B,Nc,N,N]."""
    x, maps = _c(x), _c(maps)
    return np.asarray(mask, dtype=np.float64) * dft2(maps[None] * x[:, None])


def mri_adj(k, maps, mask):
    """A^H k = sum_c conj(C_c) F~^H (M k[b, c]).  [B,Nc,N,N] -> [B,N,N]."""
    k, maps = _c(k), _c(maps)
    return np.sum(np.conj(maps)[None] * idft2(np.asarray(mask, dtype=np.float64) * k), axis=1)


def coil_weights(maps):
    """1 / sum_c |C_c|^2 pixelwise (0 where every map vanishes)."""
    d = np.sum(np.abs(_c(maps)) ** 2, axis=0)
    out = np.zeros_like(d)
    np.divide(1.0, d, out=out, where=d > 0)
    return out


def mri_pinv(k, maps, mask):
    """A^dagger k = D^-1 A^H k (coil-weighted zero-filled inverse)."""
    return coil_weights(maps)[None] * mri_adj(k, maps, mask)


def selection_matrix(coils, nc):
    """The classical coil-subsampling sketch's coil matrix: row r selects
    coil coils[r] (one identity block per row block)."""
    coils = np.asarray(coils, dtype=np.int64)
    G = np.zeros((coils.size, nc))
    G[np.arange(coils.size), coils] = 1.0
    return G


def coil_mix(G, z):
    """out[..., r, :, :] = sum_l G[r, l] z[..., l, :, :]  (S = G (x) I_d)."""
    G, z = _c(G), _c(z)
    return np.einsum("rl,...lpq->...rpq", G, z)


def coil_covariance(k):
    """V[i, j] = kbar_i^H kbar_j / (d - 1) for one measurement k [Nc, N, N],
    each coil centred over its d samples (Algorithm 3, first steps)."""
    k = _c(k).reshape(k.shape[0], -1)
    d = k.shape[1]
    kb = k - k.mean(axis=1, keepdims=True)
    return np.conj(kb) @ kb.T / (d - 1)


def pca_coils(V, L):
    """The L dominant eigenvectors of the Hermitian V as columns of Q [Nc, L]
    (descending eigenvalues), each with its largest-modulus entry real and
    positive, and the L eigenvalues."""
    w, Q = np.linalg.eigh(_c(V))
    order = np.argsort(w)[::-1][:L]
    w, Q = w[order], Q[:, order]
    for j in range(L):
        i = int(np.argmax(np.abs(Q[:, j])))
        Q[:, j] *= np.conj(Q[i, j]) / np.abs(Q[i, j])
    return Q, w


def coil_sketch_matrix(L, R, signs):
    """S_c = [[I_R, 0], [0, S_low]] with S_low = signs, [Mc - R, L - R] of +-1."""
    signs = np.asarray(signs, dtype=np.float64)
    mc = R + signs.shape[0]
    if signs.shape[1] != L - R:
        raise ValueError("S_low must have L - R columns")
    S = np.zeros((mc, L))
    S[:R, :R] = np.eye(R)
    S[R:, R:] = signs
    return S


def _rot(z, cos_sin):
    """T_c z for complex z [N,N]: the bilinear rotation of the real and the
    imaginary parts; -> [C,N,N]."""
    return oracle.rotate(z.real, cos_sin) + 1j * oracle.rotate(z.imag, cos_sin)


def _rot_adj(h, cos_sin):
    return oracle.rotate_adj(h.real, cos_sin) + 1j * oracle.rotate_adj(h.imag, cos_sin)


def mri_ei_loss_grad(x, y, maps, mask, cos_sin, lam=1.0):
    """Sketched EI loss of Algorithm 3 with the network taken as the
    identity, and its gradient with respect to the real and imaginary parts
    of the image (returned as one complex array, d/dRe + i d/dIm):

        L = sum_b ( ||y_b - A x_b||^2 + (lam / C) sum_c ||T_c x_b - P T_c x_b||^2 ),
        P = A^dagger A = D^-1 A^H A,

    A = M F C with the (sketched) maps given and y the (sketched) k-space.
    x [B,N,N] complex; y [B,Nc,N,N]; cos_sin [C,2]."""
    x, y = _c(x), _c(y)
    cs = np.asarray(cos_sin, dtype=np.float64).reshape(-1, 2)
    C = cs.shape[0]
    w = coil_weights(maps)
    loss, grad = 0.0, np.zeros_like(x)
    for b in range(x.shape[0]):
        r_mc = y[b] - mri_fwd(x[b][None], maps, mask)[0]
        g = -2.0 * mri_adj(r_mc[None], maps, mask)[0]
        loss += float(np.sum(np.abs(r_mc) ** 2))
        z = _rot(x[b], cs)                                       # [C,N,N]
        Pz = w[None] * mri_adj(mri_fwd(z, maps, mask), maps, mask)
        r = z - Pz
        loss += lam / C * float(np.sum(np.abs(r) ** 2))
        # d||r||^2 = 2 Re<r, (I - P) dz>: the gradient in z is 2 (I - P)^H r,
        # with P^H = A^H A D^-1 (D real)
        gz = 2.0 * (r - mri_adj(mri_fwd(w[None] * r, maps, mask), maps, mask))
        g += lam / C * _rot_adj(gz, cs)
        grad[b] = g
    return loss, grad

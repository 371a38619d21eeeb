/*
 * skei_mri.h -- C ABI of the multicoil MRI operator and its coil sketches
 * (Xu, Li, Tang, arXiv 2411.05771, Sec. 3.4 and Algorithm 3), part of the
 * same library as skei_ct.h and sharing its error codes.
 *
 *   A x   = M F (C x)                       the forward model of Eq. (e:mri)
 *   A^H k = sum_c conj(C_c) F~^H (M k_c)    its adjoint
 *   D^-1 A^H k, D = sum_c |C_c|^2           the coil-weighted pseudo-inverse
 *                                           used for A^dagger
 *   (S z)_r = sum_l G[r][l] z_l             a sketch acting on the coil index
 *                                           (S = G (x) I_d): coil selection
 *                                           (the classical sketch), the PCA
 *                                           compression k Q_L and the coil
 *                                           sketch S_c = [I_R 0; 0 S_low]
 *   V, Q_L                                  the coil covariance and its
 *                                           dominant eigenvectors (PCA coil
 *                                           compression of Algorithm 3)
 *
 * Conventions.  Complex values are interleaved float pairs (re, im), the
 * layout of torch.complex64.  An image x is [B][N][N]; coil maps C are
 * [Nc][N][N]; k-space is [B][Nc][N][N]; the mask M (the diagonal of the
 * sampling operator, usually 0/1) is a real [N][N] array shared by the coils
 * and images.  F~ is the orthonormal 2-D DFT with no shift:
 *   (F~ z)[u][v] = (1/N) sum_{p,q} z[p][q] exp(-2 pi i (u p + v q) / N).
 * N is a power of two, 4 <= N <= SKEI_MRI_MAX_N.  Device pointers unless
 * stated; `stream` is a hipStream_t (NULL = the default stream); every call
 * is asynchronous on it.  Errors: SKEI_EINVAL (null pointer, size < 1, N not
 * a power of two in range), SKEI_ERANGE (grid or sizes out of range),
 * SKEI_ELAUNCH (the launch failed); nothing is enqueued on an error found
 * before the first launch.  Results are deterministic: every sum runs in a
 * fixed order.
 */
#ifndef SKEI_MRI_H
#define SKEI_MRI_H

#include <stddef.h>

#include "skei_ct.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SKEI_MRI_MAX_N 1024

/* k = M F~(C W x) for every image and coil (Eq. e:mri; W = I when
 * `weights` is NULL, else the real [n][n] pixel weights -- A W is the
 * transpose of the weighted adjoint below).  maps [nc][n][n] complex, x
 * [batch][n][n] complex, mask [n][n] real, k [batch][nc][n][n] complex
 * (written; it also holds the row-transformed intermediate, so it must not
 * overlap x, maps or the weights). */
int skei_mri_fwd(const float *maps, int nc, int n, const float *x, int batch, const float *mask,
                 const float *weights, float *k, void *stream);

/* x = W sum_c conj(C_c) F~^H(M k_c): the adjoint A^H, or with `weights` (a
 * real [n][n] array, NULL = all ones) the weighted adjoint used for the
 * pseudo-inverse.  work: caller-owned device scratch of at least
 * skei_mri_work_bytes(nc, n, batch) bytes (overwritten; must not overlap k
 * or x).  k is not modified. */
int skei_mri_adj(const float *maps, int nc, int n, const float *k, int batch, const float *mask,
                 const float *weights, float *x, float *work, void *stream);

/* Bytes of device scratch skei_mri_adj needs (batch * nc * n * n complex). */
size_t skei_mri_work_bytes(int nc, int n, int batch);

/* weights[p] = 1 / sum_c |C_c[p]|^2 (0 where every map vanishes; the sum in
 * double), the pixel weights of the pseudo-inverse D^-1 A^H. */
int skei_coil_weights(const float *maps, int nc, int n, float *weights, void *stream);

/* out[b][r][p] = sum_l G[r][l] z[b][l][p], G a complex [m_out][l_in] matrix
 * in device memory, z [batch][l_in][d] and out [batch][m_out][d] complex
 * (out must not overlap z).  Applies S = G (x) I_d to coil stacks of images,
 * maps or k-space: a 0/1 row-selection G is the classical coil-subsampling
 * sketch (bitwise coil selection), G = Q_L^T the PCA compression, G = S_c
 * the coil sketch.  1 <= m_out, l_in <= 1024. */
int skei_coil_mix(const float *G, int m_out, int l_in, const float *z, int batch, long long d, float *out,
                  void *stream);

/* V[i][j] = kbar_i^H kbar_j / (d - 1) for one measurement k [nc][d] complex,
 * each coil centred over its d samples, accumulated in double: the coil
 * covariance of Algorithm 3.  V is a device array of nc * nc complex
 * doubles (re, im).  2 <= d, 1 <= nc <= 64. */
int skei_coil_covariance(const float *k, int nc, long long d, double *V, void *stream);

/* HOST call (host pointers, synchronous): the L dominant eigenvectors of the
 * Hermitian V [nc][nc] (complex doubles, as skei_coil_covariance writes it)
 * by cyclic Jacobi rotations, in descending eigenvalue order, as the columns
 * of Q [nc][L] (complex doubles, row-major), each scaled so that its entry
 * of largest modulus (the first such) is real and positive; w [L] receives
 * the eigenvalues.  1 <= L <= nc <= 64. */
int skei_coil_pca(const double *V, int nc, int L, double *Q, double *w);

#ifdef __cplusplus
}
#endif

#endif /* SKEI_MRI_H */

// C ABI of the multicoil MRI operator and coil sketches (include/skei_mri.h):
// argument checks, then the launches of k_mri.hip; the PCA eigensolver runs
// on the host.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "mri.h"

namespace {

using skei::mri_size_ok;
using cplx = std::complex<double>;

inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }
inline const float2 *C2(const float *p) { return reinterpret_cast<const float2 *>(p); }
inline float2 *C2(float *p) { return reinterpret_cast<float2 *>(p); }

int check_planes(int nc, int n, int batch)
{
    if (nc < 1 || batch < 1 || !mri_size_ok(n)) return SKEI_EINVAL;
    if ((long long)batch * nc * (n / std::min(n, std::max(1, 2048 / n))) > 0x7fffffffLL) return SKEI_ERANGE;
    return SKEI_OK;
}

// Cyclic Jacobi for a Hermitian matrix A (n x n, row-major, overwritten):
// each rotation first turns the pivot a_pq real by a phase on column and
// row q, then zeroes it with a real plane rotation.  On return the diagonal
// holds the eigenvalues and the columns of U the eigenvectors.
void hermitian_jacobi(std::vector<cplx> &A, int n, std::vector<cplx> &U)
{
    U.assign((size_t)n * n, cplx(0.0, 0.0));
    for (int i = 0; i < n; i++) U[(size_t)i * n + i] = 1.0;
    auto a = [&](int r, int c) -> cplx & { return A[(size_t)r * n + c]; };
    double scale = 0.0;
    for (const cplx &v : A) scale += std::norm(v);
    scale = std::sqrt(scale);
    for (int sweep = 0; sweep < 100; sweep++) {
        double off = 0.0;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) off += std::norm(a(p, q));
        if (std::sqrt(off) <= 1e-15 * scale || off == 0.0) break;
        for (int p = 0; p < n; p++) {
            for (int q = p + 1; q < n; q++) {
                const double h = std::abs(a(p, q));
                if (h == 0.0) continue;
                const cplx ph = a(p, q) / h;   // a_pq = h ph
                const double app = a(p, p).real(), aqq = a(q, q).real();
                const double tau = (aqq - app) / (2.0 * h);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                // G = diag(1, conj(ph)) [[c, s], [-s, c]] on columns p, q:
                //   col p <- c col p - s conj(ph) col q,  col q <- s col p + c conj(ph) col q
                const cplx gqp = -s * std::conj(ph), gqq = c * std::conj(ph);
                for (int r = 0; r < n; r++) {
                    const cplx xp = a(r, p), xq = a(r, q);
                    a(r, p) = c * xp + gqp * xq;
                    a(r, q) = s * xp + gqq * xq;
                    const cplx up = U[(size_t)r * n + p], uq = U[(size_t)r * n + q];
                    U[(size_t)r * n + p] = c * up + gqp * uq;
                    U[(size_t)r * n + q] = s * up + gqq * uq;
                }
                // rows: A <- G^H A
                for (int r = 0; r < n; r++) {
                    const cplx xp = a(p, r), xq = a(q, r);
                    a(p, r) = c * xp + std::conj(gqp) * xq;
                    a(q, r) = s * xp + std::conj(gqq) * xq;
                }
                a(p, q) = 0.0;
                a(q, p) = 0.0;
                a(p, p) = a(p, p).real();
                a(q, q) = a(q, q).real();
            }
        }
    }
}

}  // namespace

extern "C" {

int skei_mri_fwd(const float *maps, int nc, int n, const float *x, int batch, const float *mask,
                 const float *weights, float *k, void *stream)
{
    if (!maps || !x || !mask || !k) return SKEI_EINVAL;
    if (int rc = check_planes(nc, n, batch)) return rc;
    return skei::launch_mri_fwd(C2(maps), nc, n, C2(x), batch, mask, weights, C2(k), S(stream));
}

size_t skei_mri_work_bytes(int nc, int n, int batch)
{
    if (nc < 1 || n < 1 || batch < 1) return 0;
    return (size_t)batch * nc * n * n * sizeof(float2);
}

int skei_mri_adj(const float *maps, int nc, int n, const float *k, int batch, const float *mask,
                 const float *weights, float *x, float *work, void *stream)
{
    if (!maps || !k || !mask || !x || !work) return SKEI_EINVAL;
    if (int rc = check_planes(nc, n, batch)) return rc;
    return skei::launch_mri_adj(C2(maps), nc, n, C2(k), batch, mask, weights, C2(x), C2(work), S(stream));
}

int skei_coil_weights(const float *maps, int nc, int n, float *weights, void *stream)
{
    if (!maps || !weights || nc < 1 || n < 1) return SKEI_EINVAL;
    return skei::launch_coil_weights(C2(maps), nc, (long long)n * n, weights, S(stream));
}

int skei_coil_mix(const float *G, int m_out, int l_in, const float *z, int batch, long long d, float *out,
                  void *stream)
{
    if (!G || !z || !out || m_out < 1 || l_in < 1 || batch < 1 || d < 1) return SKEI_EINVAL;
    if (m_out > 1024 || l_in > 1024) return SKEI_ERANGE;
    return skei::launch_coil_mix(C2(G), m_out, l_in, C2(z), d, batch, C2(out), S(stream));
}

int skei_coil_covariance(const float *k, int nc, long long d, double *V, void *stream)
{
    if (!k || !V || nc < 1 || d < 2) return SKEI_EINVAL;
    if (nc > 64) return SKEI_ERANGE;
    return skei::launch_coil_cov(C2(k), nc, d, V, S(stream));
}

int skei_coil_pca(const double *V, int nc, int L, double *Q, double *w)
{
    if (!V || !Q || !w || nc < 1 || L < 1 || L > nc) return SKEI_EINVAL;
    if (nc > 64) return SKEI_ERANGE;
    std::vector<cplx> A((size_t)nc * nc), U;
    for (int i = 0; i < nc; i++)
        for (int j = 0; j < nc; j++) {
            // the Hermitian part (V is Hermitian up to rounding)
            const cplx vij(V[2 * ((size_t)i * nc + j)], V[2 * ((size_t)i * nc + j) + 1]);
            const cplx vji(V[2 * ((size_t)j * nc + i)], V[2 * ((size_t)j * nc + i) + 1]);
            A[(size_t)i * nc + j] = 0.5 * (vij + std::conj(vji));
        }
    hermitian_jacobi(A, nc, U);
    std::vector<int> order(nc);
    for (int i = 0; i < nc; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return A[(size_t)a * nc + a].real() > A[(size_t)b * nc + b].real();
    });
    for (int j = 0; j < L; j++) {
        const int e = order[j];
        w[j] = A[(size_t)e * nc + e].real();
        int imax = 0;
        for (int i = 1; i < nc; i++)
            if (std::abs(U[(size_t)i * nc + e]) > std::abs(U[(size_t)imax * nc + e])) imax = i;
        const cplx um = U[(size_t)imax * nc + e];
        const cplx ph = std::abs(um) > 0.0 ? std::conj(um) / std::abs(um) : cplx(1.0, 0.0);
        for (int i = 0; i < nc; i++) {
            cplx v = U[(size_t)i * nc + e] * ph;
            if (i == imax) v = cplx(std::abs(um), 0.0);
            Q[2 * ((size_t)i * L + j)] = v.real();
            Q[2 * ((size_t)i * L + j) + 1] = v.imag();
        }
    }
    return SKEI_OK;
}

}  // extern "C"

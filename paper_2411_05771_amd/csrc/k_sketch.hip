// Dense measurement-space sketches of CT sinograms (the Gaussian and
// Rademacher sketches S of Sec. 2.3 and of the proof of Theorem 1, applied to
// whole projections): with S = G (x) I_{N_det} for a dense G in R^{m x N_theta},
//     S y   : out[b][i][c] = sum_a G[i][a] y[b][a][c]      (m x N_det per image)
//     S^T r : out[b][a][c] = sum_i G[i][a] r[b][i][c]      (N_theta x N_det)
// Both are a batch of dense products C = L Y with the same left matrix, so
// they run on the matrix cores: v_mfma_f32_16x16x4f32 (FP32 in, FP32
// accumulate).  Lane layout on gfx950 (measured): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and holds D[4 (l / 16) + r][l % 16]
// in accumulator register r.
//
// A workgroup of four waves owns a 64 x 64 tile of one image's output (each
// wave a 16-row strip) or, when that gives too few workgroups to fill the
// chip, a 32 x 32 tile (each wave a 16 x 16 quarter).  K runs in chunks of
// 32: both operand tiles are staged in LDS (zero-filled past the edges), the
// next chunk's loads in flight while the waves issue the current one's MFMAs.  The left matrix is read
// through strides (G row-major for S, its transpose for S^T).
#include "skei_internal.h"

namespace skei {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kKc = 32;   // K per LDS chunk

// TM x TN output tile per workgroup of four waves.  STRIPS: wave w owns rows
// 16w .. 16w + 15 across the tile (TM = 64), one left fragment feeding TN/16
// MFMA blocks per k-step; otherwise the waves are arranged 2 x 2, each owning
// a (TM/2) x (TN/2) quarter.
template <int TM, int TN, bool STRIPS>
__global__ void __launch_bounds__(256) k_sketch_rows(const float *__restrict__ G, long long g_row, long long g_col,
                                                      const float *__restrict__ Y, float *__restrict__ out, int M,
                                                      int K, int L)
{
    static_assert(!STRIPS || TM == 64, "strips are 16 rows per wave");
    constexpr int BR = STRIPS ? 1 : TM / 32, BC = STRIPS ? TN / 16 : TN / 32;   // 16 x 16 blocks per wave
    __shared__ float As[TM][kKc + 1];   // left tile: row r, k
    __shared__ float Bs[kKc][TN + 1];   // right tile: k, column c
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = STRIPS ? 16 * w : (w >> 1) * (TM / 2), wc = STRIPS ? 0 : (w & 1) * (TN / 2);
    const int c0 = blockIdx.x * TN, r0 = blockIdx.y * TM, b = blockIdx.z;
    const float *Yb = Y + (size_t)b * K * L;
    f4 acc[BR][BC];
#pragma unroll
    for (int i = 0; i < BR; i++)
#pragma unroll
        for (int j = 0; j < BC; j++) acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};

    // Chunk k0's operands are loaded into registers while chunk k0 - kKc is
    // multiplied out of LDS, then stored to LDS behind a barrier.  Left
    // elements are assigned so that consecutive threads read consecutive
    // addresses of G (along k for S, along r for S^T).
    constexpr int NA = TM * kKc / 256, NB = kKc * TN / 256;
    const bool a_along_k = g_col == 1;
    float ra[NA], rb[NB];
    auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < NA; i++) {
            const int e = tid + 256 * i;
            const int r = a_along_k ? e / kKc : e % TM, k = a_along_k ? e % kKc : e / TM;
            const int gr = r0 + r, gk = k0 + k;
            ra[i] = (gr < M && gk < K) ? G[gr * g_row + gk * g_col] : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < NB; i++) {
            const int e = tid + 256 * i;
            const int k = e / TN, c = e % TN;
            const int gk = k0 + k, gc = c0 + c;
            rb[i] = (gk < K && gc < L) ? Yb[(size_t)gk * L + gc] : 0.0f;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int i = 0; i < NA; i++) {
            const int e = tid + 256 * i;
            const int r = a_along_k ? e / kKc : e % TM, k = a_along_k ? e % kKc : e / TM;
            As[r][k] = ra[i];
        }
#pragma unroll
        for (int i = 0; i < NB; i++) {
            const int e = tid + 256 * i;
            Bs[e / TN][e % TN] = rb[i];
        }
    };
    load(0);
    store();
    __syncthreads();
    for (int k0 = 0; k0 < K; k0 += kKc) {
        const bool more = k0 + kKc < K;
        if (more) load(k0 + kKc);
#pragma unroll
        for (int kk = 0; kk < kKc; kk += 4) {
            float a[BR];
#pragma unroll
            for (int i = 0; i < BR; i++) a[i] = As[wr + 16 * i + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < BC; j++) {
                const float bv = Bs[kk + (lane >> 4)][wc + 16 * j + (lane & 15)];
#pragma unroll
                for (int i = 0; i < BR; i++)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], bv, acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
        if (more) {
            store();
            __syncthreads();
        }
    }
    float *ob = out + (size_t)b * M * L;
#pragma unroll
    for (int i = 0; i < BR; i++)
#pragma unroll
        for (int j = 0; j < BC; j++) {
            const int gc = c0 + wc + 16 * j + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int gr = r0 + wr + 16 * i + 4 * (lane >> 4) + r;
                if (gr < M && gc < L) ob[(size_t)gr * L + gc] = acc[i][j][r];
            }
        }
}

}  // namespace

int launch_sketch_rows(const float *G, int m, int n_rows, const float *y, int batch, int row_len, bool transpose,
                       float *out, hipStream_t st)
{
    // S y: left = G (m x n_rows), K = n_rows, output rows m.
    // S^T r: left = G^T (n_rows x m), K = m, output rows n_rows.
    const int M = transpose ? n_rows : m, K = transpose ? m : n_rows;
    const long long g_row = transpose ? 1 : n_rows, g_col = transpose ? n_rows : 1;
    // 64 x 64 tiles in strips when they give the chip at least two workgroups
    // per CU, 32 x 32 quarters otherwise (measured on MI355X, S^T of 16
    // sinograms with 360 angles and 363 detectors from m = 90: 19.3 us in
    // strips against 23.4 us in quarters)
    const long long big = (long long)((row_len + 63) / 64) * ((M + 63) / 64) * batch;
    if (big >= 512) {
        const dim3 grid((unsigned)((row_len + 63) / 64), (unsigned)((M + 63) / 64), (unsigned)batch);
        hipLaunchKernelGGL((k_sketch_rows<64, 64, true>), grid, dim3(256), 0, st, G, g_row, g_col, y, out, M, K,
                           row_len);
    } else {
        const dim3 grid((unsigned)((row_len + 31) / 32), (unsigned)((M + 31) / 32), (unsigned)batch);
        hipLaunchKernelGGL((k_sketch_rows<32, 32, false>), grid, dim3(256), 0, st, G, g_row, g_col, y, out, M, K,
                           row_len);
    }
    return check_launch();
}

}  // namespace skei

// Ram-Lak ramp filter along detector rows (FBP's filtering step; Kak & Slaney
// ch. 3 with unit detector spacing), as a linear convolution with zero padding.
//
// Written in the symmetric form  q[k] = h(0) p[k] + sum_e h(2e+1) (p[k-2e-1] + p[k+2e+1]):
// the even taps are zero, and the odd taps h(2e+1) = -1/(pi (2e+1))^2 are the
// same for every lane at a given e (a scalar load), so each lane does two
// conflict-free LDS reads, one add and one double-precision FMA per pair of
// taps.  Accumulating in double removes the cancellation error of the
// high-pass sum (terms of size ~p, result of size ~p/N).
#include "skei_internal.h"

namespace skei {
namespace {

template <int RPT, typename IN>
__global__ void __launch_bounds__(256) k_ramp(const IN *__restrict__ p, int n_det,
                                              const double *__restrict__ hodd, float scale,
                                              float *__restrict__ q)
{
    extern __shared__ __align__(16) unsigned char ramp_raw[];
    IN *row = reinterpret_cast<IN *>(ramp_raw);   // [pad | n_det values | pad], pad = n_det + 1
    const int pad = n_det + 1;
    const int r = blockIdx.x;
    const int tid = threadIdx.x, bs = blockDim.x;
    const IN *src = p + (size_t)r * n_det;
    for (int e = tid; e < 3 * n_det + 2; e += bs) {
        const int j = e - pad;
        row[e] = (j >= 0 && j < n_det) ? src[j] : (IN)0;
    }
    __syncthreads();

    double acc[RPT];
#pragma unroll
    for (int i = 0; i < RPT; i++) {
        const int k = tid + i * bs;
        acc[i] = (k < n_det) ? 0.25 * (double)row[pad + k] : 0.0;
    }
    const int E = (n_det + 1) / 2;              // offsets 1, 3, ..., 2E-1 >= n_det - 1
    for (int e = 0; e < E; e++) {
        const double h = hodd[e];
        const int d = 2 * e + 1;
#pragma unroll
        for (int i = 0; i < RPT; i++) {
            const int k = min(tid + i * bs, n_det - 1);
            const double pair = (double)row[pad + k - d] + (double)row[pad + k + d];
            acc[i] = fma(h, pair, acc[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < RPT; i++) {
        const int k = tid + i * bs;
        if (k < n_det) q[(size_t)r * n_det + k] = (float)(acc[i] * (double)scale);
    }
}

template <typename IN>
int ramp_launch(const skei_geom *g, const IN *p, int rows, float scale, float *q, hipStream_t st)
{
    const int n_det = g->n_det;
    const int rpt = (n_det + 255) / 256;
    const int per = (n_det + rpt - 1) / rpt;
    const int block = ((per + 63) / 64) * 64;
    const size_t shm = sizeof(IN) * (size_t)(3 * n_det + 2);
    if (shm > 64 * 1024) return SKEI_ERANGE;
    const dim3 grid(rows);
#define SKEI_RAMP_CASE(P)                                                                                  \
    case P:                                                                                                \
        hipLaunchKernelGGL((k_ramp<P, IN>), grid, dim3(block), shm, st, p, n_det, g->hodd, scale, q); \
        break;
    switch (rpt) {
        SKEI_RAMP_CASE(1)
        SKEI_RAMP_CASE(2)
        SKEI_RAMP_CASE(3)
        SKEI_RAMP_CASE(4)
        SKEI_RAMP_CASE(5)
        SKEI_RAMP_CASE(6)
        SKEI_RAMP_CASE(7)
        SKEI_RAMP_CASE(8)
    default: return SKEI_ERANGE;
    }
#undef SKEI_RAMP_CASE
    return check_launch();
}

}  // namespace

int launch_ramp(const skei_geom *g, const float *pf, const double *pd, int rows, float scale, float *q,
                hipStream_t st)
{
    return pd ? ramp_launch<double>(g, pd, rows, scale, q, st) : ramp_launch<float>(g, pf, rows, scale, q, st);
}

}  // namespace skei

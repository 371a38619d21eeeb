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
#include "work.h"

namespace skei {
namespace {

template <int RPT, typename IN>
__device__ __forceinline__ void ramp_item(const RampJob &J, long long r, IN *row)
{
    // row = [pad | n_det values | pad], pad = n_det + 1
    const int n_det = J.n_det;
    const int pad = n_det + 1;
    const int tid = threadIdx.x, bs = blockDim.x;
    const IN *src = static_cast<const IN *>(J.p) + (size_t)r * n_det;
    const double *__restrict__ hodd = J.hodd;
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
        if (k < n_det) J.q[(size_t)r * n_det + k] = (float)(acc[i] * (double)J.scale);
    }
}

template <int RPT, typename IN>
__global__ void __launch_bounds__(256) k_ramp(const JobList<RampJob> L)
{
    extern __shared__ __align__(16) unsigned char ramp_raw[];
    IN *row = reinterpret_cast<IN *>(ramp_raw);
    for_each_item(L, [&](const RampJob &J, long long r) { ramp_item<RPT, IN>(J, r, row); });
}

template <int RPT, typename IN>
int ramp_launch1(int block, size_t shm, const JobList<RampJob> &L, hipStream_t st)
{
    const long long grid = launch_grid(L, reinterpret_cast<const void *>(&k_ramp<RPT, IN>), block, shm);
    if (grid <= 0 || grid > 0x7fffffffLL) return SKEI_ERANGE;
    hipLaunchKernelGGL((k_ramp<RPT, IN>), dim3((unsigned)grid), dim3(block), shm, st, L);
    return check_launch();
}

template <typename IN>
int ramp_launch(int rpt, int block, size_t shm, const JobList<RampJob> &L, hipStream_t st)
{
    if (L.total <= 0) return SKEI_OK;
    if (block < 64 || block > 256 || block % 64 || shm > 64 * 1024) return SKEI_ERANGE;
    switch (rpt) {
    case 1: return ramp_launch1<1, IN>(block, shm, L, st);
    case 2: return ramp_launch1<2, IN>(block, shm, L, st);
    case 3: return ramp_launch1<3, IN>(block, shm, L, st);
    case 4: return ramp_launch1<4, IN>(block, shm, L, st);
    case 5: return ramp_launch1<5, IN>(block, shm, L, st);
    case 6: return ramp_launch1<6, IN>(block, shm, L, st);
    case 7: return ramp_launch1<7, IN>(block, shm, L, st);
    case 8: return ramp_launch1<8, IN>(block, shm, L, st);
    default: return SKEI_ERANGE;
    }
}

}  // namespace

void ramp_shape(int n_det, int &rpt, int &block)
{
    rpt = (n_det + 255) / 256;
    const int per = (n_det + rpt - 1) / rpt;
    block = ((per + 63) / 64) * 64;
}

size_t ramp_shm(int n_det, bool in_double)
{
    return (in_double ? sizeof(double) : sizeof(float)) * (size_t)(3 * n_det + 2);
}

RampJob make_ramp_job(const skei_geom *g, const void *p, long long rows, float scale, float *q)
{
    RampJob J{};
    J.p = p;
    J.q = q;
    J.hodd = g->hodd;
    J.n_det = g->n_det;
    J.scale = scale;
    J.items = rows;
    return J;
}

int ramp_run(bool in_double, int rpt, int block, size_t shm, const JobList<RampJob> &L, hipStream_t st)
{
    return in_double ? ramp_launch<double>(rpt, block, shm, L, st) : ramp_launch<float>(rpt, block, shm, L, st);
}

int launch_ramp(const skei_geom *g, const float *pf, const double *pd, long long rows, float scale, float *q,
                hipStream_t st)
{
    const bool dbl = pd != nullptr;
    const RampJob J = make_ramp_job(g, dbl ? (const void *)pd : (const void *)pf, rows, scale, q);
    int rpt, block;
    ramp_shape(g->n_det, rpt, block);
    return ramp_run(dbl, rpt, block, ramp_shm(g->n_det, dbl), inline_jobs(&J, 1), st);
}

}  // namespace skei

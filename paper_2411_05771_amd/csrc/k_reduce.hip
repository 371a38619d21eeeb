// Deterministic reductions for the EI loss: each block sums a fixed,
// contiguous slice in double precision and writes one partial; a single block
// then adds the partials in a fixed order.  Results do not depend on timing or
// on what else runs on the device.
#include "skei_internal.h"
#include "work.h"

namespace skei {
namespace {

constexpr int kRedBlock = 1024;
constexpr size_t kRedChunk = 4096;   // elements per partial

__device__ __forceinline__ double block_sum(double v, double *sh)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int tid = threadIdx.x;
    if ((tid & 63) == 0) sh[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (tid == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) s += sh[w];
    return s;   // valid in thread 0
}

__global__ void __launch_bounds__(kRedBlock) k_sumsq(const float *__restrict__ a, const float *__restrict__ b,
                                                     size_t len, double *__restrict__ partial)
{
    __shared__ double sh[kRedBlock / 64];
    const size_t begin = (size_t)blockIdx.x * kRedChunk;
    const size_t end = begin + kRedChunk < len ? begin + kRedChunk : len;
    double acc = 0.0;
    for (size_t i = begin + threadIdx.x; i < end; i += kRedBlock) {
        const double d = b ? (double)a[i] - (double)b[i] : (double)a[i];
        acc = fma(d, d, acc);
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// The same fixed order as the loss items of the ramp launch (fixed_order_loss).
__device__ __forceinline__ void reduce_item(const RedJob &J)
{
    fixed_order_loss(J.p0, J.n0, J.w0, J.p1, J.n1, J.w1, J.out);
}

__global__ void __launch_bounds__(kRedBlock) k_reduce2(const JobList<RedJob> L)
{
    for_each_item(L, [&](const RedJob &J, long long) { reduce_item(J); });
}

}  // namespace

size_t sumsq_partials(size_t len) { return (len + kRedChunk - 1) / kRedChunk; }

int launch_sumsq(const float *a, const float *b, size_t len, double *partial, hipStream_t st)
{
    const size_t blocks = sumsq_partials(len);
    if (blocks == 0 || blocks > 0x7fffffff) return SKEI_ERANGE;
    hipLaunchKernelGGL(k_sumsq, dim3((unsigned)blocks), dim3(kRedBlock), 0, st, a, b, len, partial);
    return check_launch();
}

int reduce_run(const JobList<RedJob> &L, hipStream_t st)
{
    if (L.total <= 0) return SKEI_OK;
    const long long grid = launch_grid(L, reinterpret_cast<const void *>(&k_reduce2), kRedBlock, 0);
    if (grid <= 0 || grid > 0x7fffffffLL) return SKEI_ERANGE;
    hipLaunchKernelGGL(k_reduce2, dim3((unsigned)grid), dim3(kRedBlock), 0, st, L);
    return check_launch();
}

int launch_reduce2(const double *p0, size_t n0, double w0, const double *p1, size_t n1, double w1, double *out,
                   hipStream_t st)
{
    RedJob J{};
    J.p0 = p0;
    J.p1 = p1;
    J.out = out;
    J.n0 = (long long)n0;
    J.n1 = (long long)n1;
    J.w0 = w0;
    J.w1 = w1;
    J.items = 1;
    return reduce_run(inline_jobs(&J, 1), st);
}

}  // namespace skei

// Device-side dispatch of a job list (see JobList in skei_internal.h): maps
// each workgroup to (job, item) pairs and calls the kernel's item body.
#pragma once

#include "skei_internal.h"

namespace skei {

typedef __attribute__((address_space(4))) const unsigned int cword_t;

// Reads a job from a device table into scalar registers (the table is
// read-only while kernels run; `at` is wave-uniform).
template <typename Job>
__device__ __forceinline__ Job load_job(const Job *table, int at)
{
    static_assert(sizeof(Job) % 4 == 0, "job size");
    Job j;
    const cword_t *src = (const cword_t *)(table + at);
    unsigned int *dst = reinterpret_cast<unsigned int *>(&j);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(Job) / 4); i++) dst[i] = src[i];
    return j;
}

__device__ __forceinline__ long long uniform64(long long v)
{
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(unsigned long long)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ long long load_ll(const long long *p, int at)
{
    const cword_t *w = (const cword_t *)(p + at);
    return (long long)(((unsigned long long)w[1] << 32) | w[0]);
}

// Index of the job owning global item g: the largest j with first[j] <= g.
__device__ __forceinline__ int find_job(const long long *first, int njobs, long long g)
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (load_ll(first, mid) <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Runs body(job, item) for the workgroup's item(s).  body must be executed by
// every thread of the workgroup (it may hold barriers) and must not assume
// anything about LDS contents on entry.
template <typename Job, typename Body>
__device__ __forceinline__ void for_each_item(const JobList<Job> &L, Body &&body)
{
    if (!L.jobs) {
        const int x = blockIdx.x % kXcds;
        const long long item = L.inl_xr[x] + blockIdx.x / kXcds;
        if (item >= L.inl_xr[x + 1]) return;
        if (L.ninl > 1 && item >= L.inl_first[1]) {
            body(L.inl[1], item - L.inl_first[1]);
        } else {
            body(L.inl[0], item);
        }
        return;
    }
    if (!L.wq) {
        const int x = blockIdx.x % kXcds;
        const long long g = load_ll(L.xr, x) + blockIdx.x / kXcds;
        if (g >= load_ll(L.xr, x + 1)) return;
        const int j = find_job(L.first, L.njobs, g);
        body(load_job(L.jobs, j), g - load_ll(L.first, j));
        return;
    }
    // Persistent: workgroup L lives on XCD x0 = L % 8 as the s-th (s = L / 8)
    // of its XCD's nbx workgroups.  It first runs its static share of its
    // XCD's range -- items s, s + nbx, s + 2 nbx, ... of the first
    // q = floor(span / nbx) * nbx items, no atomics -- then the range's
    // remainder and, after that, the other XCDs' remainders are handed out
    // one item per draw by per-XCD cursors.
    __shared__ long long s_item;
    const int x0 = blockIdx.x % kXcds;
    const long long nbx = gridDim.x / kXcds, slot = blockIdx.x / kXcds;
    // the cursors of the next launch of this stage start from zero
    if (blockIdx.x == 0 && threadIdx.x < kXcds)
        __hip_atomic_store(&L.wq_next->next[threadIdx.x], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    {
        const long long beg = load_ll(L.xr, x0), end = load_ll(L.xr, x0 + 1);
        const long long q = (end - beg) / nbx;
        for (long long k = 0; k < q; k++) {
            if (k > 0) __syncthreads();
            const long long g = beg + slot + k * nbx;
            const int j = find_job(L.first, L.njobs, g);
            body(load_job(L.jobs, j), g - load_ll(L.first, j));
        }
    }
    for (int qx = 0; qx < kXcds; qx++) {
        const int x = (x0 + qx) % kXcds;
        const long long xb = load_ll(L.xr, x), end = load_ll(L.xr, x + 1);
        const long long beg = xb + (end - xb) / nbx * nbx;   // the range's remainder
        if (beg >= end) continue;
        const unsigned span = (unsigned)(end - beg);
        for (;;) {
            __syncthreads();   // the previous item is done with s_item and with LDS
            if (threadIdx.x == 0) {
                // a plain load first: exhausted remainders are skipped without a
                // read-modify-write on their cursor
                const unsigned seen = __hip_atomic_load(&L.wq->next[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_item = seen >= span ? end : beg + (long long)atomicAdd(&L.wq->next[x], 1u);
            }
            __syncthreads();
            const long long g = uniform64(s_item);
            if (g >= end) break;
            const int j = find_job(L.first, L.njobs, g);
            body(load_job(L.jobs, j), g - load_ll(L.first, j));
        }
    }
}

// out = w0 * sum(p0[0..n0)) + w1 * sum(p1[0..n1)) (p1 may be null), by the
// first 256 threads of the workgroup (blockDim.x >= 256): thread-strided
// sums, a butterfly per wave, then the four wave sums in a fixed order -- the
// same order whatever kernel or block size runs it.  Every thread calls it.
__device__ __forceinline__ void fixed_order_loss(const double *p0, long long n0, double w0, const double *p1,
                                                 long long n1, double w1, double *out)
{
    __shared__ double wave_part[2][4];
    const int t = threadIdx.x;
    if (t < 256) {
        double a = 0.0, e = 0.0;
        for (long long i = t; i < n0; i += 256) a += p0[i];
        if (p1)
            for (long long i = t; i < n1; i += 256) e += p1[i];
        for (int o = 32; o > 0; o >>= 1) {
            a += __shfl_xor(a, o);
            e += __shfl_xor(e, o);
        }
        if ((t & 63) == 0) {
            wave_part[0][t >> 6] = a;
            wave_part[1][t >> 6] = e;
        }
    }
    __syncthreads();
    if (t == 0) {
        const double a = (wave_part[0][0] + wave_part[0][1]) + (wave_part[0][2] + wave_part[0][3]);
        const double e = (wave_part[1][0] + wave_part[1][1]) + (wave_part[1][2] + wave_part[1][3]);
        *out = w0 * a + (p1 ? w1 * e : 0.0);
    }
    __syncthreads();   // wave_part may be reused by the workgroup's next item
}

// Workgroups of `kernel` that the current device holds at once (cached).
int resident_workgroups(const void *kernel, int block, size_t shm);

// Grid size of a launch over L with `block` threads and `shm` dynamic LDS
// bytes; persistent launches fill the device once (occupancy-limited), but
// never exceed one workgroup per item.
template <typename Job>
inline long long launch_grid(const JobList<Job> &L, const void *kernel, int block, size_t shm)
{
    if (!L.jobs || !L.wq) return L.grid_static;
    long long grid = L.persistent_grid;
    if (grid <= 0) {
        const int per_device = resident_workgroups(kernel, block, shm);
        if (per_device <= 0) return -1;
        grid = per_device;
    }
    if (grid > L.total) grid = L.total;
    grid = kXcds * ((grid + kXcds - 1) / kXcds);
    return grid;
}

}  // namespace skei

// Ram-Lak ramp filter along detector rows (FBP's filtering step; Kak & Slaney
// ch. 3 with unit detector spacing), as a linear convolution with zero padding.
//
// Written in the symmetric form  q[k] = h(0) p[k] + sum_e h(2e+1) (p[k-2e-1] + p[k+2e+1]):
// the even taps are zero and the odd taps are wave-uniform scalar loads.
// Each thread owns V consecutive outputs and one of S fixed groups of taps,
// and keeps two register windows, p[k-d .. k-d+V) and p[k+d .. k+d+V):
// stepping d by 2 shifts each window by two entries, so a tap costs two new
// values per side for V outputs.  Accumulation is in double (it removes the
// cancellation error of the high-pass sum: terms of size ~p, result of size
// ~p/N), in increasing offset within a group; the S group sums are added in
// a fixed order.
#include <algorithm>

#include "skei_internal.h"
#include "work.h"

namespace skei {
namespace {

constexpr int kRampV = 8;   // outputs per thread
constexpr int kRampS = 4;   // tap groups per output (summed in a fixed order)
constexpr int kRampSumRows = 4;   // rows per row-sum-of-squares item (one wave each)

// Taps stepped per output: every odd offset below N_det, rounded up to whole
// groups of 4 taps per tap group.  row = [pad | n_det values | pad] in double
// with pad = 2 E + V + 2, so every window read stays inside the row.
__device__ __host__ __forceinline__ int ramp_taps(int n_det)
{
    const int q = 4 * kRampS;
    return ((n_det + 1) / 2 + q - 1) / q * q;
}
__device__ __host__ __forceinline__ int ramp_pad(int n_det) { return 2 * ramp_taps(n_det) + kRampV + 2; }
// threads of one tap group: enough for n_det outputs, in whole waves, so that
// the tap index is uniform across every wave
__device__ __host__ __forceinline__ int ramp_group(int n_det) { return ((n_det + kRampV - 1) / kRampV + 63) / 64 * 64; }

// Skewed-position offsets of the window reads of a 4-tap step (see ramp_item):
// left reads L[1], L[0] from the left base, right reads R[V-2], R[V-1] from
// the right base, for each of the step's 4 taps.
constexpr int kL[4][2] = {{0, -2}, {-3, -4}, {-5, -6}, {-7, -8}};
constexpr int kR[4][2] = {{3, 4}, {5, 6}, {7, 9}, {10, 11}};

template <typename IN>
__device__ __forceinline__ void ramp_item(const RampJob &J, long long r, double *row)
{
    constexpr int V = kRampV, S = kRampS;
    const int n_det = J.n_det;
    const int E = ramp_taps(n_det), ES = E / S;
    const int pad = ramp_pad(n_det);
    const int tid = threadIdx.x, bs = blockDim.x;
    if (J.loss) {
        fixed_order_loss(J.s0, J.n0, J.w0, J.s1, J.n1, J.w1, J.loss);
        return;
    }
    if (J.partial) {
        // row sums of squares, kRampSumRows rows per item: wave w takes row
        // kRampSumRows r + w, lane-strided then a butterfly, so the order does
        // not depend on the launch's block size (always >= 4 waves)
        const long long row_i = r * kRampSumRows + (tid >> 6);
        if (tid < 64 * kRampSumRows && row_i < J.rows) {
            const IN *p = static_cast<const IN *>(J.p) + (size_t)row_i * n_det;
            double s = 0.0;
            for (int k = tid & 63; k < n_det; k += 64) {
                const double v = (double)p[k];
                s = fma(v, v, s);
            }
            for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
            if ((tid & 63) == 0) J.partial[row_i] = s;
        }
        return;
    }
    const int per = ramp_group(n_det);          // threads per tap group (whole waves)
    const int len = n_det + 2 * pad;
    double *part = row + len + (len >> 3) + 1;  // [S - 1][per * V] partial sums
    const IN *src = static_cast<const IN *>(J.p) + (size_t)r * n_det;
    // the taps are read-only and wave-uniform: scalar loads
    typedef __attribute__((address_space(4))) const double ctap_t;
    const ctap_t *hodd = (const ctap_t *)J.hodd;
    // Row element q sits at LDS position q + q / 8: a thread's V = 8 outputs
    // start 9 doubles after its neighbour's, which spreads a wave's reads
    // over distinct banks.
    for (int e = tid; e < n_det + 2 * pad; e += bs) {
        const int j = e - pad;
        row[e + (e >> 3)] = (j >= 0 && j < n_det) ? (double)src[j] : 0.0;
    }
    __syncthreads();

    // thread (group sg, slot t): outputs k0 .. k0 + V - 1, taps e in [sg ES, (sg + 1) ES)
    const int sg = tid / per, t = tid - sg * per;
    const int k0 = t * V;
    double acc[V];
    if (sg < S) {
        // p[k0 + o] for an offset o: element pad + 8 t + o at 9 t + (pad + o) + (pad + o) / 8
        const double *c = row + 9 * t;
        auto at = [&](int o) { const int q = pad + o; return c[q + (q >> 3)]; };
        const int e0 = __builtin_amdgcn_readfirstlane(sg * ES);   // groups are whole waves
        double L[V], R[V];
#pragma unroll
        for (int i = 0; i < V; i++) {
            acc[i] = sg == 0 ? 0.25 * at(i) : 0.0;
            L[i] = at(i - 2 * e0 - 1);   // p[k0 + i - d], d = 2 e0 + 1
            R[i] = at(i + 2 * e0 + 1);   // p[k0 + i + d]
        }
        // The taps are a multiple of 16, so pad = 2 E + 10 = 2 (mod 8) and e0
        // is a multiple of 4.  A 4-tap step at e then reads left elements
        // a - 2u and a - 2u - 1 with a = pad - 2e - 2 = 0 (mod 8), and right
        // elements b + 2u and b + 2u + 1 with b = pad + 2e + 9 = 3 (mod 8):
        // their skewed positions are fixed offsets from 9 a / 8 and 9 (b - 3) / 8,
        // and both bases move by 9 per step, so no read needs address arithmetic.
        const double *pl = c + 9 * ((pad - 2 * e0 - 2) >> 3);
        const double *pr = c + 9 * ((pad + 2 * e0 + 9) >> 3);
        for (int e = e0; e < e0 + ES; e += 4, pl -= 9, pr += 9) {
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const double h = hodd[e + u];
#pragma unroll
                for (int i = 0; i < V; i++) acc[i] = fma(h, L[i] + R[i], acc[i]);
                // d -> d + 2: the left window moves two entries down, the right one two up
#pragma unroll
                for (int i = V - 1; i >= 2; i--) L[i] = L[i - 2];
                L[1] = pl[kL[u][0]];   // p[k0 - d - 1]
                L[0] = pl[kL[u][1]];   // p[k0 - d - 2]
#pragma unroll
                for (int i = 0; i < V - 2; i++) R[i] = R[i + 2];
                R[V - 2] = pr[kR[u][0]];   // p[k0 + d + V]
                R[V - 1] = pr[kR[u][1]];   // p[k0 + d + V + 1]
            }
        }
        if (sg > 0) {
#pragma unroll
            for (int i = 0; i < V; i++) part[(sg - 1) * per * V + k0 + i] = acc[i];
        }
    }
    __syncthreads();
    if (sg == 0) {
#pragma unroll
        for (int i = 0; i < V; i++) {
            const int k = k0 + i;
            double v = acc[i];
#pragma unroll
            for (int g = 1; g < S; g++) v += part[(g - 1) * per * V + k];
            if (k < n_det) J.q[(size_t)r * n_det + k] = (float)(v * (double)J.scale);
        }
    }
}

template <typename IN>
__global__ void __launch_bounds__(1024) k_ramp(const JobList<RampJob> L)
{
    extern __shared__ __align__(16) unsigned char ramp_raw[];
    double *row = reinterpret_cast<double *>(ramp_raw);
    for_each_item(L, [&](const RampJob &J, long long r) { ramp_item<IN>(J, r, row); });
}

template <typename IN>
int ramp_launch(int block, size_t shm, const JobList<RampJob> &L, hipStream_t st)
{
    if (L.total <= 0) return SKEI_OK;
    if (block < 64 || block > 1024 || block % 64 || shm > 160 * 1024) return SKEI_ERANGE;
    const long long grid = launch_grid(L, reinterpret_cast<const void *>(&k_ramp<IN>), block, shm);
    if (grid <= 0 || grid > 0x7fffffffLL) return SKEI_ERANGE;
    hipLaunchKernelGGL((k_ramp<IN>), dim3((unsigned)grid), dim3(block), shm, st, L);
    return check_launch();
}

}  // namespace

int ramp_block(int n_det) { return kRampS * ramp_group(n_det); }

// Host walk of every LDS read ramp_item makes for rows of n_det samples, with
// the kernel's own layout formulas and offset tables: out = {lowest index,
// highest index read by a thread that owns an output, highest index read by
// any thread (idle threads past the row end included), last index of the
// row area, elements allocated}, all in doubles from the start of the row.
void ramp_lds_reads(int n_det, long long out[5])
{
    constexpr int V = kRampV, S = kRampS;
    const int E = ramp_taps(n_det), ES = E / S, pad = ramp_pad(n_det), per = ramp_group(n_det);
    const long long len = n_det + 2LL * pad;
    long long lo = 1LL << 60, hi_active = -1, hi_any = -1;
    auto see = [&](long long pos, bool active) {
        lo = std::min(lo, pos);
        hi_any = std::max(hi_any, pos);
        if (active) hi_active = std::max(hi_active, pos);
    };
    for (int sg = 0; sg < S; sg++) {
        const int e0 = sg * ES;
        for (int t = 0; t < per; t++) {
            const bool active = t * V < n_det;
            const long long c = 9LL * t;
            for (int i = 0; i < V; i++) {
                for (const int o : {i - 2 * e0 - 1, i + 2 * e0 + 1}) {
                    const long long q = pad + o;
                    see(c + q + (q >> 3), active);
                }
            }
            long long pl = c + 9LL * ((pad - 2 * e0 - 2) >> 3), pr = c + 9LL * ((pad + 2 * e0 + 9) >> 3);
            for (int e = e0; e < e0 + ES; e += 4, pl -= 9, pr += 9)
                for (int u = 0; u < 4; u++) {
                    see(pl + kL[u][0], active);
                    see(pl + kL[u][1], active);
                    see(pr + kR[u][0], active);
                    see(pr + kR[u][1], active);
                }
        }
    }
    out[0] = lo;
    out[1] = hi_active;
    out[2] = hi_any;
    out[3] = (len - 1) + ((len - 1) >> 3);
    out[4] = (long long)(ramp_shm(n_det) / sizeof(double));
}

size_t ramp_shm(int n_det)
{
    const size_t len = (size_t)(n_det + 2 * ramp_pad(n_det));
    return sizeof(double) * (len + (len >> 3) + 1 + (size_t)(kRampS - 1) * ramp_group(n_det) * kRampV);
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

RampJob make_row_sumsq_job(const skei_geom *g, const float *p, long long rows, double *partial)
{
    RampJob J{};
    J.p = p;
    J.partial = partial;
    J.n_det = g->n_det;
    J.rows = rows;
    J.items = (rows + kRampSumRows - 1) / kRampSumRows;
    return J;
}

RampJob make_loss_job(const RedJob &r)
{
    RampJob J{};
    J.s0 = r.p0;
    J.n0 = r.n0;
    J.w0 = r.w0;
    J.s1 = r.p1;
    J.n1 = r.n1;
    J.w1 = r.w1;
    J.loss = r.out;
    J.n_det = 1;
    J.items = 1;
    return J;
}

int ramp_run(bool in_double, int block, size_t shm, const JobList<RampJob> &L, hipStream_t st)
{
    return in_double ? ramp_launch<double>(block, shm, L, st) : ramp_launch<float>(block, shm, L, st);
}

int launch_ramp(const skei_geom *g, const float *pf, const double *pd, long long rows, float scale, float *q,
                hipStream_t st)
{
    const bool dbl = pd != nullptr;
    const RampJob J = make_ramp_job(g, dbl ? (const void *)pd : (const void *)pf, rows, scale, q);
    return ramp_run(dbl, ramp_block(g->n_det), ramp_shm(g->n_det), inline_jobs(&J, 1), st);
}

}  // namespace skei

// Pixel-driven gathers over the listed angles: the Joseph adjoint A_S^T and
// the FBP backprojection B_S.  Neither scatters, so there are no atomics.
//
// A workgroup owns a 16 x 16 pixel tile of one image.  For every listed angle
// the tile projects onto fewer than 16*sqrt(2) + 2 detectors, so the angle's
// sinogram row is staged into LDS only over a 32-bin window; the per-angle
// constants (cos, sin, the window offset of the tile origin in double
// precision, Joseph weights) are staged beside it.  Each pixel then reads one
// 8-byte LDS entry per angle: (value, next value) for the Joseph adjoint, or
// (value, next - value) for the linear-interpolation backprojection.
// Positions are formed in double relative to the tile origin, so the
// interpolation weights carry only their final float rounding.
#include <cmath>

#include "skei_internal.h"
#include "work.h"

namespace skei {
namespace {

enum Kind : int { kJosephAdj = 0, kBackproject = 1 };

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

struct GatherAngle {
    double c, s, t0;   // cos, sin, detector coordinate of the tile origin within the window
    float w, wm1;      // Joseph width max(|cos|,|sin|) and w - 1
};

// A workgroup holds a 16 x 16 tile x GA angle groups; each thread owns PPT
// pixels of one tile row (columns dx, dx + 16/PPT, ...), so the per-angle
// constants, window staging and the row's share of the position are shared
// by PPT pixels.  The listed angles
// are split into four fixed classes (r % 4); each class is summed in
// increasing r, and the four class sums are added in a fixed order.  Thread
// (pixel group, ga) owns the classes ga, ga + GA, ...  Positions are relative
// to the fixed 16 x 16 tile grid, so every pixel's arithmetic is the same
// whatever GA, PPT, the batch size or the other jobs of the launch -- results
// are bitwise invariant.
constexpr int kClasses = 4;

template <int KIND, int GA, int PPT>
__device__ __forceinline__ void gather_item(const GatherJob &J, long long item)
{
    constexpr int TILE = 16, NPIX = TILE * TILE, TPG = NPIX / PPT, BS = TPG * GA, WIN = 2 * TILE;
    constexpr int CW = TILE / PPT;   // column step between a thread's pixels
    constexpr int NC = kClasses / GA;
    __shared__ GatherAngle prm[kAngleChunk];
    __shared__ int kst[kAngleChunk];                  // first detector of each window
    __shared__ float iw2[kAngleChunk];                // 1/w^2 (Joseph weights)
    __shared__ float2 win[kAngleChunk * WIN];
    __shared__ float part[kClasses][NPIX];
    __shared__ float tileT[TILE][TILE + 1];
    __shared__ double pss[NPIX];
    static_assert(kAngleChunk % kClasses == 0, "angle chunks must keep the classes aligned");

    const int n = J.n, n_det = J.n_det, m = J.m;
    const int32_t *__restrict__ idx = J.idx;
    const AngleRow *__restrict__ tab = J.tab;
    const int tiles_x = (n + TILE - 1) / TILE;
    const int tiles = tiles_x * tiles_x;
    const int b = (int)(item / tiles), tile = (int)(item - (long long)b * tiles);
    const int i0 = (tile / tiles_x) * TILE, j0 = (tile % tiles_x) * TILE;
    const int tid = threadIdx.x;
    // TPG is a multiple of 64, so the angle group is wave-uniform: scalar loop control
    static_assert(TPG % 64 == 0, "angle groups are whole waves");
    const int pg = tid % TPG, ga = __builtin_amdgcn_readfirstlane(tid / TPG);
    // pixel v of this thread: row pg / CW, column pg % CW + v CW
    auto pix = [&](int v) { return (pg / CW) * TILE + pg % CW + v * CW; };
    const double fdy = (double)(pg / CW);
    double fdx[PPT];
#pragma unroll
    for (int v = 0; v < PPT; v++) fdx[v] = (double)(pg % CW + v * CW);
    const double cN = 0.5 * (n - 1), cD = 0.5 * (n_det - 1);
    const float *src = J.in + (size_t)b * m * n_det;

    float acc[NC][PPT];
#pragma unroll
    for (int c = 0; c < NC; c++)
#pragma unroll
        for (int v = 0; v < PPT; v++) acc[c][v] = 0.0f;
    for (int A0 = 0; A0 < m; A0 += kAngleChunk) {
        const int Ac = min(kAngleChunk, m - A0);
        __syncthreads();
        for (int a = tid; a < Ac; a += BS) {
            const AngleRow t = tab[idx[A0 + a]];
            const double c = t.cd, s = t.sd;
            const double X0 = j0 - cN, Y0 = i0 - cN;
            const double org = X0 * c + Y0 * s + cD;
            const double tmin = org + fmin(0.0, (TILE - 1) * c) + fmin(0.0, (TILE - 1) * s);
            const double k0 = floor(tmin) - 1.0;
            prm[a] = GatherAngle{c, s, org - k0, t.w, t.w - 1.0f};
            kst[a] = (int)k0;
            iw2[a] = t.inv_w2;
        }
        __syncthreads();
        for (int e = tid; e < Ac * WIN; e += BS) {
            const int a = e / WIN, wi = e % WIN;
            const int k = kst[a] + wi;
            const float *row = src + (size_t)(A0 + a) * n_det;
            const float v0 = (k >= 0 && k < n_det) ? row[k] : 0.0f;
            const float v1 = (k + 1 >= 0 && k + 1 < n_det) ? row[k + 1] : 0.0f;
            if (KIND == kJosephAdj)
                win[e] = make_float2(v0 * iw2[a], v1 * iw2[a]);
            else
                win[e] = make_float2(v0, v1 - v0);
        }
        __syncthreads();
#pragma unroll 2
        for (int a4 = 0; a4 < Ac; a4 += kClasses) {
#pragma unroll
            for (int c = 0; c < NC; c++) {
                const int a = a4 + ga + c * GA;
                if (a < Ac) {
                    const GatherAngle p = prm[a];
                    const float2 *wa_row = win + a * WIN;
                    const double trow = fma(fdy, p.s, p.t0);
#pragma unroll
                    for (int v = 0; v < PPT; v++) {
                        // window-local detector coordinate in double: exact to ~1e-15 px
                        const double tl = fma(fdx[v], p.c, trow);
                        const int k0 = (int)tl;                          // 1 <= tl < WIN - 1 by construction
                        const float f = (float)__builtin_amdgcn_fract(tl);
                        const float2 e = wa_row[k0];
                        if (KIND == kJosephAdj) {
                            // weights Lambda((k - t)/w)/w for k = k0, k0+1 (the 1/w^2 is in the
                            // window); both are <= 1, so the clamps fold into the add
                            const float wa = __builtin_amdgcn_fmed3f(p.w - f, 0.0f, 1.0f);
                            const float wb = __builtin_amdgcn_fmed3f(f + p.wm1, 0.0f, 1.0f);
                            acc[c][v] = fmaf(wa, e.x, acc[c][v]);
                            acc[c][v] = fmaf(wb, e.y, acc[c][v]);
                        } else {
                            acc[c][v] += e.x;
                            acc[c][v] = fmaf(f, e.y, acc[c][v]);
                        }
                    }
                }
            }
        }
    }
    float sum[PPT];
    if constexpr (GA == 1) {
#pragma unroll
        for (int v = 0; v < PPT; v++) sum[v] = ((acc[0][v] + acc[1][v]) + acc[2][v]) + acc[3][v];
    } else {
#pragma unroll
        for (int c = 0; c < NC; c++)
#pragma unroll
            for (int v = 0; v < PPT; v++) part[ga + c * GA][pix(v)] = acc[c][v];
        __syncthreads();
#pragma unroll
        for (int v = 0; v < PPT; v++) {
            const int px = pix(v);
            sum[v] = ((part[0][px] + part[1][px]) + part[2][px]) + part[3][px];
        }
    }

    // the threads of angle group 0 write the tile
    const bool resid = J.other != nullptr;
#pragma unroll
    for (int v = 0; v < PPT; v++) {
        const int px = pix(v), dx = px % TILE, dy = px / TILE;
        const int i = i0 + dy, j = j0 + dx;
        float out = 0.0f;
        double ss = 0.0;
        if (ga == 0 && i < n && j < n) {
            const size_t o = ((size_t)b * n + i) * n + j;
            out = sum[v] * J.scale;
            if (resid) {
                out = J.other[o] - out;
                ss = (double)out * (double)out;
            }
            J.out[o] = out;
        }
        if (ga == 0) {
            if (J.outT) tileT[dy][dx] = out;
            if (resid && J.partial) pss[px] = ss;
        }
    }
    if (J.outT) {   // the tile again, transposed through LDS (coalesced stores)
        __syncthreads();
        if (ga == 0) {
#pragma unroll
            for (int v = 0; v < PPT; v++) {
                const int px = pix(v), dx = px % TILE, dy = px / TILE;
                const int it = j0 + dy, jt = i0 + dx;
                if (it < n && jt < n) J.outT[((size_t)b * n + it) * n + jt] = tileT[dx][dy];
            }
        }
    }
    if (resid && J.partial) {
        // per-pixel squares summed in a fixed order, whatever the launch shape:
        // lane l of the first wave adds pixels l, l + 64, l + 128, l + 192,
        // then the wave reduces its lanes
        __syncthreads();
        if (tid < 64) {
            double s4 = ((pss[tid] + pss[tid + 64]) + pss[tid + 128]) + pss[tid + 192];
            s4 = wave_sum(s4);
            if (tid == 0) J.partial[item] = s4;
        }
    }
}

template <int KIND, int GA, int PPT>
__global__ void __launch_bounds__(256 * GA / PPT) k_gather(const JobList<GatherJob> L)
{
    for_each_item(L, [&](const GatherJob &J, long long item) { gather_item<KIND, GA, PPT>(J, item); });
}

template <int KIND, int GA, int PPT>
int gather_launch(const JobList<GatherJob> &L, hipStream_t st)
{
    if (L.total <= 0) return SKEI_OK;
    constexpr int block = 256 * GA / PPT;
    const long long grid = launch_grid(L, reinterpret_cast<const void *>(&k_gather<KIND, GA, PPT>), block, 0);
    if (grid <= 0 || grid > 0x7fffffffLL) return SKEI_ERANGE;
    hipLaunchKernelGGL((k_gather<KIND, GA, PPT>), dim3((unsigned)grid), dim3(block), 0, st, L);
    return check_launch();
}

template <int KIND>
int gather_launch_ga(int ga, const JobList<GatherJob> &L, hipStream_t st)
{
    switch (ga) {
    case 1: return gather_launch<KIND, 1, 1>(L, st);
    case 2: return gather_launch<KIND, 2, 1>(L, st);
    case 4: return gather_launch<KIND, 4, 1>(L, st);
    case 14: return gather_launch<KIND, 1, 4>(L, st);
    case 24: return gather_launch<KIND, 2, 4>(L, st);
    case 44: return gather_launch<KIND, 4, 4>(L, st);
    default: return SKEI_ERANGE;
    }
}

// The window must hold the tile's projection span (< 15*sqrt(2)) plus the
// one-bin lead and the interpolation neighbour.
static_assert(2 * 16 >= 2 + 22 + 2, "detector window too small for the pixel tile");

}  // namespace

// Default gather shape for up to m listed angles: four angle groups with four
// pixels per thread once there are enough angles to share, else one of each.
int gather_groups_auto(int m) { return m >= 64 ? 44 : 1; }

size_t gather_items(int n, int batch)
{
    const size_t t = (size_t)((n + 15) / 16);
    return t * t * batch;
}

GatherJob make_gather_job(const skei_geom *g, const float *in, int batch, const int32_t *idx, int m, float scale,
                          float *out, const float *other, double *partial, float *outT)
{
    GatherJob J{};
    J.in = in;
    J.idx = idx;
    J.tab = g->tab;
    J.out = out;
    J.other = other;
    J.partial = partial;
    J.outT = outT;
    J.n = g->n;
    J.n_det = g->n_det;
    J.m = m;
    J.scale = scale;
    J.items = (long long)gather_items(g->n, batch);
    return J;
}

int gather_run(int kind, int ga, const JobList<GatherJob> &L, hipStream_t st)
{
    return kind == kGatherJosephAdj ? gather_launch_ga<kJosephAdj>(ga, L, st)
                                    : gather_launch_ga<kBackproject>(ga, L, st);
}

int launch_gather(int kind, const skei_geom *g, const float *in, int batch, const int32_t *idx, int m, float scale,
                  float *out, const float *other, double *partial, float *outT, hipStream_t st)
{
    const GatherJob J = make_gather_job(g, in, batch, idx, m, scale, out, other, partial, outT);
    return gather_run(kind, gather_groups_auto(m), inline_jobs(&J, 1), st);
}

}  // namespace skei

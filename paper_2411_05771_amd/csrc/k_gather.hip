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

// XCD-major tile mapping (workgroup L runs on XCD L % 8): each XCD takes a
// contiguous range of (image, tile) items, so an image's tiles share one L2.
__device__ __forceinline__ bool decode_item(int total, int &item)
{
    const int L = blockIdx.x;
    const int per = (total + 7) >> 3;
    const int pos = L >> 3;
    item = (L & 7) * per + pos;
    return pos < per && item < total;
}

// A workgroup holds a 16 x 16 tile x GA angle groups: thread (pixel, ga) sums
// the listed angles r with r % GA == ga, and the GA partial sums are added in a
// fixed order through LDS.  GA depends only on m, and positions are relative
// to the fixed 16 x 16 tile grid, so every pixel's arithmetic is the same
// whatever the batch size -- results are bitwise batch invariant.
template <int KIND, int MODE, int GA>
__global__ void __launch_bounds__(256 * GA) k_gather(const float *__restrict__ in, int n, int n_det,
                                                     const int32_t *__restrict__ idx, int m,
                                                     const AngleRow *__restrict__ tab, float scale,
                                                     float *__restrict__ out, const float *__restrict__ other,
                                                     double *__restrict__ partial, int total,
                                                     float *__restrict__ outT)
{
    constexpr int TILE = 16, NPIX = TILE * TILE, BS = NPIX * GA, WIN = 2 * TILE;
    __shared__ GatherAngle prm[kAngleChunk];
    __shared__ int kst[kAngleChunk];                  // first detector of each window
    __shared__ float iw2[kAngleChunk];                // 1/w^2 (Joseph weights)
    __shared__ float2 win[kAngleChunk * WIN];
    __shared__ float part[GA][NPIX];
    __shared__ float tileT[TILE][TILE + 1];
    __shared__ double red[NPIX / 64];

    int item;
    if (!decode_item(total, item)) return;
    const int tiles_x = (n + TILE - 1) / TILE;
    const int tiles = tiles_x * tiles_x;
    const int b = item / tiles, tile = item - b * tiles;
    const int i0 = (tile / tiles_x) * TILE, j0 = (tile % tiles_x) * TILE;
    const int tid = threadIdx.x;
    const int px = tid % NPIX, ga = tid / NPIX;
    const int dx = px % TILE, dy = px / TILE;
    const double fdx = (double)dx, fdy = (double)dy;
    const double cN = 0.5 * (n - 1), cD = 0.5 * (n_det - 1);
    const float *src = in + (size_t)b * m * n_det;

    float acc = 0.0f;
    for (int A0 = 0; A0 < m; A0 += kAngleChunk) {
        const int Ac = min(kAngleChunk, m - A0);
        __syncthreads();
        for (int a = tid; a < Ac; a += BS) {
            const AngleRow t = tab[idx[A0 + a]];
            const double c = t.c, s = t.s;
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
#pragma unroll 4
        for (int a = ga; a < Ac; a += GA) {
            const GatherAngle p = prm[a];
            // window-local detector coordinate in double: exact to ~1e-15 px,
            // at the same issue rate as float on this device
            const double tl = fma(fdx, p.c, fma(fdy, p.s, p.t0));
            const int k0 = (int)tl;                          // 1 <= tl < WIN - 1 by construction
            const float f = (float)__builtin_amdgcn_fract(tl);
            const float2 e = win[a * WIN + k0];
            if (KIND == kJosephAdj) {
                // weights Lambda((k - t)/w)/w for k = k0, k0+1 (the 1/w^2 is in the window)
                const float wa = fmaxf(p.w - f, 0.0f);
                const float wb = fmaxf(f + p.wm1, 0.0f);
                acc = fmaf(wa, e.x, acc);
                acc = fmaf(wb, e.y, acc);
            } else {
                acc += e.x;
                acc = fmaf(f, e.y, acc);
            }
        }
    }
    if (GA > 1) {
        part[ga][px] = acc;
        __syncthreads();
        acc = part[0][px];
#pragma unroll
        for (int g = 1; g < GA; g++) acc += part[g][px];
    }

    // the threads of angle group 0 write the tile
    const int i = i0 + dy, j = j0 + dx;
    double ss = 0.0;
    float v = 0.0f;
    if (ga == 0 && i < n && j < n) {
        const size_t o = ((size_t)b * n + i) * n + j;
        v = acc * scale;
        if (MODE == kResidSub) {
            v = other[o] - v;
            ss = (double)v * (double)v;
        }
        out[o] = v;
    }
    if (outT) {   // the tile again, transposed through LDS (coalesced stores)
        if (ga == 0) tileT[dy][dx] = v;
        __syncthreads();
        const int it = j0 + dy, jt = i0 + dx;
        if (ga == 0 && it < n && jt < n) outT[((size_t)b * n + it) * n + jt] = tileT[dx][dy];
    }
    if (MODE == kResidSub && partial) {
        ss = wave_sum(ss);
        if ((tid & 63) == 0 && tid < NPIX) red[tid >> 6] = ss;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < NPIX / 64; w++) s += red[w];
            partial[item] = s;
        }
    }
}

// Angle groups per pixel: a function of m only (never of the batch).
int angle_groups(int m) { return m >= 256 ? 4 : m >= 64 ? 2 : 1; }

template <int KIND, int GA>
int gather_launch_g(const skei_geom *g, const float *in, int batch, const int32_t *idx, int m, float scale,
                    float *out, const float *other, double *partial, hipStream_t st, float *outT)
{
    const int n = g->n;
    const long long tiles = (long long)((n + 15) / 16) * ((n + 15) / 16);
    const long long total = tiles * batch;
    if (total > 0x0fffffffLL) return SKEI_ERANGE;
    const dim3 grid((unsigned)(8 * ((total + 7) / 8))), block(256 * GA);
    if (other)
        hipLaunchKernelGGL((k_gather<KIND, kResidSub, GA>), grid, block, 0, st, in, n, g->n_det, idx, m, g->tab,
                           scale, out, other, partial, (int)total, outT);
    else
        hipLaunchKernelGGL((k_gather<KIND, kPlain, GA>), grid, block, 0, st, in, n, g->n_det, idx, m, g->tab,
                           scale, out, nullptr, nullptr, (int)total, outT);
    return check_launch();
}

template <int KIND>
int gather_launch(const skei_geom *g, const float *in, int batch, const int32_t *idx, int m, float scale,
                  float *out, const float *other, double *partial, hipStream_t st, float *outT = nullptr)
{
    switch (angle_groups(m)) {
    case 4: return gather_launch_g<KIND, 4>(g, in, batch, idx, m, scale, out, other, partial, st, outT);
    case 2: return gather_launch_g<KIND, 2>(g, in, batch, idx, m, scale, out, other, partial, st, outT);
    default: return gather_launch_g<KIND, 1>(g, in, batch, idx, m, scale, out, other, partial, st, outT);
    }
}

// The window must hold the tile's projection span (< 15*sqrt(2)) plus the
// one-bin lead and the interpolation neighbour.
static_assert(2 * 16 >= 2 + 22 + 2, "detector window too small for the pixel tile");

}  // namespace

size_t gather_partials(const skei_geom *g, int batch)
{
    const size_t t = (size_t)((g->n + 15) / 16);
    return t * t * batch;
}

int launch_radon_adj(const skei_geom *g, const float *y, int batch, const int32_t *idx, int m, float *x,
                     const float *other, hipStream_t st)
{
    return gather_launch<kJosephAdj>(g, y, batch, idx, m, 1.0f, x, other, nullptr, st);
}

int launch_backproject(const skei_geom *g, const float *q, int batch, const int32_t *idx, int m, float scale,
                       float *x, const float *other, double *partial, hipStream_t st, float *xT)
{
    return gather_launch<kBackproject>(g, q, batch, idx, m, scale, x, other, partial, st, xT);
}

}  // namespace skei

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
// Positions inside the tile are small numbers (tile-local coordinates), so the
// float rounding of the interpolation position stays near 2e-6 px.
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

template <int KIND, int MODE>
__global__ void __launch_bounds__(256) k_gather(const float *__restrict__ in, int n, int n_det,
                                                const int32_t *__restrict__ idx, int m,
                                                const AngleRow *__restrict__ tab, float scale,
                                                float *__restrict__ out, const float *__restrict__ other,
                                                double *__restrict__ partial)
{
    __shared__ float4 prm[kAngleChunk];               // (cos, sin, window-local origin, w)
    __shared__ int kst[kAngleChunk];                  // first detector of each window
    __shared__ float iw2[kAngleChunk];                // 1/w^2 (Joseph weights)
    __shared__ float2 win[kAngleChunk * kWin];
    __shared__ double red[4];

    const int tiles_x = (n + kTile - 1) / kTile;
    const int tile = blockIdx.x, b = blockIdx.y;
    const int i0 = (tile / tiles_x) * kTile, j0 = (tile % tiles_x) * kTile;
    const int tid = threadIdx.x;
    const int dx = tid & (kTile - 1), dy = tid >> 4;
    const float fdx = (float)dx, fdy = (float)dy;
    const double cN = 0.5 * (n - 1), cD = 0.5 * (n_det - 1);
    const float *src = in + (size_t)b * m * n_det;

    float acc = 0.0f;
    for (int A0 = 0; A0 < m; A0 += kAngleChunk) {
        const int Ac = min(kAngleChunk, m - A0);
        __syncthreads();
        if (tid < Ac) {
            const AngleRow t = tab[idx[A0 + tid]];
            const double c = t.c, s = t.s;
            const double X0 = j0 - cN, Y0 = i0 - cN;
            const double org = X0 * c + Y0 * s + cD;
            const double tmin = org + fmin(0.0, (kTile - 1) * c) + fmin(0.0, (kTile - 1) * s);
            const double k0 = floor(tmin) - 1.0;
            prm[tid] = make_float4(t.c, t.s, (float)(org - k0), t.w);
            kst[tid] = (int)k0;
            iw2[tid] = t.inv_w2;
        }
        __syncthreads();
        for (int e = tid; e < Ac * kWin; e += 256) {
            const int a = e / kWin, wi = e % kWin;
            const int k = kst[a] + wi;
            const float *row = src + (size_t)(A0 + a) * n_det;
            const float v0 = (k >= 0 && k < n_det) ? row[k] : 0.0f;
            const float v1 = (k + 1 >= 0 && k + 1 < n_det) ? row[k + 1] : 0.0f;
            if (KIND == kJosephAdj) {
                win[e] = make_float2(v0 * iw2[a], v1 * iw2[a]);
            } else {
                win[e] = make_float2(v0, v1 - v0);
            }
        }
        __syncthreads();
        for (int a = 0; a < Ac; a++) {
            const float4 p = prm[a];
            const float tl = fmaf(fdx, p.x, fmaf(fdy, p.y, p.z));
            const int k0 = (int)tl;                          // tl >= 1 by construction
            const float f = tl - (float)k0;
            const float2 e = win[a * kWin + k0];
            if (KIND == kJosephAdj) {
                // weights Lambda((k - t)/w)/w for k = k0, k0+1 (the 1/w^2 is in the window)
                const float wa = fmaxf(p.w - f, 0.0f);
                const float wb = fmaxf(f + (p.w - 1.0f), 0.0f);
                acc = fmaf(wa, e.x, acc);
                acc = fmaf(wb, e.y, acc);
            } else {
                acc += e.x;
                acc = fmaf(f, e.y, acc);
            }
        }
    }

    const int i = i0 + dy, j = j0 + dx;
    double ss = 0.0;
    if (i < n && j < n) {
        const size_t o = ((size_t)b * n + i) * n + j;
        float v = acc * scale;
        if (MODE == kResidSub) {
            v = other[o] - v;
            ss = (double)v * (double)v;
        }
        out[o] = v;
    }
    if (MODE == kResidSub && partial) {
        ss = wave_sum(ss);
        if ((tid & 63) == 0) red[tid >> 6] = ss;
        __syncthreads();
        if (tid == 0) partial[(size_t)b * gridDim.x + tile] = red[0] + red[1] + red[2] + red[3];
    }
}

template <int KIND>
int gather_launch(const skei_geom *g, const float *in, int batch, const int32_t *idx, int m, float scale,
                  float *out, const float *other, double *partial, hipStream_t st)
{
    const int n = g->n;
    const int tiles = ((n + kTile - 1) / kTile) * ((n + kTile - 1) / kTile);
    const dim3 grid(tiles, batch);
    if (other)
        hipLaunchKernelGGL((k_gather<KIND, kResidSub>), grid, dim3(256), 0, st, in, n, g->n_det, idx, m, g->tab,
                           scale, out, other, partial);
    else
        hipLaunchKernelGGL((k_gather<KIND, kPlain>), grid, dim3(256), 0, st, in, n, g->n_det, idx, m, g->tab,
                           scale, out, nullptr, nullptr);
    return check_launch();
}

// The window must hold the tile's projection span (< (kTile-1)*sqrt(2)) plus
// the one-bin lead and the interpolation neighbour.
static_assert(kWin >= 2 + 22 + 2, "detector window too small for the pixel tile");

}  // namespace

size_t gather_partials(const skei_geom *g, int batch)
{
    const size_t t = (size_t)((g->n + kTile - 1) / kTile);
    return t * t * batch;
}

int launch_radon_adj(const skei_geom *g, const float *y, int batch, const int32_t *idx, int m, float *x,
                     const float *other, hipStream_t st)
{
    return gather_launch<kJosephAdj>(g, y, batch, idx, m, 1.0f, x, other, nullptr, st);
}

int launch_backproject(const skei_geom *g, const float *q, int batch, const int32_t *idx, int m, float scale,
                       float *x, const float *other, double *partial, hipStream_t st)
{
    return gather_launch<kBackproject>(g, q, batch, idx, m, scale, x, other, partial, st);
}

}  // namespace skei

// Image rotations T_phi (the transformation group of Sec. 4.1.3) and their
// exact transpose, both as gathers.
//
// T_phi: output pixel (X, Y) samples the input bilinearly at
//   u = cos X + sin Y + cN (column),  v = -sin X + cos Y + cN (row),
// zero outside.  The transpose is evaluated per input pixel p' by visiting the
// output pixels whose sample point lies within one pixel of p' in both
// coordinates -- a rotated 2 x 2 square, whose bounding box holds at most 3 x 3
// pixel centres -- and recomputing each candidate's bilinear weight with
// exactly the expressions of the forward kernel, so the two kernels apply
// bitwise-identical matrix entries.
#include <cmath>

#include "skei_internal.h"

namespace skei {
namespace {

struct Sample {
    int i0, j0;
    float au, av;
};

// The one place where a sample point and its bilinear fractions are computed.
// Positions are formed in double precision (a float position near the image
// border would carry ~ulp(N) of rounding into every weight).
__device__ __forceinline__ Sample sample_point(int i, int j, float c, float s, double cN)
{
    const double X = (double)j - cN, Y = (double)i - cN;
    const double cd = c, sd = s;
    const double u = fma(cd, X, fma(sd, Y, cN));
    const double v = fma(-sd, X, fma(cd, Y, cN));
    const double fu = floor(u), fv = floor(v);
    Sample r;
    r.j0 = (int)fu;
    r.i0 = (int)fv;
    r.au = (float)(u - fu);
    r.av = (float)(v - fv);
    return r;
}

// One 16 x 16 output tile per workgroup; the tile is also written transposed
// (through LDS, so both stores are coalesced) when outT is given.
__global__ void __launch_bounds__(256) k_rotate(const float *__restrict__ x, int n, int copies,
                                                const float *__restrict__ cs, float *__restrict__ out,
                                                float *__restrict__ outT)
{
    __shared__ float tile[16][17];
    const int tiles_x = (n + 15) / 16;
    const int i0 = (blockIdx.x / tiles_x) * 16, j0 = (blockIdx.x % tiles_x) * 16;
    const int bc = blockIdx.y;                 // b * copies + c
    const int b = bc / copies, c = bc - b * copies;
    const int dx = threadIdx.x & 15, dy = threadIdx.x >> 4;
    const int i = i0 + dy, j = j0 + dx;
    const double cN = 0.5 * (double)(n - 1);
    float acc = 0.0f;
    if (i < n && j < n) {
        const Sample sp = sample_point(i, j, cs[2 * c], cs[2 * c + 1], cN);
        const float *img = x + (size_t)b * n * n;
#pragma unroll
        for (int di = 0; di < 2; di++) {
            const int ii = sp.i0 + di;
            const float wv = di ? sp.av : 1.0f - sp.av;
#pragma unroll
            for (int dj = 0; dj < 2; dj++) {
                const int jj = sp.j0 + dj;
                const float wu = dj ? sp.au : 1.0f - sp.au;
                if (ii >= 0 && ii < n && jj >= 0 && jj < n) acc = fmaf(wv * wu, img[(size_t)ii * n + jj], acc);
            }
        }
        out[(size_t)bc * n * n + (size_t)i * n + j] = acc;
    }
    if (outT) {
        tile[dy][dx] = acc;
        __syncthreads();
        const int it = j0 + dy, jt = i0 + dx;   // transposed position: row = original column
        if (it < n && jt < n) outT[(size_t)bc * n * n + (size_t)it * n + jt] = tile[dx][dy];
    }
}

// xT[b][j][i] = x[b][i][j], 16 x 16 tiles through LDS.
__global__ void __launch_bounds__(256) k_transpose(const float *__restrict__ x, int n, float *__restrict__ xT)
{
    __shared__ float tile[16][17];
    const int tiles_x = (n + 15) / 16;
    const int i0 = (blockIdx.x / tiles_x) * 16, j0 = (blockIdx.x % tiles_x) * 16;
    const size_t off = (size_t)blockIdx.y * n * n;
    const int dx = threadIdx.x & 15, dy = threadIdx.x >> 4;
    if (i0 + dy < n && j0 + dx < n) tile[dy][dx] = x[off + (size_t)(i0 + dy) * n + j0 + dx];
    __syncthreads();
    if (j0 + dy < n && i0 + dx < n) xT[off + (size_t)(j0 + dy) * n + i0 + dx] = tile[dx][dy];
}

// g[b][p'] = alpha * sum_c sum_p T_c[p][p'] h[b][c][p] + beta * add[b][p']
// A workgroup covers 64 consecutive pixels x 4 copy groups (copies c = grp,
// grp+4, ...); the four partial sums are added in a fixed order through LDS.
constexpr int kRotPix = 64, kRotGroups = 4;

__global__ void __launch_bounds__(256) k_rotate_adj(const float *__restrict__ h, int n, int copies,
                                                    const float *__restrict__ cs, float alpha,
                                                    const float *__restrict__ add, float beta,
                                                    float *__restrict__ g)
{
    __shared__ float part[kRotGroups][kRotPix];
    const int px = threadIdx.x & (kRotPix - 1), grp = threadIdx.x / kRotPix;
    const int p = blockIdx.x * kRotPix + px;
    const int b = blockIdx.y;
    const bool in = p < n * n;
    float acc = 0.0f;
    if (in) {
        const int ip = p / n, jp = p - ip * n;
        const double cN = 0.5 * (double)(n - 1);
        const double Xp = (double)jp - cN, Yp = (double)ip - cN;
        for (int c = grp; c < copies; c += kRotGroups) {
            const float co = cs[2 * c], si = cs[2 * c + 1];
            const float *hc = h + ((size_t)b * copies + c) * n * n;
            // centre of the candidate set: the output position whose sample is p'
            const double colc = fma((double)co, Xp, fma(-(double)si, Yp, cN));
            const double rowc = fma((double)si, Xp, fma((double)co, Yp, cN));
            const double hw = fabs((double)co) + fabs((double)si) + 1e-6;
            const int jlo = (int)ceil(colc - hw), ilo = (int)ceil(rowc - hw);
#pragma unroll
            for (int di = 0; di < 3; di++) {
                const int i = ilo + di;
                if (i < 0 || i >= n) continue;
#pragma unroll
                for (int dj = 0; dj < 3; dj++) {
                    const int j = jlo + dj;
                    if (j < 0 || j >= n) continue;
                    const Sample sp = sample_point(i, j, co, si, cN);
                    const int ei = ip - sp.i0, ej = jp - sp.j0;
                    if ((unsigned)ei > 1u || (unsigned)ej > 1u) continue;
                    const float wv = ei ? sp.av : 1.0f - sp.av;
                    const float wu = ej ? sp.au : 1.0f - sp.au;
                    acc = fmaf(wv * wu, hc[(size_t)i * n + j], acc);
                }
            }
        }
    }
    part[grp][px] = acc;
    __syncthreads();
    if (grp == 0 && in) {
        const float s = ((part[0][px] + part[1][px]) + part[2][px]) + part[3][px];
        float v = alpha * s;
        if (add) v = fmaf(beta, add[(size_t)b * n * n + p], v);
        g[(size_t)b * n * n + p] = v;
    }
}

}  // namespace

int launch_rotate(const float *x, int batch, int copies, int n, const float *cs, float *out, hipStream_t st,
                  float *outT)
{
    const int t = (n + 15) / 16;
    const dim3 grid(t * t, batch * copies);
    hipLaunchKernelGGL(k_rotate, grid, dim3(256), 0, st, x, n, copies, cs, out, outT);
    return check_launch();
}

int launch_transpose(const float *x, int batch, int n, float *xT, hipStream_t st)
{
    const int t = (n + 15) / 16;
    const dim3 grid(t * t, batch);
    hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, st, x, n, xT);
    return check_launch();
}

int launch_rotate_adj(const float *h, int batch, int copies, int n, const float *cs, float alpha,
                      const float *add, float beta, float *g, hipStream_t st)
{
    const dim3 grid((n * n + kRotPix - 1) / kRotPix, batch);
    hipLaunchKernelGGL(k_rotate_adj, grid, dim3(256), 0, st, h, n, copies, cs, alpha, add, beta, g);
    return check_launch();
}

}  // namespace skei

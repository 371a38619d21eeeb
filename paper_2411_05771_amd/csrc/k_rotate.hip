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
#include "work.h"

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

// One 16 x 16 output tile per work item, 64 threads, four rows of the tile
// per thread (more loads in flight per thread); the tile is also written
// transposed (through LDS, so both stores are coalesced) when outT is given.
// Jobs without rotations (cs == nullptr) copy / transpose the image exactly.
constexpr int kRotThreads = 64;

__device__ __forceinline__ void rotate_item(const RotJob &J, long long item)
{
    __shared__ float tile[16][17];
    const int n = J.n, copies = J.copies;
    const int tiles_x = (n + 15) / 16;
    const int tiles = tiles_x * tiles_x;
    const long long bc = item / tiles;          // b * copies + c
    const int t = (int)(item - bc * tiles);
    const int i0 = (t / tiles_x) * 16, j0 = (t % tiles_x) * 16;
    const long long b = bc / copies;
    const int c = (int)(bc - b * copies);
    const int dx = threadIdx.x & 15, dy0 = threadIdx.x >> 4;   // rows dy0, dy0 + 4, dy0 + 8, dy0 + 12
    const float *img = J.x + (size_t)b * n * n;
    const double cN = 0.5 * (double)(n - 1);
    // c is uniform over the workgroup and the rotation table is read-only
    // while kernels run: scalar loads
    const cword_t *csw = J.cs ? (const cword_t *)(J.cs + 2 * __builtin_amdgcn_readfirstlane(c)) : nullptr;
    const float co = csw ? __uint_as_float(csw[0]) : 1.0f, si = csw ? __uint_as_float(csw[1]) : 0.0f;
    // Every tap is loaded unconditionally from a clamped address and zeroed
    // when it falls outside the image, so the sixteen loads of a thread are
    // all in flight together; adding an exact zero leaves a sum unchanged.
    float acc[4];
    if (J.cs) {
        float v[4][4], w[4][4];
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const Sample sp = sample_point(i0 + dy0 + 4 * r, j0 + dx, co, si, cN);
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const int di = k >> 1, dj = k & 1;
                const int ii = sp.i0 + di, jj = sp.j0 + dj;
                const bool ok = ii >= 0 && ii < n && jj >= 0 && jj < n;
                const float t = img[ok ? (size_t)ii * n + jj : 0];
                v[r][k] = ok ? t : 0.0f;
                w[r][k] = (di ? sp.av : 1.0f - sp.av) * (dj ? sp.au : 1.0f - sp.au);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; r++) {
            float a = 0.0f;
#pragma unroll
            for (int k = 0; k < 4; k++) a = fmaf(w[r][k], v[r][k], a);
            acc[r] = a;
        }
    } else {
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int i = i0 + dy0 + 4 * r, j = j0 + dx;
            const bool ok = i < n && j < n;
            const float t = img[ok ? (size_t)i * n + j : 0];
            acc[r] = ok ? t : 0.0f;
        }
    }
    if (J.out) {
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int i = i0 + dy0 + 4 * r, j = j0 + dx;
            if (i < n && j < n) J.out[(size_t)bc * n * n + (size_t)i * n + j] = acc[r];
        }
    }
    if (J.outT) {
        __syncthreads();   // an earlier item of this workgroup may still read the tile
#pragma unroll
        for (int r = 0; r < 4; r++) tile[dy0 + 4 * r][dx] = acc[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int dy = dy0 + 4 * r;
            const int it = j0 + dy, jt = i0 + dx;   // transposed position: row = original column
            if (it < n && jt < n) J.outT[(size_t)bc * n * n + (size_t)it * n + jt] = tile[dx][dy];
        }
    }
}

__global__ void __launch_bounds__(kRotThreads) k_rotate(const JobList<RotJob> L)
{
    for_each_item(L, [&](const RotJob &J, long long item) { rotate_item(J, item); });
}

// g[b][p'] = alpha * sum_c sum_p T_c[p][p'] h[b][c][p] + beta * add[b][p']
// A work item covers 64 consecutive pixels x 4 copy groups (copies c = grp,
// grp+4, ...); the four partial sums are added in a fixed order through LDS.
constexpr int kRotPix = 64, kRotGroups = 4;

__device__ __forceinline__ void rotate_adj_item(const RotAdjJob &J, long long item)
{
    __shared__ float part[kRotGroups][kRotPix];
    const int n = J.n, copies = J.copies;
    const long long blocks = ((long long)n * n + kRotPix - 1) / kRotPix;
    const long long b = item / blocks;
    // one wave per copy group: grp is wave-uniform, so a copy's cos / sin are scalar loads
    const int px = threadIdx.x & (kRotPix - 1), grp = __builtin_amdgcn_readfirstlane(threadIdx.x / kRotPix);
    const int p = (int)(item - b * blocks) * kRotPix + px;
    const bool in = p < n * n;
    float acc = 0.0f;
    if (in) {
        const int ip = p / n, jp = p - ip * n;
        const double cN = 0.5 * (double)(n - 1);
        const double Xp = (double)jp - cN, Yp = (double)ip - cN;
        for (int c = grp; c < copies; c += kRotGroups) {
            // the rotation table is read-only while kernels run: scalar loads
            const cword_t *csw = (const cword_t *)(J.cs + 2 * c);
            const float co = __uint_as_float(csw[0]), si = __uint_as_float(csw[1]);
            const float *hc = J.h + ((size_t)b * copies + c) * n * n;
            // centre of the candidate set: the output position whose sample is p'
            const double colc = fma((double)co, Xp, fma(-(double)si, Yp, cN));
            const double rowc = fma((double)si, Xp, fma((double)co, Yp, cN));
            const double hw = fabs((double)co) + fabs((double)si) + 1e-6;
            const int jlo = (int)ceil(colc - hw), ilo = (int)ceil(rowc - hw);
            // all nine candidates are loaded (clamped address) before any is
            // used; a candidate that does not touch p' contributes an exact zero
            float v[9], w[9];
#pragma unroll
            for (int k = 0; k < 9; k++) {
                const int i = ilo + k / 3, j = jlo + k % 3;
                const Sample sp = sample_point(i, j, co, si, cN);
                const int ei = ip - sp.i0, ej = jp - sp.j0;
                const bool ok = i >= 0 && i < n && j >= 0 && j < n && (unsigned)ei <= 1u && (unsigned)ej <= 1u;
                const float t = hc[ok ? (size_t)i * n + j : (size_t)p];
                v[k] = ok ? t : 0.0f;
                w[k] = (ei ? sp.av : 1.0f - sp.av) * (ej ? sp.au : 1.0f - sp.au);
            }
#pragma unroll
            for (int k = 0; k < 9; k++) acc = fmaf(w[k], v[k], acc);
        }
    }
    __syncthreads();   // an earlier item of this workgroup may still read part[]
    part[grp][px] = acc;
    __syncthreads();
    if (grp == 0 && in) {
        const float s = ((part[0][px] + part[1][px]) + part[2][px]) + part[3][px];
        float v = J.alpha * s;
        const size_t o = (size_t)b * n * n + p;
        if (J.add) v = fmaf(J.beta, J.add[o], v);
        J.g[o] = v;
        if (J.x_upd) J.x_upd[o] = fmaf(-J.step, v, J.x_upd[o]);
    }
}

__global__ void __launch_bounds__(256) k_rotate_adj(const JobList<RotAdjJob> L)
{
    for_each_item(L, [&](const RotAdjJob &J, long long item) { rotate_adj_item(J, item); });
}

}  // namespace

RotJob make_rot_job(const float *x, int batch, int copies, int n, const float *cs, float *out, float *outT)
{
    RotJob J{};
    J.x = x;
    J.cs = cs;
    J.out = out;
    J.outT = outT;
    J.n = n;
    J.copies = cs ? copies : 1;
    const long long t = (n + 15) / 16;
    J.items = t * t * batch * J.copies;
    return J;
}

RotAdjJob make_rot_adj_job(const float *h, int batch, int copies, int n, const float *cs, float alpha,
                           const float *add, float beta, float *g)
{
    RotAdjJob J{};
    J.h = h;
    J.cs = cs;
    J.add = add;
    J.g = g;
    J.n = n;
    J.copies = copies;
    J.alpha = alpha;
    J.beta = beta;
    J.items = (((long long)n * n + kRotPix - 1) / kRotPix) * batch;
    return J;
}

int rotate_run(const JobList<RotJob> &L, hipStream_t st)
{
    if (L.total <= 0) return SKEI_OK;
    const long long grid = launch_grid(L, reinterpret_cast<const void *>(&k_rotate), kRotThreads, 0);
    if (grid <= 0 || grid > 0x7fffffffLL) return SKEI_ERANGE;
    hipLaunchKernelGGL(k_rotate, dim3((unsigned)grid), dim3(kRotThreads), 0, st, L);
    return check_launch();
}

int rotate_adj_run(const JobList<RotAdjJob> &L, hipStream_t st)
{
    if (L.total <= 0) return SKEI_OK;
    const long long grid = launch_grid(L, reinterpret_cast<const void *>(&k_rotate_adj), 256, 0);
    if (grid <= 0 || grid > 0x7fffffffLL) return SKEI_ERANGE;
    hipLaunchKernelGGL(k_rotate_adj, dim3((unsigned)grid), dim3(256), 0, st, L);
    return check_launch();
}

int launch_rotate(const float *x, int batch, int copies, int n, const float *cs, float *out, float *outT,
                  hipStream_t st)
{
    const RotJob J = make_rot_job(x, batch, copies, n, cs, out, outT);
    return rotate_run(inline_jobs(&J, 1), st);
}

int launch_rotate_adj(const float *h, int batch, int copies, int n, const float *cs, float alpha,
                      const float *add, float beta, float *g, hipStream_t st)
{
    const RotAdjJob J = make_rot_adj_job(h, batch, copies, n, cs, alpha, add, beta, g);
    return rotate_adj_run(inline_jobs(&J, 1), st);
}

}  // namespace skei

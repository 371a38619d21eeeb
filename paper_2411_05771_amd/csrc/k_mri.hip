// Multicoil MRI operator of Eq. (e:mri), k = M F (C x), its adjoint, and the
// coil-domain steps of the coil sketches (Sec. 3.4, Algorithm 3).
//
// Layout: complex values are interleaved float2 (re, im); an image x is
// [B][N][N], coil maps C are [Nc][N][N], k-space is [B][Nc][N][N], the mask
// M (the diagonal of the sampling operator) is a real [N][N] array shared by
// the coils.  F~ is the orthonormal 2-D DFT with no shift, N a power of two.
//
// The 2-D DFT runs as two passes of batched 1-D transforms through HBM: a
// workgroup stages W lines of one N x N plane in LDS (rows: W consecutive
// rows; columns: a strip of W consecutive columns, read as W-wide row
// segments), runs a radix-2 Stockham transform on them (natural order in and
// out, log2 N stages ping-ponging between two LDS buffers), and writes the
// lines back.  Twiddles exp(-+2 pi i t / N) are formed per workgroup in FP64
// and rounded once.  Each pass scales by 1/sqrt(N), so the 2-D transform is
// orthonormal.  The coil multiply is fused into the forward row pass, the
// mask into the forward column store and the adjoint column load; the
// adjoint's coil sum (with optional pixel weights) is a separate pass.
#include <algorithm>
#include <cmath>

#include "mri.h"

namespace skei {
namespace {

constexpr int kFftThreads = 256;
constexpr int kFftElems = 2048;     // most complex elements staged per workgroup
constexpr int kFftMinElems = 512;   // fewest, when the launch is small
constexpr long long kFftTargetGrid = 512;   // two workgroups per CU

enum Pass : int { kRowsFwd = 0, kColsFwd = 1, kColsAdj = 2, kRowsAdj = 3 };

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// W lines of length N of plane `plane` (b * nc + c), group g of the plane's
// N / W line groups.
//   kRowsFwd: in = x [B][N][N], out = k; loads x[b] * C[c] (* wgt), rows.
//   kColsFwd: in = out = k (in place), columns, mask on store.
//   kColsAdj: in = k, out = work, columns, mask on load, inverse.
//   kRowsAdj: in = out = work (in place), rows, inverse.
template <int PASS>
__global__ void __launch_bounds__(kFftThreads) k_fft_lines(const float2 *in, float2 *out,
                                                         const float2 *__restrict__ maps,
                                                         const float *__restrict__ mask,
                                                         const float *__restrict__ wgt, int n, int log_n, int w,
                                                         int nc, int groups)
{
    constexpr bool kRows = PASS == kRowsFwd || PASS == kRowsAdj;
    constexpr bool kInverse = PASS == kColsAdj || PASS == kRowsAdj;
    extern __shared__ float2 lds[];
    const int pitch = n + 1;                 // padded line pitch (float2)
    float2 *buf0 = lds, *buf1 = lds + w * pitch, *tw = lds + 2 * w * pitch;
    const int tid = threadIdx.x;
    const long long item = blockIdx.x;
    const long long plane = item / groups;
    const int g = (int)(item - plane * groups);
    const size_t nn = (size_t)n * n;
    const int b = (int)(plane / nc), c = (int)(plane - (long long)b * nc);

    for (int t = tid; t < n / 2; t += kFftThreads) {
        double s, co;
        sincospi((kInverse ? 2.0 : -2.0) * t / n, &s, &co);
        tw[t] = make_float2((float)co, (float)s);
    }
    // stage the lines: element e -> (line l, position t), consecutive
    // threads on consecutive addresses
    const int total = w * n;
    const float2 *src = (PASS == kRowsFwd ? in + (size_t)b * nn : in + (size_t)plane * nn);
    for (int e = tid; e < total; e += kFftThreads) {
        int l, t;
        size_t at;
        if (kRows) {
            l = e / n, t = e - l * n;
            at = (size_t)(g * w + l) * n + t;
        } else {
            t = e / w, l = e - t * w;
            at = (size_t)t * n + g * w + l;
        }
        float2 v = src[at];
        if (PASS == kRowsFwd) {
            v = cmul(v, maps[(size_t)c * nn + at]);
            if (wgt) {
                const float wv = wgt[at];
                v = make_float2(v.x * wv, v.y * wv);
            }
        }
        if (PASS == kColsAdj) {
            const float mk = mask[at];
            v = make_float2(v.x * mk, v.y * mk);
        }
        buf0[l * pitch + t] = v;
    }
    __syncthreads();
    // radix-2 Stockham: stage s (span ns = 2^s) reads a[j], a[j + N/2] and
    // writes b[(j / ns) 2 ns + j % ns] and the same + ns
    float2 *a = buf0, *bb = buf1;
    const int half = n >> 1;
    for (int s = 0; s < log_n; s++) {
        const int ns = 1 << s;
        for (int q = tid; q < w * half; q += kFftThreads) {
            const int l = q >> (log_n - 1), j = q & (half - 1);
            const int jm = j & (ns - 1);
            const float2 wt = tw[jm << (log_n - 1 - s)];
            const float2 v0 = a[l * pitch + j], v1 = cmul(a[l * pitch + j + half], wt);
            const int d = ((j >> s) << (s + 1)) + jm;
            bb[l * pitch + d] = make_float2(v0.x + v1.x, v0.y + v1.y);
            bb[l * pitch + d + ns] = make_float2(v0.x - v1.x, v0.y - v1.y);
        }
        __syncthreads();
        float2 *tmp = a;
        a = bb;
        bb = tmp;
    }
    const float scale = 1.0f / sqrtf((float)n);
    float2 *dst = out + (size_t)plane * nn;
    for (int e = tid; e < total; e += kFftThreads) {
        int l, t;
        size_t at;
        if (kRows) {
            l = e / n, t = e - l * n;
            at = (size_t)(g * w + l) * n + t;
        } else {
            t = e / w, l = e - t * w;
            at = (size_t)t * n + g * w + l;
        }
        float2 v = a[l * pitch + t];
        float sc = scale;
        if (PASS == kColsFwd) sc *= mask[at];
        dst[at] = make_float2(v.x * sc, v.y * sc);
    }
}

// x[b][p] = wgt[p] * sum_c conj(C_c[p]) z[b][c][p], the coils summed in
// increasing c; wgt may be null (1).
__global__ void __launch_bounds__(256) k_coil_combine(const float2 *__restrict__ z, const float2 *__restrict__ maps,
                                                      const float *__restrict__ wgt, int nc, long long d,
                                                      int batch, float2 *__restrict__ x)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d * batch) return;
    const long long b = i / d, p = i - b * d;
    float2 acc = make_float2(0.0f, 0.0f);
    for (int c = 0; c < nc; c++) {
        const float2 m = maps[(size_t)c * d + p], v = z[((size_t)b * nc + c) * d + p];
        acc.x += m.x * v.x + m.y * v.y;   // conj(m) v
        acc.y += m.x * v.y - m.y * v.x;
    }
    const float s = wgt ? wgt[p] : 1.0f;
    x[i] = make_float2(acc.x * s, acc.y * s);
}

// out[b][r][p] = sum_l G[r][l] z[b][l][p] (G complex [m_out][l_in]), l in
// increasing order.
__global__ void __launch_bounds__(256) k_coil_mix(const float2 *__restrict__ G, int m_out, int l_in,
                                                  const float2 *__restrict__ z, long long d, int batch,
                                                  float2 *__restrict__ out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per = (long long)m_out * d;
    if (i >= per * batch) return;
    const long long b = i / per, rp = i - b * per, r = rp / d, p = rp - r * d;
    float2 acc = make_float2(0.0f, 0.0f);
    for (int l = 0; l < l_in; l++) {
        const float2 gv = G[r * l_in + l], v = z[((size_t)b * l_in + l) * d + p];
        acc.x += gv.x * v.x - gv.y * v.y;
        acc.y += gv.x * v.y + gv.y * v.x;
    }
    out[i] = acc;
}

// wgt[p] = 1 / sum_c |C_c[p]|^2 (0 where every map vanishes), summed in double.
__global__ void __launch_bounds__(256) k_coil_weights(const float2 *__restrict__ maps, int nc, long long d,
                                                      float *__restrict__ wgt)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= d) return;
    double s = 0.0;
    for (int c = 0; c < nc; c++) {
        const float2 m = maps[(size_t)c * d + p];
        s += (double)m.x * m.x + (double)m.y * m.y;
    }
    wgt[p] = s > 0.0 ? (float)(1.0 / s) : 0.0f;
}

// One workgroup per coil pair (i, j): S_ij = sum_p conj(k_i[p]) k_j[p] and the
// coil sums s_i, s_j in double, per-thread strided partial sums then a fixed
// tree; V_ij = (S_ij - conj(s_i) s_j / d) / (d - 1), written as (re, im).
__global__ void __launch_bounds__(256) k_coil_cov(const float2 *__restrict__ k, int nc, long long d,
                                                  double *__restrict__ V)
{
    __shared__ double red[6][256];
    const int i = blockIdx.x / nc, j = blockIdx.x - (blockIdx.x / nc) * nc, tid = threadIdx.x;
    const float2 *ki = k + (size_t)i * d, *kj = k + (size_t)j * d;
    double sr = 0, si = 0, ar = 0, ai = 0, br = 0, bi = 0;
    for (long long p = tid; p < d; p += 256) {
        const double xr = ki[p].x, xi = ki[p].y, yr = kj[p].x, yi = kj[p].y;
        sr += xr * yr + xi * yi;   // conj(x) y
        si += xr * yi - xi * yr;
        ar += xr, ai += xi, br += yr, bi += yi;
    }
    red[0][tid] = sr, red[1][tid] = si, red[2][tid] = ar, red[3][tid] = ai, red[4][tid] = br, red[5][tid] = bi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o)
            for (int q = 0; q < 6; q++) red[q][tid] += red[q][tid + o];
        __syncthreads();
    }
    if (tid == 0) {
        const double dd = (double)d;
        // conj(s_i) s_j
        const double mr = red[2][0] * red[4][0] + red[3][0] * red[5][0];
        const double mi = red[2][0] * red[5][0] - red[3][0] * red[4][0];
        V[2 * ((size_t)i * nc + j)] = (red[0][0] - mr / dd) / (dd - 1.0);
        V[2 * ((size_t)i * nc + j) + 1] = (red[1][0] - mi / dd) / (dd - 1.0);
    }
}

int fft_pass_launch(int pass, const float2 *in, float2 *out, const float2 *maps, const float *mask,
                    const float *wgt, int n, int nc, int batch, hipStream_t st)
{
    int log_n = 0;
    while ((1 << log_n) < n) log_n++;
    // lines per workgroup: 2048 points, halved while the launch has fewer
    // than ~2 workgroups per CU, down to 512 points (measured on MI355X at
    // 128^2 x 15 coils: 20.5 -> 13.0 us for A; a line's arithmetic does not
    // depend on the grouping, so results are bitwise the same)
    const long long planes = (long long)batch * nc;
    int w = n >= kFftElems ? 1 : std::min(kFftElems / n, n);
    while (w > 1 && w * n > kFftMinElems && planes * (n / w) < kFftTargetGrid) w >>= 1;
    const int groups = n / w;
    const long long grid = planes * groups;
    if (grid > 0x7fffffffLL) return SKEI_ERANGE;
    const size_t lds = sizeof(float2) * (2 * (size_t)w * (n + 1) + n / 2);
    switch (pass) {
    case kRowsFwd:
        hipLaunchKernelGGL((k_fft_lines<kRowsFwd>), dim3((unsigned)grid), dim3(kFftThreads), lds, st, in, out, maps,
                           mask, wgt, n, log_n, w, nc, groups);
        break;
    case kColsFwd:
        hipLaunchKernelGGL((k_fft_lines<kColsFwd>), dim3((unsigned)grid), dim3(kFftThreads), lds, st, in, out, maps,
                           mask, wgt, n, log_n, w, nc, groups);
        break;
    case kColsAdj:
        hipLaunchKernelGGL((k_fft_lines<kColsAdj>), dim3((unsigned)grid), dim3(kFftThreads), lds, st, in, out, maps,
                           mask, wgt, n, log_n, w, nc, groups);
        break;
    default:
        hipLaunchKernelGGL((k_fft_lines<kRowsAdj>), dim3((unsigned)grid), dim3(kFftThreads), lds, st, in, out, maps,
                           mask, wgt, n, log_n, w, nc, groups);
        break;
    }
    return check_launch();
}

// 256-thread blocks covering `count` threads, or 0 when that exceeds a grid
long long blocks_for(long long count)
{
    const long long b = (count + 255) / 256;
    return b <= 0x7fffffffLL ? b : 0;
}

}  // namespace

bool mri_size_ok(int n) { return n >= 4 && n <= kMriMaxN && (n & (n - 1)) == 0; }

int launch_mri_fwd(const float2 *maps, int nc, int n, const float2 *x, int batch, const float *mask,
                   const float *wgt, float2 *k, hipStream_t st)
{
    int rc = fft_pass_launch(kRowsFwd, x, k, maps, mask, wgt, n, nc, batch, st);
    if (rc) return rc;
    return fft_pass_launch(kColsFwd, k, k, maps, mask, nullptr, n, nc, batch, st);
}

int launch_mri_adj(const float2 *maps, int nc, int n, const float2 *k, int batch, const float *mask,
                   const float *wgt, float2 *x, float2 *work, hipStream_t st)
{
    int rc = fft_pass_launch(kColsAdj, k, work, maps, mask, nullptr, n, nc, batch, st);
    if (rc) return rc;
    rc = fft_pass_launch(kRowsAdj, work, work, maps, mask, nullptr, n, nc, batch, st);
    if (rc) return rc;
    const long long d = (long long)n * n, blocks = blocks_for(d * batch);
    if (blocks == 0) return SKEI_ERANGE;
    hipLaunchKernelGGL(k_coil_combine, dim3((unsigned)blocks), dim3(256), 0, st, work, maps, wgt, nc, d, batch, x);
    return check_launch();
}

int launch_coil_mix(const float2 *G, int m_out, int l_in, const float2 *z, long long d, int batch, float2 *out,
                    hipStream_t st)
{
    const long long blocks = blocks_for((long long)m_out * d * batch);
    if (blocks == 0) return SKEI_ERANGE;
    hipLaunchKernelGGL(k_coil_mix, dim3((unsigned)blocks), dim3(256), 0, st, G, m_out, l_in, z, d, batch, out);
    return check_launch();
}

int launch_coil_weights(const float2 *maps, int nc, long long d, float *wgt, hipStream_t st)
{
    const long long blocks = blocks_for(d);
    if (blocks == 0) return SKEI_ERANGE;
    hipLaunchKernelGGL(k_coil_weights, dim3((unsigned)blocks), dim3(256), 0, st, maps, nc, d, wgt);
    return check_launch();
}

int launch_coil_cov(const float2 *k, int nc, long long d, double *V, hipStream_t st)
{
    hipLaunchKernelGGL(k_coil_cov, dim3((unsigned)(nc * nc)), dim3(256), 0, st, k, nc, d, V);
    return check_launch();
}

}  // namespace skei

// Ray-driven kernels: Joseph forward projection A_S and the transposed
// pixel-driven backprojection B_S^T.
//
// One workgroup owns one (image, listed angle, detector segment): its lanes are
// consecutive detectors, i.e. parallel rays that cross every image line along
// the angle's major axis.  The image is streamed through LDS in chunks of R
// lines -- rows when Joseph steps along rows, columns (transposed on the way
// in) otherwise -- so every tap is an LDS read of a line that the whole
// workgroup shares, and all global reads are contiguous.  Each ray's minor
// coordinate is recomputed from its indices with one FMA per line, so there is
// no running-sum drift.  Taps that fall off the image are clamped into
// zero-padded LDS borders instead of being branched around.
#include <algorithm>

#include "skei_internal.h"

namespace skei {
namespace {

constexpr int kSegMax = 2048;   // detectors per workgroup (rays per thread <= 8)

struct RayCfg {
    int block, rpt, nseg, seg;
};

RayCfg ray_config(int n_det)
{
    RayCfg c;
    c.nseg = (n_det + kSegMax - 1) / kSegMax;
    c.seg = (n_det + c.nseg - 1) / c.nseg;
    c.rpt = (c.seg + 255) / 256;
    const int per = (c.seg + c.rpt - 1) / c.rpt;
    c.block = ((per + 63) / 64) * 64;
    return c;
}

int line_stride(int n)
{
    int s = n + 2 * kLinePad;
    return (s % 2 == 0) ? s + 1 : s;   // odd stride: conflict-free transposed staging
}

// Default chunk height: the largest multiple of 4 lines (<= 64, <= n) whose
// LDS footprint stays within `budget` bytes.
int default_lines(int n, size_t elem_bytes, size_t budget)
{
    const size_t per_line = (size_t)line_stride(n) * elem_bytes;
    int r = (int)(budget / per_line);
    r = std::min(r, 64);
    r = std::min(r, ((n + 3) / 4) * 4);
    r = (r / 4) * 4;
    return std::max(r, 4);
}

__device__ __forceinline__ int wave_min(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_max(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Major-axis index range [lo, hi] over which ray minor coordinate u0 + M*du
// lies in (-margin_lo, n + margin_hi); empty range -> lo > hi.
__device__ __forceinline__ void ray_range(float u0, float du, int n, int &lo, int &hi)
{
    const float a = -2.0f, b = (float)n + 1.0f;
    if (fabsf(du) < 1e-12f) {
        if (u0 > a && u0 < b) {
            lo = 0;
            hi = n - 1;
        } else {
            lo = n;
            hi = -1;
        }
        return;
    }
    const float t1 = (a - u0) / du, t2 = (b - u0) / du;
    const float tl = fmaxf(floorf(fminf(t1, t2)) - 1.0f, 0.0f);
    const float th = fminf(ceilf(fmaxf(t1, t2)) + 1.0f, (float)(n - 1));
    lo = (int)tl;
    hi = (int)th;
}

// Walk of a flattened (line, unit) index space by a workgroup: each thread
// starts at unit `tid` and advances by `bs` units with a carry, so no integer
// division happens inside the staging loops.
struct Walk {
    int l, c;
    __device__ Walk(int tid, int units) : l(tid / units), c(tid % units) {}
    __device__ __forceinline__ void step(int sl, int sc, int units)
    {
        c += sc;
        l += sl;
        if (c >= units) {
            c -= units;
            l += 1;
        }
    }
};

// ---------------------------------------------------------------------------
// Stage lines [M0, M0+Rc) of image `img` into LDS.  Entry j of a line holds
// (v[j], v[j+1] - v[j]) with v[-1] = v[n] = 0, so a linear interpolation at
// u = j + f is  e.x + f * e.y  (one LDS read, two VALU ops).  Entries
// j <= -2 and j >= n are zero and are written once per kernel.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void stage_pairs(float2 *lds, const float *__restrict__ img, int n, int stride,
                                            int M0, int Rc, bool rows)
{
    const int tid = threadIdx.x, bs = blockDim.x;
    if ((n & 3) == 0 && (rows || (Rc & 3) == 0)) {
        if (rows) {
            const int units = n >> 2;                  // float4 per line
            const int total = Rc * units;
            Walk w(tid, units);
            const int sl = bs / units, sc = bs % units;
            for (int e = tid; e < total; e += bs, w.step(sl, sc, units)) {
                const float *src = img + (size_t)(M0 + w.l) * n + 4 * w.c;
                const float4 v = *reinterpret_cast<const float4 *>(src);
                const float nx = (4 * w.c + 4 < n) ? src[4] : 0.0f;
                float4 *dst = reinterpret_cast<float4 *>(lds + w.l * stride + kLinePad + 4 * w.c);
                // two 16-byte LDS writes per unit (float2 pairs)
                float2 *d2 = reinterpret_cast<float2 *>(dst);
                d2[0] = make_float2(v.x, v.y - v.x);
                d2[1] = make_float2(v.y, v.z - v.y);
                d2[2] = make_float2(v.z, v.w - v.z);
                d2[3] = make_float2(v.w, nx - v.w);
            }
        } else {
            const int units = Rc >> 2;                 // float4 per image row within the chunk
            const int total = n * units;
            Walk w(tid, units);
            const int sl = bs / units, sc = bs % units;
            for (int e = tid; e < total; e += bs, w.step(sl, sc, units)) {
                const int i = w.l;                     // image row = position along the staged columns
                const float *src = img + (size_t)i * n + M0 + 4 * w.c;
                const float4 v = *reinterpret_cast<const float4 *>(src);
                float4 nx = make_float4(0.f, 0.f, 0.f, 0.f);
                if (i + 1 < n) nx = *reinterpret_cast<const float4 *>(src + n);
                float2 *d = lds + (4 * w.c) * stride + kLinePad + i;
                d[0] = make_float2(v.x, nx.x - v.x);
                d[stride] = make_float2(v.y, nx.y - v.y);
                d[2 * stride] = make_float2(v.z, nx.z - v.z);
                d[3 * stride] = make_float2(v.w, nx.w - v.w);
            }
        }
    } else {
        const int total = Rc * n;
        Walk w(tid, n);
        const int sl = bs / n, sc = bs % n;
        for (int e = tid; e < total; e += bs, w.step(sl, sc, n)) {
            const int l = w.l, j = w.c;
            float v, nx;
            if (rows) {
                const float *src = img + (size_t)(M0 + l) * n;
                v = src[j];
                nx = (j + 1 < n) ? src[j + 1] : 0.0f;
            } else {
                v = img[(size_t)j * n + M0 + l];
                nx = (j + 1 < n) ? img[(size_t)(j + 1) * n + M0 + l] : 0.0f;
            }
            lds[l * stride + kLinePad + j] = make_float2(v, nx - v);
        }
    }
    // entry j = -1 of each line: (0, v[0])
    for (int l = tid; l < Rc; l += bs) {
        const float v0 = rows ? img[(size_t)(M0 + l) * n] : img[M0 + l];
        lds[l * stride + kLinePad - 1] = make_float2(0.0f, v0);
    }
}

// Plain float lines (for the 4-tap B_S^T walk): entry j holds v[j].
__device__ __forceinline__ void stage_values(float *lds, const float *__restrict__ img, int n, int stride,
                                             int M0, int Rc, bool rows)
{
    const int tid = threadIdx.x, bs = blockDim.x;
    if ((n & 3) == 0 && (rows || (Rc & 3) == 0)) {
        if (rows) {
            const int units = n >> 2;
            const int total = Rc * units;
            Walk w(tid, units);
            const int sl = bs / units, sc = bs % units;
            for (int e = tid; e < total; e += bs, w.step(sl, sc, units)) {
                const float4 v = *reinterpret_cast<const float4 *>(img + (size_t)(M0 + w.l) * n + 4 * w.c);
                float *d = lds + w.l * stride + kLinePad + 4 * w.c;
                d[0] = v.x;
                d[1] = v.y;
                d[2] = v.z;
                d[3] = v.w;
            }
        } else {
            const int units = Rc >> 2;
            const int total = n * units;
            Walk w(tid, units);
            const int sl = bs / units, sc = bs % units;
            for (int e = tid; e < total; e += bs, w.step(sl, sc, units)) {
                const int i = w.l;
                const float4 v = *reinterpret_cast<const float4 *>(img + (size_t)i * n + M0 + 4 * w.c);
                float *d = lds + (4 * w.c) * stride + kLinePad + i;
                d[0] = v.x;
                d[stride] = v.y;
                d[2 * stride] = v.z;
                d[3 * stride] = v.w;
            }
        }
    } else {
        const int total = Rc * n;
        Walk w(tid, n);
        const int sl = bs / n, sc = bs % n;
        for (int e = tid; e < total; e += bs, w.step(sl, sc, n)) {
            const int l = w.l, j = w.c;
            lds[l * stride + kLinePad + j] = rows ? img[(size_t)(M0 + l) * n + j] : img[(size_t)j * n + M0 + l];
        }
    }
}

template <typename T>
__device__ __forceinline__ void zero_borders(T *lds, int n, int stride, int R)
{
    const int tid = threadIdx.x, bs = blockDim.x;
    const int nb = stride - n;                       // border entries per line
    for (int e = tid; e < R * nb; e += bs) {
        const int l = e / nb, p = e - l * nb;
        const int pos = p < kLinePad ? p : n + p;    // [0, PAD) and [PAD+n, stride)
        lds[l * stride + pos] = T{};
    }
}

// ---------------------------------------------------------------------------
// K1: y[b][r][k] = (1/w) * sum_M lerp(line_M, u(k, M))      (Joseph)
// MODE kResidSub: y = yfull[b][idx[r]][k] - that, plus per-block sum of y^2.
// ---------------------------------------------------------------------------
template <int RPT, int MODE>
__global__ void __launch_bounds__(256) k_radon_fwd(const float *__restrict__ x, int n, int n_det,
                                                   const int32_t *__restrict__ idx, int m,
                                                   const AngleRow *__restrict__ tab, int R, int stride,
                                                   int seg, float *__restrict__ y,
                                                   const float *__restrict__ yfull, int n_angles,
                                                   double *__restrict__ partial)
{
    extern __shared__ float2 lds2[];
    __shared__ double red[8];
    const int r = blockIdx.x, b = blockIdx.y, sg = blockIdx.z;
    const int a = idx[r];
    const AngleRow t = tab[a];
    const float *img = x + (size_t)b * n * n;
    const int k_begin = sg * seg, k_end = min(n_det, k_begin + seg);
    const int tid = threadIdx.x, bs = blockDim.x;
    const bool rows = t.rows != 0;

    float u0[RPT], acc[RPT];
    int lo = n, hi = -1;
#pragma unroll
    for (int q = 0; q < RPT; q++) {
        const int k = k_begin + tid + q * bs;
        u0[q] = fmaf((float)k, t.inv_m, t.base);
        acc[q] = 0.0f;
        if (k < k_end) {
            int l0, h0;
            ray_range(u0[q], t.du, n, l0, h0);
            lo = min(lo, l0);
            hi = max(hi, h0);
        }
    }
    lo = __builtin_amdgcn_readfirstlane(wave_min(lo));
    hi = __builtin_amdgcn_readfirstlane(wave_max(hi));

    zero_borders(lds2, n, stride, R);
    const float ulo = -(float)kLinePad + 0.5f, uhi = (float)n + 1.5f;
    for (int M0 = 0; M0 < n; M0 += R) {
        const int Rc = min(R, n - M0);
        __syncthreads();
        stage_pairs(lds2, img, n, stride, M0, Rc, rows);
        __syncthreads();
        const int lb = max(lo - M0, 0), le = min(hi - M0, Rc - 1);
        for (int l = lb; l <= le; l++) {
            const float Mf = (float)(M0 + l);
            const float2 *line = lds2 + l * stride + kLinePad;
#pragma unroll
            for (int q = 0; q < RPT; q++) {
                float u = fmaf(Mf, t.du, u0[q]);
                u = __builtin_amdgcn_fmed3f(u, ulo, uhi);
                const float fl = floorf(u);
                const float f = u - fl;
                const float2 e = line[(int)fl];
                acc[q] += e.x;
                acc[q] = fmaf(f, e.y, acc[q]);
            }
        }
    }

    double ss = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; q++) {
        const int k = k_begin + tid + q * bs;
        if (k < k_end) {
            float v = acc[q] * t.scale;
            if (MODE == kResidSub) {
                v = yfull[((size_t)b * n_angles + a) * n_det + k] - v;
                ss += (double)v * (double)v;
            }
            y[((size_t)b * m + r) * n_det + k] = v;
        }
    }
    if (MODE == kResidSub) {
        ss = wave_sum(ss);
        const int wid = tid >> 6, nw = bs >> 6;
        if ((tid & 63) == 0) red[wid] = ss;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < nw; w++) s += red[w];
            partial[((size_t)b * m + r) * gridDim.z + sg] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// K5: q[b][r][k] = sum_M sum_{j} Lambda(w (j - u(k,M))) line_M[j]      (B_S^T)
// The pixels within unit distance of the ray in s are the (at most 3) line
// entries within 1/w of u; the four candidates j0-1 .. j0+2 cover them.
// ---------------------------------------------------------------------------
template <int RPT>
__global__ void __launch_bounds__(256) k_bp_T(const float *__restrict__ x, int n, int n_det,
                                              const int32_t *__restrict__ idx, int m,
                                              const AngleRow *__restrict__ tab, int R, int stride, int seg,
                                              float *__restrict__ q)
{
    extern __shared__ float lds1[];
    const int r = blockIdx.x, b = blockIdx.y, sg = blockIdx.z;
    const int a = idx[r];
    const AngleRow t = tab[a];
    const float *img = x + (size_t)b * n * n;
    const int k_begin = sg * seg, k_end = min(n_det, k_begin + seg);
    const int tid = threadIdx.x, bs = blockDim.x;
    const bool rows = t.rows != 0;
    const float w = t.w;
    const float c_m1 = 1.0f - w, c_m2 = 1.0f - 2.0f * w;

    float u0[RPT], acc[RPT];
    int lo = n, hi = -1;
#pragma unroll
    for (int p = 0; p < RPT; p++) {
        const int k = k_begin + tid + p * bs;
        u0[p] = fmaf((float)k, t.inv_m, t.base);
        acc[p] = 0.0f;
        if (k < k_end) {
            int l0, h0;
            ray_range(u0[p], t.du, n, l0, h0);
            lo = min(lo, l0);
            hi = max(hi, h0);
        }
    }
    lo = __builtin_amdgcn_readfirstlane(wave_min(lo));
    hi = __builtin_amdgcn_readfirstlane(wave_max(hi));

    zero_borders(lds1, n, stride, R);
    const float ulo = -2.5f, uhi = (float)n + 0.5f;
    for (int M0 = 0; M0 < n; M0 += R) {
        const int Rc = min(R, n - M0);
        __syncthreads();
        stage_values(lds1, img, n, stride, M0, Rc, rows);
        __syncthreads();
        const int lb = max(lo - M0, 0), le = min(hi - M0, Rc - 1);
        for (int l = lb; l <= le; l++) {
            const float Mf = (float)(M0 + l);
            const float *line = lds1 + l * stride + kLinePad;
#pragma unroll
            for (int p = 0; p < RPT; p++) {
                float u = fmaf(Mf, t.du, u0[p]);
                u = __builtin_amdgcn_fmed3f(u, ulo, uhi);
                const float fl = floorf(u);
                const float f = u - fl;
                const float *e = line + (int)fl;
                const float wa = fmaxf(fmaf(-w, f, c_m1), 0.0f);   // j0-1: 1 - w (1 + f)
                const float wb = fmaf(-w, f, 1.0f);                // j0  : 1 - w f
                const float wc = fmaf(w, f, c_m1);                 // j0+1: 1 - w (1 - f)
                const float wd = fmaxf(fmaf(w, f, c_m2), 0.0f);    // j0+2: 1 - w (2 - f)
                float s = acc[p];
                s = fmaf(wa, e[-1], s);
                s = fmaf(wb, e[0], s);
                s = fmaf(wc, e[1], s);
                s = fmaf(wd, e[2], s);
                acc[p] = s;
            }
        }
    }
#pragma unroll
    for (int p = 0; p < RPT; p++) {
        const int k = k_begin + tid + p * bs;
        if (k < k_end) q[((size_t)b * m + r) * n_det + k] = acc[p];
    }
}

template <int MODE>
int fwd_dispatch(const RayCfg &c, dim3 grid, size_t shm, hipStream_t st, const float *x, int n, int n_det,
                 const int32_t *idx, int m, const AngleRow *tab, int R, int stride, float *y,
                 const float *yfull, int n_angles, double *partial)
{
#define SKEI_FWD_CASE(P)                                                                                \
    case P:                                                                                             \
        hipLaunchKernelGGL((k_radon_fwd<P, MODE>), grid, dim3(c.block), shm, st, x, n, n_det, idx, m, \
                           tab, R, stride, c.seg, y, yfull, n_angles, partial);                         \
        break;
    switch (c.rpt) {
        SKEI_FWD_CASE(1)
        SKEI_FWD_CASE(2)
        SKEI_FWD_CASE(3)
        SKEI_FWD_CASE(4)
        SKEI_FWD_CASE(5)
        SKEI_FWD_CASE(6)
        SKEI_FWD_CASE(7)
        SKEI_FWD_CASE(8)
    default: return SKEI_ERANGE;
    }
#undef SKEI_FWD_CASE
    return check_launch();
}

}  // namespace

size_t radon_fwd_partials(const skei_geom *g, int batch, int m)
{
    return (size_t)batch * m * ray_config(g->n_det).nseg;
}

int launch_radon_fwd(const skei_geom *g, const float *x, int batch, const int32_t *idx, int m, float *y,
                     const float *yfull, double *partial, int lines_per_chunk, hipStream_t st)
{
    const int n = g->n, n_det = g->n_det;
    const RayCfg c = ray_config(n_det);
    const int stride = line_stride(n);
    int R = lines_per_chunk > 0 ? lines_per_chunk : default_lines(n, sizeof(float2), 34 * 1024);
    R = std::max(4, std::min(R, ((n + 3) / 4) * 4));
    R = (R / 4) * 4;
    const size_t shm = (size_t)R * stride * sizeof(float2);
    if (shm > 64 * 1024) return SKEI_ERANGE;
    const dim3 grid(m, batch, c.nseg);
    if (yfull)
        return fwd_dispatch<kResidSub>(c, grid, shm, st, x, n, n_det, idx, m, g->tab, R, stride, y, yfull,
                                       g->n_angles, partial);
    return fwd_dispatch<kPlain>(c, grid, shm, st, x, n, n_det, idx, m, g->tab, R, stride, y, nullptr,
                                g->n_angles, nullptr);
}

int launch_bp_T(const skei_geom *g, const float *x, int batch, const int32_t *idx, int m, float *q,
                int lines_per_chunk, hipStream_t st)
{
    const int n = g->n, n_det = g->n_det;
    const RayCfg c = ray_config(n_det);
    const int stride = line_stride(n);
    int R = lines_per_chunk > 0 ? lines_per_chunk : default_lines(n, sizeof(float), 34 * 1024);
    R = std::max(4, std::min(R, ((n + 3) / 4) * 4));
    R = (R / 4) * 4;
    const size_t shm = (size_t)R * stride * sizeof(float);
    if (shm > 64 * 1024) return SKEI_ERANGE;
    const dim3 grid(m, batch, c.nseg);
#define SKEI_BPT_CASE(P)                                                                                     \
    case P:                                                                                                  \
        hipLaunchKernelGGL((k_bp_T<P>), grid, dim3(c.block), shm, st, x, n, n_det, idx, m, g->tab, R, stride, \
                           c.seg, q);                                                                        \
        break;
    switch (c.rpt) {
        SKEI_BPT_CASE(1)
        SKEI_BPT_CASE(2)
        SKEI_BPT_CASE(3)
        SKEI_BPT_CASE(4)
        SKEI_BPT_CASE(5)
        SKEI_BPT_CASE(6)
        SKEI_BPT_CASE(7)
        SKEI_BPT_CASE(8)
    default: return SKEI_ERANGE;
    }
#undef SKEI_BPT_CASE
    return check_launch();
}

}  // namespace skei

// Ray-driven kernels: Joseph forward projection A_S and the transpose B_S^T of
// the pixel-driven FBP backprojection.
//
// A workgroup owns a group of G consecutive listed angles of one image and one
// detector segment; its rays are (angle, detector) pairs, i.e. families of
// parallel lines that cross every image line along the angle's major axis.
// The image is streamed through LDS in chunks of R lines -- rows for angles
// that Joseph steps along rows, columns (transposed on the way in) for the
// others, in two passes when a group straddles 45 or 135 degrees -- so every
// tap is an LDS read and the G angles share each staged chunk.  Only the span
// of each line that the group's rays can touch is staged.
//
// Ray positions are 32.32 fixed-point numbers stepped by exact integer adds
// (u(k, M+1) = u(k, M) + du), so the interpolation position carries no
// rounding that grows with the image size; out-of-image taps are clamped onto
// zero-padded LDS borders instead of being branched around.  Sums are kept in
// float over aligned 16-line blocks (forward) or a line (B^T) and in double
// across them, so results do not depend on the launch shape.
//
// Workgroups are mapped XCD-major: consecutive work items (same image) go to
// the same XCD, so each XCD's L2 holds only its share of the images.
#include <algorithm>

#include "skei_internal.h"

namespace skei {
namespace {

constexpr int kBlock = 256;                  // threads per workgroup
constexpr int kMaxG = 8;                     // listed angles per workgroup
constexpr int kRaysMax = 8 * kBlock;         // rays per workgroup (8 per thread)
constexpr float kTwoM32 = 2.3283064365386963e-10f;   // 2^-32

enum Kind : int { kFwd = 0, kBpT = 1 };

struct Plan {
    int G, nseg, seg, rpt, R, stride, ngroups;
    long long total;
    size_t shm;
};

int line_stride(int n)
{
    const int s = n + 2 * kLinePad;
    return (s % 2 == 0) ? s + 1 : s;         // odd stride: transposed staging spreads over banks
}

// Launch plan.  elem = bytes per staged LDS entry (8: value/difference pairs,
// 4: plain values); `units_per_line` bounds the staged entries of a line.
int make_plan(const skei_geom *g, int batch, int m, const RayTune &t, size_t elem, Plan &p)
{
    const int n = g->n, nd = g->n_det;
    const long long base_items = (long long)batch * m;
    int G = t.group > 0 ? t.group : (base_items >= 2048 ? 4 : base_items >= 1024 ? 2 : 1);
    G = std::max(1, std::min(std::min(G, kMaxG), m));
    int nseg = t.split > 0 ? t.split : ((base_items < 512 && nd >= 128) ? 2 : 1);
    nseg = std::max(1, std::min(nseg, nd));
    for (;;) {
        const int seg = (nd + nseg - 1) / nseg;
        if ((long long)G * seg <= kRaysMax) break;
        if (G > 1)
            G--;
        else
            nseg++;
    }
    p.G = G;
    p.nseg = nseg;
    p.seg = (nd + nseg - 1) / nseg;
    p.rpt = (G * p.seg + kBlock - 1) / kBlock;
    p.stride = line_stride(n);
    const int r_lds = (int)((size_t)(34 * 1024) / ((size_t)p.stride * elem));
    int R = std::min(std::max(r_lds, 1), std::min(64, n));
    if (t.lines > 0) R = std::min(R, t.lines);
    if (R < 1) return SKEI_ERANGE;
    if (R >= 8) R &= ~3;                      // keep chunk starts 16-byte aligned when possible
    p.R = R;
    p.shm = (size_t)R * p.stride * elem;
    if (p.shm > 64 * 1024) return SKEI_ERANGE;
    p.ngroups = (m + G - 1) / G;
    p.total = (long long)batch * p.ngroups * p.nseg;
    return SKEI_OK;
}

// XCD-major work mapping: workgroup L runs on XCD L % 8; work items are split
// into 8 contiguous ranges, one per XCD.  Returns false for padding groups.
__device__ __forceinline__ bool decode_item(long long total, long long &item)
{
    const long long L = blockIdx.x;
    const long long per = (total + 7) >> 3;
    const long long pos = L >> 3;
    item = (L & 7) * per + pos;
    return pos < per && item < total;
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

// Major-axis lines [lo, hi] on which a ray's minor coordinate u0 + M*du lies
// in (-2, n+1), widened by one line for rounding; empty -> lo > hi.
__device__ __forceinline__ void ray_range(float u0, float du, int n, int &lo, int &hi)
{
    const float a = -2.0f, b = (float)n + 1.0f;
    if (fabsf(du) < 1e-12f) {
        const bool in = u0 > a && u0 < b;
        lo = in ? 0 : n;
        hi = in ? n - 1 : -1;
        return;
    }
    const float t1 = (a - u0) / du, t2 = (b - u0) / du;
    lo = (int)fmaxf(floorf(fminf(t1, t2)) - 1.0f, 0.0f);
    hi = (int)fminf(ceilf(fmaxf(t1, t2)) + 1.0f, (float)(n - 1));
}

// Index walk over a flattened (outer, inner) space: each thread starts at
// element `tid` and advances by kBlock elements with a carry (no division in
// the loops).
struct Walk {
    int o, i;
    __device__ Walk(int tid, int inner) : o(tid / inner), i(tid % inner) {}
    __device__ __forceinline__ void step(int so, int si, int inner)
    {
        i += si;
        o += so;
        if (i >= inner) {
            i -= inner;
            o += 1;
        }
    }
};

// Staging of lines [M0, M0+Rc), minor positions [cl, cl+W).  Row mode: lanes
// run along a row (coalesced loads, consecutive LDS entries).  Column mode:
// lanes run across the chunk's columns (coalesced loads of each row segment;
// the odd line stride spreads the transposed LDS writes over the banks).
// PAIRS entries hold (v[j], (v[j+1] - v[j]) * 2^-32) for the fixed-point
// fraction; plain entries hold v[j].  Latency is hidden by the other
// workgroups resident on the CU, not by registers.
template <bool PAIRS, typename T>
__device__ __forceinline__ void stage(T *lds, int stride, const float *__restrict__ img, int n, bool rows, int M0,
                                      int Rc, int cl, int W)
{
    const int tid = threadIdx.x;
    const int total = Rc * W;
    if (total <= 0) return;
    const int inner = rows ? W : Rc;
    Walk w(tid, inner);
    const int so = kBlock / inner, si = kBlock % inner;
    for (int e = tid; e < total; e += kBlock, w.step(so, si, inner)) {
        const int line = rows ? w.o : w.i;
        const int pos = cl + (rows ? w.i : w.o);
        const float *p0;
        size_t next;
        if (rows) {
            p0 = img + (size_t)(M0 + line) * n + pos;
            next = 1;
        } else {
            p0 = img + (size_t)pos * n + M0 + line;
            next = (size_t)n;
        }
        const float v = (pos >= 0 && pos < n) ? p0[0] : 0.0f;
        T *d = lds + line * stride + kLinePad + pos;
        if constexpr (PAIRS) {
            const float nx = (pos + 1 < n) ? p0[next] : 0.0f;
            *d = make_float2(v, (nx - v) * kTwoM32);
        } else {
            *d = v;
        }
    }
}

template <typename T>
__device__ __forceinline__ void zero_borders(T *lds, int n, int stride, int R)
{
    const int nb = stride - n;   // border entries per line: [0, PAD) and [PAD+n, stride)
    for (int e = threadIdx.x; e < R * nb; e += kBlock) {
        const int l = e / nb, p = e - l * nb;
        lds[l * stride + (p < kLinePad ? p : n + p)] = T{};
    }
}

// Minor-axis span touched by the group's rays of one pass over lines [M0, M0+Rc).
__device__ __forceinline__ void chunk_span(const AngleRow *ang, int gcount, int pass, int k0, int k1, int M0, int Rc,
                                           int n, int lo_clip, int &cl, int &W)
{
    float umin = 3.0e38f, umax = -3.0e38f;
    const float fk0 = (float)k0, fk1 = (float)k1, fm0 = (float)M0, fm1 = (float)(M0 + Rc - 1);
    for (int g = 0; g < gcount; g++) {
        const AngleRow &A = ang[g];
        if (A.rows != pass) continue;
        const float a0 = fmaf(fk0, A.inv_m, A.base), a1 = fmaf(fk1, A.inv_m, A.base);
        const float c00 = fmaf(fm0, A.du, a0), c01 = fmaf(fm1, A.du, a0);
        const float c10 = fmaf(fm0, A.du, a1), c11 = fmaf(fm1, A.du, a1);
        umin = fminf(umin, fminf(fminf(c00, c01), fminf(c10, c11)));
        umax = fmaxf(umax, fmaxf(fmaxf(c00, c01), fmaxf(c10, c11)));
    }
    const float lo = fmaxf(floorf(umin) - 3.0f, (float)lo_clip);
    const float hi = fminf(floorf(umax) + 4.0f, (float)(n - 1));
    if (!(hi >= lo)) {
        cl = 0;
        W = 0;
        return;
    }
    cl = (int)lo;
    W = (int)hi - cl + 1;
}

// ---------------------------------------------------------------------------
// KIND kFwd: y[b][r][k] = (1/w) sum_M lerp(line_M, u(k, M))       (Joseph A_S)
//   MODE kResidSub: y = yfull[b][idx[r]][k] - that, in double; partial[] = sum y^2.
// KIND kBpT: q[b][r][k] = sum_M sum_j Lambda(w (j - u(k, M))) line_M[j]    (B_S^T)
//   The pixels within unit distance of the ray in s are the (at most three)
//   entries within 1/w of u; the four candidates j0-1 .. j0+2 cover them.
// ---------------------------------------------------------------------------
template <int KIND, int RPT, int MODE, typename OUT>
__global__ void __launch_bounds__(kBlock) k_ray(const float *__restrict__ x, int n, int n_det,
                                                const int32_t *__restrict__ idx, int m,
                                                const AngleRow *__restrict__ tab, int G, int nseg, int seg,
                                                int ngroups, long long total, int R, int stride,
                                                OUT *__restrict__ y, const float *__restrict__ yfull, int n_angles,
                                                double *__restrict__ partial)
{
    constexpr bool PAIRS = KIND == kFwd;
    // Lowest tap entry read: j0 for the forward walk, j0 - 1 for B^T; taps
    // below -kLinePad (and above n + 1) are clamped onto the zero borders.
    constexpr int kBias = PAIRS ? kLinePad : kLinePad - 1;
    using Entry = typename std::conditional<PAIRS, float2, float>::type;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    Entry *lds = reinterpret_cast<Entry *>(lds_raw);
    __shared__ AngleRow ang[kMaxG];
    __shared__ int wrange[2][kBlock / 64];
    __shared__ double red[kBlock / 64];

    long long item;
    if (!decode_item(total, item)) return;
    const int per_img = ngroups * nseg;
    const int b = (int)(item / per_img);
    const int rem = (int)(item - (long long)b * per_img);
    const int grp = rem / nseg, sg = rem - grp * nseg;
    const int r0 = grp * G, gcount = min(G, m - r0);
    const int k_begin = sg * seg, k_len = min(seg, n_det - k_begin);
    const int tid = threadIdx.x;
    if (tid < gcount) ang[tid] = tab[idx[r0 + tid]];
    zero_borders(lds, n, stride, R);
    __syncthreads();
    const float *img = x + (size_t)b * n * n;

    int rg[RPT], rk[RPT];
    double accd[RPT];
#pragma unroll
    for (int q = 0; q < RPT; q++) {
        const int t = tid + q * kBlock;
        const bool valid = t < gcount * k_len;
        rg[q] = valid ? t / k_len : -1;
        rk[q] = valid ? k_begin + (t - rg[q] * k_len) : 0;
        accd[q] = 0.0;
    }

    for (int pass = 1; pass >= 0; --pass) {
        bool any = false;
        for (int g = 0; g < gcount; g++) any |= ang[g].rows == pass;
        if (!any) continue;

        // Rays of the other branch (and padding rays) are parked far outside
        // the image with a zero step: they read zero borders and add nothing.
        int64_t u[RPT], du[RPT];
        float facc[RPT], wg[RPT], c1[RPT], c2[RPT];
        int lo = n, hi = -1;
#pragma unroll
        for (int q = 0; q < RPT; q++) {
            const bool act = rg[q] >= 0 && ang[rg[q] < 0 ? 0 : rg[q]].rows == pass;
            const AngleRow &A = ang[rg[q] < 0 ? 0 : rg[q]];
            if (act) {
                int l0, h0;
                ray_range(fmaf((float)rk[q], A.inv_m, A.base), A.du, n, l0, h0);
                lo = min(lo, l0);
                hi = max(hi, h0);
            }
            // biased by kBias lines so that tap indices are non-negative inside
            // the padded line; a single unsigned min then clamps both ends
            u[q] = act ? A.base_fx + (int64_t)rk[q] * A.inv_fx + ((int64_t)kBias << 32) : -((int64_t)1 << 44);
            du[q] = act ? A.du_fx : 0;
            facc[q] = 0.0f;
            wg[q] = A.w * kTwoM32;
            c1[q] = 1.0f - A.w;
            c2[q] = 1.0f - 2.0f * A.w;
        }
        lo = __builtin_amdgcn_readfirstlane(wave_min(lo));
        hi = __builtin_amdgcn_readfirstlane(wave_max(hi));
        if ((tid & 63) == 0) {
            wrange[0][tid >> 6] = lo;
            wrange[1][tid >> 6] = hi;
        }
        __syncthreads();
        int blo = n, bhi = -1;
        for (int w = 0; w < kBlock / 64; w++) {
            blo = min(blo, wrange[0][w]);
            bhi = max(bhi, wrange[1][w]);
        }
#pragma unroll
        for (int q = 0; q < RPT; q++) u[q] += (int64_t)lo * du[q];   // position at the wave's first line

        const bool rows = pass == 1;
        const int lo_clip = PAIRS ? -1 : 0;
        const int k_last = k_begin + k_len - 1;
        for (int c = (blo <= bhi ? blo / R : 1), c_last = (blo <= bhi ? bhi / R : 0); c <= c_last; c++) {
            const int M0 = c * R, Rc = min(R, n - M0);
            int cl, W;
            chunk_span(ang, gcount, pass, k_begin, k_last, M0, Rc, n, lo_clip, cl, W);
            __syncthreads();
            stage<PAIRS>(lds, stride, img, n, rows, M0, Rc, cl, W);
            __syncthreads();
            const int lb = max(lo, M0), le = min(hi, M0 + Rc - 1);
            for (int M = lb; M <= le; M++) {
                // entry j of the line sits at index j + kBias of `line`
                const Entry *line = lds + (M - M0) * stride + kLinePad - kBias;
#pragma unroll
                for (int q = 0; q < RPT; q++) {
                    const unsigned jb = min((unsigned)(int)(u[q] >> 32), (unsigned)(n + 1 + kBias));
                    const float fr = (float)(uint32_t)u[q];
                    u[q] += du[q];
                    if constexpr (KIND == kFwd) {
                        const float2 e = line[jb];
                        facc[q] += e.x;
                        facc[q] = fmaf(fr, e.y, facc[q]);
                    } else {
                        const float *e = line + jb;
                        const float gq = fr * wg[q];
                        const float wa = fmaxf(c1[q] - gq, 0.0f);   // j0-1: 1 - w (1 + f)
                        const float wb = 1.0f - gq;                 // j0  : 1 - w f
                        const float wc = c1[q] + gq;                // j0+1: 1 - w (1 - f)
                        const float wd = fmaxf(c2[q] + gq, 0.0f);   // j0+2: 1 - w (2 - f)
                        float ls = wa * e[-1];
                        ls = fmaf(wb, e[0], ls);
                        ls = fmaf(wc, e[1], ls);
                        ls = fmaf(wd, e[2], ls);
                        accd[q] += (double)ls;
                    }
                }
                if constexpr (KIND == kFwd) {
                    // float partial sums over fixed, aligned 16-line blocks: the
                    // rounding does not depend on chunking, grouping or splits
                    if ((M & 15) == 15) {
#pragma unroll
                        for (int q = 0; q < RPT; q++) {
                            accd[q] += (double)facc[q];
                            facc[q] = 0.0f;
                        }
                    }
                }
            }
        }
        if constexpr (KIND == kFwd) {
#pragma unroll
            for (int q = 0; q < RPT; q++) accd[q] += (double)facc[q];
        }
        __syncthreads();
    }

    double ss = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; q++) {
        if (rg[q] < 0) continue;
        const AngleRow &A = ang[rg[q]];
        const size_t o = ((size_t)b * m + r0 + rg[q]) * n_det + rk[q];
        if constexpr (KIND == kFwd) {
            double v = accd[q] * A.scale;
            if (MODE == kResidSub) {
                const int a = idx[r0 + rg[q]];
                v = (double)yfull[((size_t)b * n_angles + a) * n_det + rk[q]] - v;
                const float vf = (float)v;
                ss += (double)vf * (double)vf;
                y[o] = vf;
            } else {
                y[o] = (OUT)v;
            }
        } else {
            y[o] = (OUT)accd[q];
        }
    }
    if (MODE == kResidSub) {
        ss = wave_sum(ss);
        if ((tid & 63) == 0) red[tid >> 6] = ss;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < kBlock / 64; w++) s += red[w];
            partial[item] = s;
        }
    }
}

template <int KIND, int MODE, typename OUT>
int ray_launch(const Plan &p, hipStream_t st, const float *x, int n, int n_det, const int32_t *idx, int m,
               const AngleRow *tab, OUT *y, const float *yfull, int n_angles, double *partial)
{
    const long long per = (p.total + 7) / 8;
    if (8 * per > 0x7fffffffLL) return SKEI_ERANGE;
    const dim3 grid((unsigned)(8 * per)), block(kBlock);
#define SKEI_RAY_CASE(P)                                                                                       \
    case P:                                                                                                    \
        hipLaunchKernelGGL((k_ray<KIND, P, MODE, OUT>), grid, block, p.shm, st, x, n, n_det, idx, m, tab, p.G, \
                           p.nseg, p.seg, p.ngroups, p.total, p.R, p.stride, y, yfull, n_angles, partial);     \
        break;
    switch (p.rpt) {
        SKEI_RAY_CASE(1)
        SKEI_RAY_CASE(2)
        SKEI_RAY_CASE(3)
        SKEI_RAY_CASE(4)
        SKEI_RAY_CASE(5)
        SKEI_RAY_CASE(6)
        SKEI_RAY_CASE(7)
        SKEI_RAY_CASE(8)
    default: return SKEI_ERANGE;
    }
#undef SKEI_RAY_CASE
    return check_launch();
}

}  // namespace

size_t radon_fwd_partials(const skei_geom *g, int batch, int m, const RayTune &tune)
{
    Plan p;
    if (make_plan(g, batch, m, tune, sizeof(float2), p) != SKEI_OK) return 0;
    return (size_t)p.total;
}

int launch_radon_fwd(const skei_geom *g, const float *x, int batch, const int32_t *idx, int m, float *y,
                     const float *yfull, double *partial, const RayTune &tune, hipStream_t st)
{
    Plan p;
    int rc = make_plan(g, batch, m, tune, sizeof(float2), p);
    if (rc) return rc;
    if (yfull)
        return ray_launch<kFwd, kResidSub, float>(p, st, x, g->n, g->n_det, idx, m, g->tab, y, yfull, g->n_angles,
                                                  partial);
    return ray_launch<kFwd, kPlain, float>(p, st, x, g->n, g->n_det, idx, m, g->tab, y, nullptr, g->n_angles,
                                           nullptr);
}

int launch_bp_T(const skei_geom *g, const float *x, int batch, const int32_t *idx, int m, float *qf, double *qd,
                const RayTune &tune, hipStream_t st)
{
    Plan p;
    int rc = make_plan(g, batch, m, tune, sizeof(float), p);
    if (rc) return rc;
    if (qd)
        return ray_launch<kBpT, kPlain, double>(p, st, x, g->n, g->n_det, idx, m, g->tab, qd, nullptr, g->n_angles,
                                                nullptr);
    return ray_launch<kBpT, kPlain, float>(p, st, x, g->n, g->n_det, idx, m, g->tab, qf, nullptr, g->n_angles,
                                           nullptr);
}

}  // namespace skei

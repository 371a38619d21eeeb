// Ray-driven kernels: Joseph forward projection A_S and the transpose B_S^T of
// the pixel-driven FBP backprojection.
//
// A workgroup owns a group of G consecutive listed angles of one image and one
// detector segment; its rays are (angle, detector) pairs, i.e. families of
// parallel lines that cross every image line along the angle's major axis.
// The image is streamed through LDS in chunks of R lines -- rows for angles
// that Joseph steps along rows, columns for the others (two passes when a
// group straddles 45 or 135 degrees) -- so every tap is an LDS read and the G
// angles share each staged chunk.
//
// Staging uses the LDS DMA path (global_load_lds): each wave instruction
// moves a contiguous run of a line straight from global memory into LDS, no
// registers involved -- 16-byte lanes along image rows, 4-byte lanes gathering
// a column (which lands transposed, i.e. line-contiguous, in LDS).  One
// buffer of two march units' height is staged, then marched; the DMA latency
// is covered by the other workgroups of the CU (two alternating half-height
// buffers measured slower: their per-chunk bookkeeping costs more than the
// latency they hide).  Only the span of each line that the group's rays can
// touch is staged.
//
// Ray positions are 32.32 fixed-point numbers stepped by exact integer adds
// (u(k, M+1) = u(k, M) + du), so the interpolation position carries no
// rounding that grows with the image size; out-of-image taps are clamped onto
// zero LDS borders instead of being branched around.  Sums are kept in float
// over aligned 16-line blocks and in double across them; the forward
// residual jobs (y - A x) use aligned 4-line float sums.  So results do not
// depend on the launch shape.
//
// In B^T a wave's rays come in blocks of 64 consecutive detectors, and each
// block marches only the lines its rays cross: rays near the edge of an
// angle's image shadow cross few lines.
//
// Workgroups are mapped XCD-major: consecutive work items (same image) go to
// the same XCD, so each XCD's L2 holds only its share of the images.
#include <algorithm>

#include "skei_internal.h"
#include "work.h"

namespace skei {
namespace {

typedef __attribute__((address_space(1))) const void gmem_t;
typedef __attribute__((address_space(3))) void lmem_t;

constexpr int kMaxWaves = 8;                 // waves per workgroup: 3, 4, 6 or 8
constexpr int kMaxG = 8;                     // listed angles per workgroup
constexpr int kMaxRpt = 4;                   // rays per thread
constexpr size_t kLdsBudget = 40 * 1024;     // staging buffer (default)
constexpr size_t kLdsMax = 160 * 1024;       // LDS of one CU (gfx950)
constexpr float kTwoM32 = 2.3283064365386963e-10f;   // 2^-32

enum Kind : int { kFwd = 0, kBpT = 1 };

// LDS line pitch in floats: kLinePad zero entries on each side, 16-byte multiple.
int line_pitch(int n) { return ((n + 2 * kLinePad) + 3) & ~3; }

}  // namespace

// Host walk of the tap positions the march reads within a staged line of an
// n-pixel image, for both kinds, from the kernel's bias and clamp constants:
// out = {lowest position, highest position, line pitch}.  Tap indices are
// clamped to [0, n + 1 + bias] by one unsigned min; positions beyond the
// image land on the zeroed pads.
void ray_lds_reads(int n, long long out[3])
{
    long long lo = 1LL << 60, hi = -1;
    for (int kind = 0; kind < 2; kind++) {
        const int bias = kind == kFwd ? kLinePad : kLinePad - 1;   // kBias of ray_item
        const long long cap = n + 1 + bias;
        const long long base = kLinePad - bias;   // `line` = start of the staged line + base
        const int first = kind == kFwd ? 0 : -1, taps = kind == kFwd ? 2 : 3;
        for (long long jb : {0LL, cap}) {
            lo = std::min(lo, base + jb + first);
            hi = std::max(hi, base + jb + first + taps - 1);
        }
    }
    out[0] = lo;
    out[1] = hi;
    out[2] = line_pitch(n);
}

int make_ray_job(const skei_geom *g, const float *x, const float *xT, int batch, const int32_t *idx, int m, void *y,
                 const float *yfull, const RayTune &t, int rpt_cap, RayJob &J, RayShape &shape)
{
    const int n = g->n, nd = g->n_det;
    const long long base_items = (long long)batch * m;
    // A launch of a few rows (one image sketched to a few angles) is as long
    // as one item's march over every image line: one angle per item and rows
    // cut into segments of ~60 detectors put more workgroups on that march,
    // up to ~640 items (measured on MI355X, the forward of one image: 512^2,
    // 726 detectors, 12 segments, 100.6 -> 62.4 us at 5 angles, 102.6 ->
    // 75.5 us at 50, slower at 100; 256^2, 363 detectors, 6 segments, 75.3 ->
    // 35.9 us at 36 angles and 75.7 -> 45.0 us at 72, slower at 360)
    const int few_seg = std::min(16, nd / 60);
    const bool few = rpt_cap == 0 && t.split == 0 && t.group == 0 && nd >= 300 && base_items * few_seg <= 640;
    // listed angles per item (G) and detector segments (nseg) for workgroups
    // of `w` waves; returns the fraction of ray slots that hold a ray
    auto layout = [&](int w, int &G, int &nseg) {
        const int block = 64 * w;
        const int cap = (rpt_cap > 0 ? std::min(rpt_cap, kMaxRpt) : kMaxRpt) * block;
        nseg = t.split > 0 ? t.split
               : few       ? few_seg
               : rpt_cap > 0 ? (nd + cap - 1) / cap : ((base_items < 512 && nd >= 128) ? 2 : 1);
        nseg = std::max(1, std::min(nseg, nd));
        G = t.group > 0 ? t.group
            : few       ? 1
                        : std::max(1, (rpt_cap > 0 ? cap : 2 * block) / ((nd + nseg - 1) / nseg));
        G = std::max(1, std::min(std::min(G, kMaxG), m));
        for (;;) {
            const int seg = (nd + nseg - 1) / nseg;
            if ((long long)G * seg <= cap) break;
            if (G > 1)
                G--;
            else
                nseg++;
        }
        const int rays = G * ((nd + nseg - 1) / nseg);
        return (double)rays / (double)(((rays + block - 1) / block) * block);
    };
    int G, nseg, waves = (t.waves == 3 || t.waves == 6 || t.waves == 8) ? t.waves : 4;
    double fill = layout(waves, G, nseg);
    if (t.waves == 0) {
        // automatic: three waves when they leave fewer ray slots empty
        int G3, nseg3;
        if (layout(3, G3, nseg3) > fill + 0.05) {
            waves = 3;
            G = G3;
            nseg = nseg3;
        }
    }
    const int block = 64 * waves;
    J = RayJob{};
    J.x = x;
    J.xT = xT;
    J.idx = idx;
    J.tab = g->tab;
    J.y = y;
    J.yfull = yfull;
    J.n = n;
    J.n_det = nd;
    J.m = m;
    J.n_angles = g->n_angles;
    J.G = G;
    J.nseg = nseg;
    J.seg = (nd + nseg - 1) / nseg;
    J.ngroups = (m + G - 1) / G;
    J.pitch = line_pitch(n);
    // lines per unrolled march unit: the largest of 16, 8, 4 whose two
    // two-unit staging buffer fits the LDS budget (4 always fits in 64 KB)
    const size_t line_bytes = (size_t)J.pitch * sizeof(float);
    int U = 2 * 16 * line_bytes <= kLdsBudget ? 16 : 2 * 8 * line_bytes <= kLdsBudget ? 8 : 4;
    size_t budget = std::max(kLdsBudget, 2 * (size_t)U * line_bytes);
    if (t.lines > 0) {
        // a requested chunk height sets the unit (16, 8 or 4 lines) and may
        // spend up to the whole LDS of a CU on the buffer
        U = t.lines >= 16 ? 16 : t.lines >= 8 ? 8 : 4;
        budget = std::min(kLdsMax, std::max(2 * (size_t)U * line_bytes, 2 * (size_t)t.lines * line_bytes));
        if (2 * (size_t)U * line_bytes > budget) return SKEI_ERANGE;
    }
    int R = (int)(budget / (2 * line_bytes));
    R = std::min(R, t.lines > 0 ? t.lines : 64);
    R = std::max(U, R / U * U);   // whole units per half
    // one staging buffer of 2R lines (whole units; 4R on request): staged,
    // then marched -- measured ahead of two alternating R-line buffers, whose
    // per-chunk bookkeeping costs more than the DMA latency they hide
    J.R = (t.units == 4 ? 4 : 2) * R;
    shape.unroll = U;
    J.resid = yfull != nullptr;
    J.items = (long long)batch * J.ngroups * J.nseg;
    shape.rpt = (G * J.seg + block - 1) / block;
    shape.waves = waves;
    shape.shm = (size_t)J.R * J.pitch * sizeof(float);
    if (shape.shm > kLdsMax || shape.rpt > (waves > 4 ? 2 : kMaxRpt)) return SKEI_ERANGE;
    return SKEI_OK;
}

namespace {

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

// Minor-axis extent of the group's rays of one pass, per listed angle: lane
// g (< gcount) holds angle g's extent at line 0 over detectors [k0, k1] and
// its drift per line; lanes without an angle of this pass hold an empty one.
struct Span {
    float amin, amax, du;
};

__device__ __forceinline__ Span span_setup(const AngleRow *ang, int gcount, int pass, int k0, int k1)
{
    const int g = threadIdx.x & 63;
    Span sp{3.0e38f, -3.0e38f, 0.0f};
    if (g < gcount && ang[g].rows == pass) {
        const AngleRow &A = ang[g];
        const float a0 = fmaf((float)k0, A.inv_m, A.base), a1 = fmaf((float)k1, A.inv_m, A.base);
        sp.amin = fminf(a0, a1);
        sp.amax = fmaxf(a0, a1);
        sp.du = A.du;
    }
    return sp;
}

// Minor-axis span [cl, cl+W) within [0, n) touched by the group's rays of one
// pass over lines [M0, M0+Rc): the union of the angles' extents (gathered
// across lanes with readlane, no LDS traffic), widened by 3 entries each
// side, and aligned to 4 entries for 16-byte DMA lanes.
__device__ __forceinline__ void chunk_span(const Span &sp, int gcount, int M0, int Rc, int n, int &cl, int &W)
{
    const float d0 = sp.du * (float)M0, d1 = sp.du * (float)(M0 + Rc - 1);
    const float lo = sp.amin + fminf(d0, d1), hi = sp.amax + fmaxf(d0, d1);
    float umin = 3.0e38f, umax = -3.0e38f;
    for (int g = 0; g < gcount; g++) {
        umin = fminf(umin, __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lo), g)));
        umax = fmaxf(umax, __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hi), g)));
    }
    const float flo = fmaxf(floorf(umin) - 3.0f, 0.0f);
    const float fhi = fminf(floorf(umax) + 4.0f, (float)(n - 1));
    if (!(fhi >= flo)) {
        cl = 0;
        W = 0;
        return;
    }
    cl = ((int)flo) & ~3;
    W = (int)fhi - cl + 1;
}

// DMA of lines [M0, M0+Rc), positions [cl, cl+W), into LDS buffer `buf`
// (entry p of line l at buf[l*pitch + kLinePad + p]).  Rows: each lane moves
// 16 bytes (4 consecutive entries; n % 4 == 0 and cl % 4 == 0), 256 entries
// per wave instruction.  Columns: each lane gathers one entry of the column,
// 64 consecutive rows per wave instruction.  Lanes past the span are masked.
template <int NW>
__device__ __forceinline__ void stage_dma(float *buf, int pitch, const float *__restrict__ img, int n, bool rows,
                                          int M0, int Rc, int cl, int W)
{
    if (W <= 0) return;
    const int lane = threadIdx.x & 63;
    // wave-uniform bookkeeping lives in scalar registers: wave w stages lines
    // w, w + NW, ... of the chunk, each in segments of one DMA instruction
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float *dst = buf + wave * pitch + kLinePad + cl;
    const int dst_step = NW * pitch;
    if (rows && (n & 3) == 0) {
        const int S = (W + 255) >> 8;
        const int off = 4 * lane;
        const float *src = img + (size_t)(M0 + wave) * n + cl;
        const size_t src_step = (size_t)NW * n;
        for (int l = wave; l < Rc; l += NW, src += src_step, dst += dst_step)
            for (int s = 0; s < S; s++) {
                const int p = s << 8;
                if (p + off < W)
                    __builtin_amdgcn_global_load_lds((gmem_t *)(src + p + off), (lmem_t *)(dst + p), 16, 0, 0);
            }
    } else {
        const int S = (W + 63) >> 6;
        // rows: entry p of line l at img[(M0 + l) n + p]; columns: at img[p n + M0 + l]
        const float *src = rows ? img + (size_t)(M0 + wave) * n + cl : img + (size_t)cl * n + M0 + wave;
        const size_t src_step = rows ? (size_t)NW * n : (size_t)NW;
        const size_t lane_step = rows ? (size_t)lane : (size_t)lane * n;
        const size_t seg_step = rows ? (size_t)64 : (size_t)64 * n;
        for (int l = wave; l < Rc; l += NW, src += src_step, dst += dst_step)
            for (int s = 0; s < S; s++) {
                const int p = s << 6;
                if (p + lane < W)
                    __builtin_amdgcn_global_load_lds((gmem_t *)(src + s * seg_step + lane_step), (lmem_t *)(dst + p),
                                                     4, 0, 0);
            }
    }
}

__device__ __forceinline__ void dma_wait() { __builtin_amdgcn_s_waitcnt(0); }

// Zeroes the lines [Rc, R) of a staging buffer: a partial last chunk leaves
// them unstaged, and whole-unit marches read them (they must add nothing).
template <int NW>
__device__ __forceinline__ void zero_tail(float *buf, int pitch, int R, int Rc)
{
    for (int e = Rc * pitch + threadIdx.x; e < R * pitch; e += 64 * NW) buf[e] = 0.0f;
}

// ---------------------------------------------------------------------------
// KIND kFwd: y[b][r][k] = (1/w) sum_M lerp(line_M, u(k, M))       (Joseph A_S)
//   resid jobs: y = yfull[b][idx[r]][k] - that, in double, with the lerps of
//   each aligned group of 4 lines summed in float and the groups in double.
// KIND kBpT: q[b][r][k] = sum_M sum_j Lambda(w (j - u(k, M))) line_M[j]    (B_S^T)
//   The pixels within unit distance of the ray in s are the entries within
//   1/w <= sqrt(2) of u.  With j1 = round(u) and g = u - j1 in [-1/2, 1/2),
//   j1 -+ 2 lie at least 3/2 away, so the three taps j1-1, j1, j1+1 cover
//   them: weights 1 - w (1 + g), 1 - w |g|, 1 - w (1 - g), clamped at 0.
// ---------------------------------------------------------------------------
template <int KIND, int RPT, int U, typename OUT, int NW>
__device__ __forceinline__ void ray_item(const RayJob &J, long long item, float *lds)
{
    constexpr int kBlock = 64 * NW, kWaves = NW;
    // Lowest tap entry read: j0 for the forward walk, j1 - 1 for B^T; taps
    // below -kLinePad (and above n + 1) are clamped onto the zero borders.
    constexpr int kBias = KIND == kFwd ? kLinePad : kLinePad - 1;
    __shared__ AngleRow ang[kMaxG];
    __shared__ int wrange[2][kMaxWaves];

    const float *__restrict__ x = J.x;
    const float *__restrict__ xT = J.xT;
    const int32_t *__restrict__ idx = J.idx;
    const AngleRow *__restrict__ tab = J.tab;
    OUT *__restrict__ y = static_cast<OUT *>(J.y);
    const float *__restrict__ yfull = J.yfull;
    const int n = J.n, n_det = J.n_det, m = J.m, n_angles = J.n_angles;
    const int G = J.G, nseg = J.nseg, seg = J.seg, ngroups = J.ngroups, R = J.R, pitch = J.pitch;
    const bool resid = KIND == kFwd && J.resid;
    const int per_img = ngroups * nseg;
    const int b = (int)(item / per_img);
    const int rem = (int)(item - (long long)b * per_img);
    const int grp = rem / nseg, sg = rem - grp * nseg;
    const int r0 = grp * G, gcount = min(G, m - r0);
    const int k_begin = sg * seg, k_len = min(seg, n_det - k_begin);
    const int tid = threadIdx.x;
    if (tid < gcount) ang[tid] = tab[idx[r0 + tid]];
    // Zero the pads of every line of the buffer: the DMA never writes them,
    // and clamped taps read them.  Entries of [0, n) outside a chunk's staged
    // span are never read (the span covers every tap of the group's rays).
    {
        const int padw = pitch - n;   // kLinePad before the line, the rest after it
        for (int e = tid; e < R * padw; e += kBlock) {
            const int l = e / padw, k = e - l * padw;
            lds[l * pitch + (k < kLinePad ? k : n + k)] = 0.0f;
        }
    }
    __syncthreads();
    const float *img = x + (size_t)b * n * n;

    // Ray slot of (thread, q).
    //  - B^T: the item's rays are cut into blocks of 64 consecutive (angle,
    //    detector) rays, one per (wave, q); lane l holds ray l of its block.
    //    Each (wave, q) block marches only the lines its own rays cross, so
    //    rays near the edge of an angle's shadow cost few lines.  Blocks are
    //    dealt boustrophedon (wave w takes blocks w, 2W-1-w, 2W+w, ...), which
    //    pairs an edge block with a central one in every wave.
    //  - Forward: blocks of 32 consecutive detectors are dealt round-robin to
    //    the waves, so every wave spans the whole detector range and marches
    //    the same lines, with a lane's RPT rays interleaved line by line (the
    //    forward tap is cheap, and marching the rays together shares the
    //    loop's scalar work between them).
    int rg[RPT], rk[RPT];
    double accd[RPT];
    const int wave_id = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int q = 0; q < RPT; q++) {
        int t;
        if constexpr (KIND == kFwd) {
            t = (lane & 31) + 32 * (wave_id + kWaves * (lane >> 5)) + q * kBlock;
        } else {
            const int blk = (q & 1) ? (q + 1) * kWaves - 1 - wave_id : q * kWaves + wave_id;
            t = 64 * blk + lane;
        }
        const bool valid = t < gcount * k_len;
        rg[q] = valid ? t / k_len : -1;
        rk[q] = valid ? k_begin + (t - rg[q] * k_len) : 0;
        accd[q] = 0.0;
    }

    for (int pass = 1; pass >= 0; --pass) {
        bool any = false;
        for (int g = 0; g < gcount; g++) any |= ang[g].rows == pass;
        if (!any) continue;
        const Span span = span_setup(ang, gcount, pass, k_begin, k_begin + k_len - 1);

        // Rays of the other branch (and padding rays) are parked far outside
        // the image with a zero step: they read zero borders and add nothing.
        int64_t u[RPT], du[RPT];
        float s0[RPT], s1[RPT], wg[RPT], cm[RPT], cp[RPT], hw[RPT];
        // line range of each ray; B^T keeps one per block (q), the forward
        // only the wave's union
        int lo[KIND == kFwd ? 1 : RPT], hi[KIND == kFwd ? 1 : RPT];
        lo[0] = n;
        hi[0] = -1;
#pragma unroll
        for (int q = 0; q < RPT; q++) {
            const int gq = rg[q] < 0 ? 0 : rg[q];
            const AngleRow &A = ang[gq];
            const bool act = rg[q] >= 0 && A.rows == pass;
            if constexpr (KIND == kFwd) {
                if (act) {
                    int l0, h0;
                    ray_range(fmaf((float)rk[q], A.inv_m, A.base), A.du, n, l0, h0);
                    lo[0] = min(lo[0], l0);
                    hi[0] = max(hi[0], h0);
                }
            } else {
                lo[q] = n;
                hi[q] = -1;
                if (act) ray_range(fmaf((float)rk[q], A.inv_m, A.base), A.du, n, lo[q], hi[q]);
            }
            // biased by kBias entries so that tap indices are non-negative
            // inside the padded line; one unsigned min clamps both ends
            // (B^T rounds to the nearest entry: its position carries +1/2)
            constexpr int64_t kHalf = KIND == kFwd ? 0 : (int64_t)1 << 31;
            u[q] = act ? A.base_fx + (int64_t)rk[q] * A.inv_fx + ((int64_t)kBias << 32) + kHalf
                       : -((int64_t)1 << 44);
            du[q] = act ? A.du_fx : 0;
            s0[q] = 0.0f;
            s1[q] = 0.0f;
            // with F = frac(u + 1/2) = g + 1/2:  1 - w (1 + g) = cm - w F,
            // 1 - w (1 - g) = cp + w F, and w g = w F + hw
            wg[q] = A.w * kTwoM32;
            cm[q] = 1.0f - 0.5f * A.w;
            cp[q] = 1.0f - 1.5f * A.w;
            hw[q] = -0.5f * A.w;
        }
        // each block's lines (wave-uniform), and the wave's union
        constexpr int kRanges = KIND == kFwd ? 1 : RPT;
        int wlo = n, whi = -1;
#pragma unroll
        for (int q = 0; q < kRanges; q++) {
            lo[q] = __builtin_amdgcn_readfirstlane(wave_min(lo[q]));
            hi[q] = __builtin_amdgcn_readfirstlane(wave_max(hi[q]));
            wlo = min(wlo, lo[q]);
            whi = max(whi, hi[q]);
        }
        if (lane == 0) {
            wrange[0][wave_id] = wlo;
            wrange[1][wave_id] = whi;
        }
        __syncthreads();
        int blo = n, bhi = -1;
        for (int w = 0; w < kWaves; w++) {
            blo = min(blo, wrange[0][w]);
            bhi = max(bhi, wrange[1][w]);
        }
        // A block marches whole U-line units, from the unit holding its first
        // line; on lines outside a ray's own range the ray reads zero borders.
        int ulo[kRanges];
#pragma unroll
        for (int q = 0; q < kRanges; q++) ulo[q] = lo[q] & ~(U - 1);
#pragma unroll
        for (int q = 0; q < RPT; q++) u[q] += (int64_t)ulo[KIND == kFwd ? 0 : q] * du[q];

        const bool rows = pass == 1;
        // column passes read rows of the transposed image when it is given
        const bool dma_rows = rows || xT != nullptr;
        const float *src = rows || !xT ? img : xT + (size_t)b * n * n;
        const unsigned cap = (unsigned)(n + 1 + kBias);
        if (blo <= bhi) {
            const int c_first = blo / R, c_last = bhi / R;
            for (int c = c_first; c <= c_last; c++) {
                const int M0 = c * R, Rc = min(R, n - M0);
                {
                    int cl, W;
                    chunk_span(span, gcount, M0, Rc, n, cl, W);
                    zero_tail<NW>(lds, pitch, R, Rc);
                    stage_dma<NW>(lds, pitch, src, n, dma_rows, M0, Rc, cl, W);
                    dma_wait();
                }
                __syncthreads();
                const float *chunk = lds;
                // Forward residual jobs sum the interpolated values of each
                // aligned group of 4 lines in float and the groups in double:
                // the data-consistency residual y - A x is ~1 % of y, so the
                // 16-line float block sums of A x would carry an error ~100x
                // larger relative to the residual.  Every grouping is fixed and
                // aligned, so the rounding does not depend on chunking or launch
                // shape.
                if constexpr (KIND == kFwd) {
                    // every ray of the wave over the wave's lines, RPT rays
                    // interleaved per line (M0 and ulo are multiples of U)
                    const int ub = max(ulo[0], M0), ue = min(whi, M0 + Rc - 1);
                    if (resid) {
                        // residual jobs: each line's lerp in float, four lines
                        // (aligned) summed in float, then added in double; the
                        // groups stay rolled: unrolled, the forward launch of
                        // one 512^2 image sketched to 5 or 10 angles (whose few
                        // residual items set its length) measured 81 -> 102 us
                        // on MI355X, with no gain at the 16-copy 256^2 step
                        // (traced 65.4 unrolled against 64.5 us)
#pragma unroll 1
                        for (int Mb = ub; Mb <= ue; Mb += U) {
                            // entry j of line Mb + l sits at index j + kBias of `line`
                            const float *ubase = chunk + (Mb - M0) * pitch + kLinePad - kBias;
#pragma unroll 1
                            for (int l4 = 0; l4 < U; l4 += 4) {
                                float v4[RPT];
#pragma unroll
                                for (int l = l4; l < l4 + 4; l++) {
                                    const float *line = ubase + l * pitch;
#pragma unroll
                                    for (int q = 0; q < RPT; q++) {
                                        const unsigned jb = min((unsigned)(int)(u[q] >> 32), cap);
                                        const float fi = (float)(uint32_t)u[q];   // fraction x 2^32
                                        u[q] += du[q];
                                        const float t0 = line[jb], t1 = line[jb + 1];
                                        const float v = fmaf(fi * kTwoM32, t1 - t0, t0);
                                        v4[q] = l == l4 ? v : v4[q] + v;
                                    }
                                }
#pragma unroll
                                for (int q = 0; q < RPT; q++) accd[q] += (double)v4[q];
                            }
                        }
                    } else {
                        for (int Mb = ub; Mb <= ue; Mb += U) {
                            const float *ubase = chunk + (Mb - M0) * pitch + kLinePad - kBias;
#pragma unroll
                            for (int l = 0; l < U; l++) {
                                const float *line = ubase + l * pitch;
#pragma unroll
                                for (int q = 0; q < RPT; q++) {
                                    const unsigned jb = min((unsigned)(int)(u[q] >> 32), cap);
                                    const float fi = (float)(uint32_t)u[q];   // fraction x 2^32
                                    u[q] += du[q];
                                    const float t0 = line[jb], t1 = line[jb + 1];
                                    s0[q] += t0;
                                    s1[q] = fmaf(fi, t1 - t0, s1[q]);
                                }
                            }
                            // float sums over fixed, aligned 16-line blocks
                            if (((Mb + U) & 15) == 0) {
#pragma unroll
                                for (int q = 0; q < RPT; q++) {
                                    accd[q] += fma((double)s1[q], (double)kTwoM32, (double)s0[q]);
                                    s0[q] = 0.0f;
                                    s1[q] = 0.0f;
                                }
                            }
                        }
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < RPT; q++) {
                        // units of this chunk that block q marches (M0 and ulo are multiples of U)
                        const int qr = KIND == kFwd ? 0 : q;
                        const int ub = max(ulo[qr], M0), ue = min(hi[qr], M0 + Rc - 1);
                        // Lines run in units of U inside fixed, aligned 16-line
                        // blocks; the float block sum goes to double once the
                        // block's last line is marched.  Each unit runs in two
                        // phases: every line's tap address and LDS loads first,
                        // then the weights and sums, so its loads are in flight
                        // together instead of one line at a time.
#pragma unroll 1
                        for (int Bb = ub & ~15; Bb <= ue; Bb += 16) {
                            const int u1 = min(ue, Bb + 15);
#pragma unroll 1
                            for (int Mb = max(ub, Bb); Mb <= u1; Mb += U) {
                                const float *ubase = chunk + (Mb - M0) * pitch + kLinePad - kBias;
                                float tap[U][3], fr[U];
#pragma unroll
                                for (int l = 0; l < U; l++) {
                                    const unsigned jb = min((unsigned)(int)(u[q] >> 32), cap);
                                    fr[l] = (float)(uint32_t)u[q];   // fraction x 2^32
                                    u[q] += du[q];
                                    const float *e = ubase + l * pitch + jb - 1;
#pragma unroll
                                    for (int t = 0; t < 3; t++) tap[l][t] = e[t];
                                }
#pragma unroll
                                for (int l = 0; l < U; l++) {
                                    const float fi = fr[l];
                                    // the clamps fold into the FMAs (weights are <= 1)
                                    const float wm = __builtin_amdgcn_fmed3f(fmaf(-fi, wg[q], cm[q]), 0.0f, 1.0f);
                                    const float w0 = 1.0f - fabsf(fmaf(fi, wg[q], hw[q]));
                                    const float wp = __builtin_amdgcn_fmed3f(fmaf(fi, wg[q], cp[q]), 0.0f, 1.0f);
                                    s0[q] = fmaf(wm, tap[l][0], s0[q]);
                                    s0[q] = fmaf(w0, tap[l][1], s0[q]);
                                    s0[q] = fmaf(wp, tap[l][2], s0[q]);
                                }
                            }
                            if (u1 == Bb + 15) {   // the block is complete
                                accd[q] += (double)s0[q];
                                s0[q] = 0.0f;
                            }
                        }
                    }
                }
                __syncthreads();   // the chunk is marched before the next one lands
            }
        } else {
            __syncthreads();
        }
#pragma unroll
        for (int q = 0; q < RPT; q++) {
            if constexpr (KIND == kFwd)
                accd[q] += fma((double)s1[q], (double)kTwoM32, (double)s0[q]);
            else
                accd[q] += (double)s0[q];
        }
    }

#pragma unroll
    for (int q = 0; q < RPT; q++) {
        if (rg[q] < 0) continue;
        const AngleRow &A = ang[rg[q]];
        const size_t o = ((size_t)b * m + r0 + rg[q]) * n_det + rk[q];
        if constexpr (KIND == kFwd) {
            double v = accd[q] * A.scale;
            if (resid) {
                const int a = idx[r0 + rg[q]];
                y[o] = (float)((double)yfull[((size_t)b * n_angles + a) * n_det + rk[q]] - v);
            } else {
                y[o] = (OUT)v;
            }
        } else {
            y[o] = (OUT)accd[q];
        }
    }
}

template <int KIND, int RPT, int U, typename OUT, int NW>
__global__ void __launch_bounds__(64 * NW) k_ray(const JobList<RayJob> L)
{
    extern __shared__ __align__(16) float lds[];
    for_each_item(L, [&](const RayJob &J, long long item) { ray_item<KIND, RPT, U, OUT, NW>(J, item, lds); });
}

// The forward projector with a register budget: its residual loop would
// otherwise raise the whole kernel's allocation (to ~90 VGPRs, 5 waves per
// SIMD), while the fast march needs ~70; a launch of a few thousand waves
// then no longer stays resident in one pass (measured 63 -> 75 us at 256^2).
template <int RPT, int U, int NW>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(RPT <= 2 ? 7 : 1)))
    k_ray_fwd(const JobList<RayJob> L)
{
    extern __shared__ __align__(16) float lds[];
    for_each_item(L, [&](const RayJob &J, long long item) { ray_item<kFwd, RPT, U, float, NW>(J, item, lds); });
}

template <int KIND, int RPT, int U, typename OUT, int NW>
int ray_launch1(size_t shm, const JobList<RayJob> &L, hipStream_t st)
{
    const void *fn = KIND == kFwd ? reinterpret_cast<const void *>(&k_ray_fwd<RPT, U, NW>)
                                  : reinterpret_cast<const void *>(&k_ray<KIND, RPT, U, OUT, NW>);
    const long long grid = launch_grid(L, fn, 64 * NW, shm);
    if (grid <= 0 || grid > 0x7fffffffLL) return SKEI_ERANGE;
    if constexpr (KIND == kFwd)
        hipLaunchKernelGGL((k_ray_fwd<RPT, U, NW>), dim3((unsigned)grid), dim3(64 * NW), shm, st, L);
    else
        hipLaunchKernelGGL((k_ray<KIND, RPT, U, OUT, NW>), dim3((unsigned)grid), dim3(64 * NW), shm, st, L);
    return check_launch();
}

template <int KIND, int U, typename OUT, int NW>
int ray_launch_u(int rpt, size_t shm, const JobList<RayJob> &L, hipStream_t st)
{
    switch (rpt) {
    case 1: return ray_launch1<KIND, 1, U, OUT, NW>(shm, L, st);
    case 2: return ray_launch1<KIND, 2, U, OUT, NW>(shm, L, st);
    case 3: return ray_launch1<KIND, 3, U, OUT, NW>(shm, L, st);
    case 4: return ray_launch1<KIND, 4, U, OUT, NW>(shm, L, st);
    default: return SKEI_ERANGE;
    }
}

template <int KIND, typename OUT, int NW>
int ray_launch_w(int rpt, int unroll, size_t shm, const JobList<RayJob> &L, hipStream_t st)
{
    switch (unroll) {
    case 16: return ray_launch_u<KIND, 16, OUT, NW>(rpt, shm, L, st);
    case 8: return ray_launch_u<KIND, 8, OUT, NW>(rpt, shm, L, st);
    case 4: return ray_launch_u<KIND, 4, OUT, NW>(rpt, shm, L, st);
    default: return SKEI_ERANGE;
    }
}

// Six- and eight-wave workgroups hold one or two rays per thread.
template <int KIND, typename OUT, int NW>
int ray_launch_wide(int rpt, int unroll, size_t shm, const JobList<RayJob> &L, hipStream_t st)
{
    if (rpt == 1) {
        switch (unroll) {
        case 16: return ray_launch1<KIND, 1, 16, OUT, NW>(shm, L, st);
        case 8: return ray_launch1<KIND, 1, 8, OUT, NW>(shm, L, st);
        case 4: return ray_launch1<KIND, 1, 4, OUT, NW>(shm, L, st);
        default: return SKEI_ERANGE;
        }
    }
    if (rpt == 2) {
        switch (unroll) {
        case 16: return ray_launch1<KIND, 2, 16, OUT, NW>(shm, L, st);
        case 8: return ray_launch1<KIND, 2, 8, OUT, NW>(shm, L, st);
        case 4: return ray_launch1<KIND, 2, 4, OUT, NW>(shm, L, st);
        default: return SKEI_ERANGE;
        }
    }
    return SKEI_ERANGE;
}

template <int KIND, typename OUT>
int ray_launch(const RayShape &sh, const JobList<RayJob> &L, hipStream_t st)
{
    if (L.total <= 0) return SKEI_OK;
    if (sh.waves == 3) return ray_launch_w<KIND, OUT, 3>(sh.rpt, sh.unroll, sh.shm, L, st);
    if (sh.waves == 4) return ray_launch_w<KIND, OUT, 4>(sh.rpt, sh.unroll, sh.shm, L, st);
    if (sh.waves == 6) return ray_launch_wide<KIND, OUT, 6>(sh.rpt, sh.unroll, sh.shm, L, st);
    if (sh.waves == 8) return ray_launch_wide<KIND, OUT, 8>(sh.rpt, sh.unroll, sh.shm, L, st);
    return SKEI_ERANGE;
}

}  // namespace

int ray_run(int kind, bool out_double, const RayShape &sh, const JobList<RayJob> &L, hipStream_t st)
{
    if (sh.shm > kLdsMax) return SKEI_ERANGE;
    if (kind == kRayFwd) return out_double ? SKEI_EINVAL : ray_launch<kFwd, float>(sh, L, st);
    return out_double ? ray_launch<kBpT, double>(sh, L, st) : ray_launch<kBpT, float>(sh, L, st);
}

int launch_radon_fwd(const skei_geom *g, const float *x, const float *xT, int batch, const int32_t *idx, int m,
                     float *y, const float *yfull, const RayTune &tune, hipStream_t st)
{
    RayJob J;
    RayShape sh;
    int rc = make_ray_job(g, x, xT, batch, idx, m, y, yfull, tune, 0, J, sh);
    if (rc) return rc;
    return ray_run(kRayFwd, false, sh, inline_jobs(&J, 1), st);
}

int launch_bp_T(const skei_geom *g, const float *x, const float *xT, int batch, const int32_t *idx, int m, float *qf,
                double *qd, const RayTune &tune, hipStream_t st)
{
    RayJob J;
    RayShape sh;
    int rc = make_ray_job(g, x, xT, batch, idx, m, qd ? (void *)qd : (void *)qf, nullptr, tune, 0, J, sh);
    if (rc) return rc;
    return ray_run(kRayBpT, qd != nullptr, sh, inline_jobs(&J, 1), st);
}

}  // namespace skei

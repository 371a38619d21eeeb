// Pixel-driven gathers over the listed angles: the Joseph adjoint A_S^T and
// the FBP backprojection B_S.  Neither scatters, so there are no atomics.
//
// A workgroup owns a 16 x 16 pixel tile of one image.  For every listed angle
// the tile projects onto fewer than 16*sqrt(2) + 2 detectors, so the angle's
// sinogram row is staged into LDS only over a 32-bin window; the per-angle
// constants (fixed-point row and column offsets of the tile's pixels within
// the window, Joseph weights) are staged beside it.  Each pixel then reads
// one 8-byte LDS entry per angle: (value, next value) for the Joseph adjoint,
// or (value, next - value) for the linear-interpolation backprojection.
// Positions are 32.32 fixed-point integers formed by integer adds, so the
// interpolation weights carry only the 2^-32 rounding of the per-angle
// constants and their final float rounding.
#include <algorithm>
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

// Per listed angle of a chunk: the column step of four pixels in 32.32 fixed
// point and the Joseph width.
struct GatherAngle {
    long long c4;      // 4 cos theta in 32.32
    float w, wm1;      // Joseph width max(|cos|,|sin|) and w - 1
};

// A workgroup holds a 16 x 16 tile x GA angle groups; each thread owns PPT
// pixels of one tile row (columns dx, dx + 16/PPT, ...), so the per-angle
// loads and the row's share of the position are shared by PPT pixels.  The
// listed angles are split into four fixed classes (r % 4); each class is
// summed in increasing r, and the four class sums are added in a fixed
// order.  Thread (pixel group, ga) owns the classes ga, ga + GA, ...
//
// Positions are exact integers in 32.32 fixed point.  Per angle the window
// coordinate of the tile origin T and the steps S = sin, C = cos are rounded
// once to 2^-32; a pixel (dy, dx) sits at T + dy S + dx C, formed by integer
// adds from a per-row table T + dy S, a per-column table (dx mod 4) C and
// steps of 4C.  Integer sums do not depend on their order, so every pixel's
// position, and with it every result, is bitwise the same whatever GA, PPT,
// the batch size or the other jobs of the launch.  The position's high word
// is the window bin, its low word the interpolation fraction (rounded once to
// float); the quantisation is below 2^-28 px.
constexpr int kClasses = 4;
constexpr int kGChunk = 32;   // listed angles staged per pass
constexpr float kFrac = 0x1p-32f;   // weight of the low word
typedef __attribute__((address_space(1))) const float gfloat;   // global memory

// One listed angle's contribution to a thread's PPT pixels.
template <int KIND, int PPT, int CW>
__device__ __forceinline__ void gather_angle(const GatherAngle &p, long long pos, const float2 *__restrict__ wa_row,
                                             float (&acc)[PPT])
{
    const long long step = (long long)(CW / 4) * p.c4;
#pragma unroll
    for (int v = 0; v < PPT; v++) {
        const int k = (int)(pos >> 32);                      // 0 <= k < WIN - 1 by construction
        const float fs = (float)(unsigned)(pos & 0xffffffffLL);   // fraction x 2^32
        const float2 e = wa_row[k];
        if (KIND == kJosephAdj) {
            // weights Lambda((k - t)/w)/w for k, k+1 (the 1/w^2 is in the
            // window); both are <= 1, so the clamps fold into the adds
            const float wa = __builtin_amdgcn_fmed3f(fmaf(fs, -kFrac, p.w), 0.0f, 1.0f);
            const float wb = __builtin_amdgcn_fmed3f(fmaf(fs, kFrac, p.wm1), 0.0f, 1.0f);
            acc[v] = fmaf(wa, e.x, acc[v]);
            acc[v] = fmaf(wb, e.y, acc[v]);
        } else {
            // the window holds (value, (next - value) 2^-32)
            acc[v] += e.x;
            acc[v] = fmaf(fs, e.y, acc[v]);
        }
        pos += step;
    }
}

template <int KIND, int GA, int PPT>
__device__ __forceinline__ void gather_item(const GatherJob &J, long long item)
{
    constexpr int TILE = 16, NPIX = TILE * TILE, TPG = NPIX / PPT, BS = TPG * GA, WIN = 2 * TILE;
    constexpr int CW = TILE / PPT;   // column step between a thread's pixels
    constexpr int NC = kClasses / GA;
    static_assert(CW % 4 == 0 || PPT == 1, "pixel columns step by multiples of four");
    __shared__ GatherAngle prm[kGChunk];
    __shared__ int kst[kGChunk];                  // first detector of each window
    __shared__ float iw2[kGChunk];                // 1/w^2 (Joseph weights)
    __shared__ long long rcol[kGChunk][4];        // (dx mod 4) C
    __shared__ float2 win[kGChunk * WIN];
    // the row table during the angle loop; the epilogue's buffers afterwards
    constexpr int kRowBytes = kGChunk * TILE * 8;
    constexpr int kEpiBytes = kClasses * NPIX * 4 + TILE * (TILE + 1) * 4 + NPIX * 8;
    __shared__ __align__(16) unsigned char shared_rows[kRowBytes > kEpiBytes ? kRowBytes : kEpiBytes];
    long long(*rrow)[TILE] = reinterpret_cast<long long(*)[TILE]>(shared_rows);   // T + dy S
    float(*part)[NPIX] = reinterpret_cast<float(*)[NPIX]>(shared_rows);
    float(*tileT)[TILE + 1] = reinterpret_cast<float(*)[TILE + 1]>(shared_rows + kClasses * NPIX * 4);
    double *pss = reinterpret_cast<double *>(shared_rows + kClasses * NPIX * 4 + TILE * (TILE + 1) * 4);
    static_assert(kGChunk % kClasses == 0, "angle chunks must keep the classes aligned");

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
    const int dy = pg / CW, dx0 = pg % CW;
    const int col4 = dx0 & 3, q0 = dx0 >> 2;   // first column = col4 + 4 q0
    const double cN = 0.5 * (n - 1), cD = 0.5 * (n_det - 1);
    const float *src = J.in + (size_t)b * m * n_det;
    const gfloat *srcg = (const gfloat *)src;

    float acc[NC][PPT];
#pragma unroll
    for (int c = 0; c < NC; c++)
#pragma unroll
        for (int v = 0; v < PPT; v++) acc[c][v] = 0.0f;
    for (int A0 = 0; A0 < m; A0 += kGChunk) {
        const int Ac = min(kGChunk, m - A0);
        __syncthreads();
        for (int a = tid; a < Ac; a += BS) {
            const AngleRow t = tab[((const __attribute__((address_space(1))) int32_t *)idx)[A0 + a]];
            const double c = t.cd, s = t.sd;
            const double X0 = j0 - cN, Y0 = i0 - cN;
            const double org = X0 * c + Y0 * s + cD;
            const double tmin = org + fmin(0.0, (TILE - 1) * c) + fmin(0.0, (TILE - 1) * s);
            const double k0 = floor(tmin) - 1.0;
            // 32.32 fixed point, each rounded once: the window coordinate of
            // the tile origin (in [1, 32)) here, cos and sin in the table
            const double tw = org - k0;
            const int th = (int)tw;
            const long long T = ((long long)th << 32) + (long long)rint(ldexp(tw - th, 32));
            const long long S = t.s_fx, C = t.c_fx;
            prm[a] = GatherAngle{4 * C, t.w, t.w - 1.0f};
            kst[a] = (int)k0;
            iw2[a] = t.inv_w2;
#pragma unroll
            for (int j = 0; j < 4; j++) rcol[a][j] = j * C;
            long long r = T;
#pragma unroll
            for (int y = 0; y < TILE; y++, r += S) rrow[a][y] = r;
        }
        __syncthreads();
        // the windows: every load of a batch is issued before any is used
        // (branch-free, indexes clamped into the row, out-of-row bins zeroed)
        constexpr int EPT = (kGChunk * WIN + BS - 1) / BS, EB = EPT < 4 ? EPT : 4;
        for (int u0 = 0; u0 < EPT; u0 += EB) {
            float v0[EB], v1[EB];
#pragma unroll
            for (int u = 0; u < EB; u++) {
                const int e = tid + (u0 + u) * BS, a = e < Ac * WIN ? e / WIN : 0;
                const int k = kst[a] + e % WIN, r = (A0 + a) * n_det;   // r < 2^31: one image's sinogram
                v0[u] = srcg[(unsigned)(r + min(max(k, 0), n_det - 1))];
                v1[u] = srcg[(unsigned)(r + min(max(k + 1, 0), n_det - 1))];
            }
#pragma unroll
            for (int u = 0; u < EB; u++) {
                const int e = tid + (u0 + u) * BS;
                if (e < Ac * WIN) {
                    const int a = e / WIN, k = kst[a] + e % WIN;
                    const float x0 = (k >= 0 && k < n_det) ? v0[u] : 0.0f;
                    const float x1 = (k + 1 >= 0 && k + 1 < n_det) ? v1[u] : 0.0f;
                    if (KIND == kJosephAdj)
                        win[e] = make_float2(x0 * iw2[a], x1 * iw2[a]);
                    else
                        win[e] = make_float2(x0, (x1 - x0) * kFrac);
                }
            }
        }
        __syncthreads();
        // whole groups of four angles, then the chunk's tail
        int a4 = 0;
#pragma unroll 1
        for (; a4 + kClasses <= Ac; a4 += kClasses) {
#pragma unroll
            for (int c = 0; c < NC; c++) {
                const int a = a4 + ga + c * GA;
                const long long pos = rrow[a][dy] + rcol[a][col4] + (CW > 4 ? q0 * prm[a].c4 : 0LL);
                gather_angle<KIND, PPT, CW>(prm[a], pos, win + a * WIN, acc[c]);
            }
        }
        if (a4 < Ac) {
#pragma unroll
            for (int c = 0; c < NC; c++) {
                const int a = a4 + ga + c * GA;
                if (a < Ac) {
                    const long long pos = rrow[a][dy] + rcol[a][col4] + (CW > 4 ? q0 * prm[a].c4 : 0LL);
                    gather_angle<KIND, PPT, CW>(prm[a], pos, win + a * WIN, acc[c]);
                }
            }
        }
    }
    __syncthreads();   // the row table's space is reused below
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
    float oth[PPT];   // the residual's other operand, loaded before any store
#pragma unroll
    for (int v = 0; v < PPT; v++) {
        const int px = pix(v), i = i0 + px / TILE, j = j0 + px % TILE;
        oth[v] = (resid && ga == 0 && i < n && j < n) ? J.other[((size_t)b * n + i) * n + j] : 0.0f;
    }
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
                out = oth[v] - out;
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

// Four-wave workgroups are held to 64 VGPRs (eight waves per SIMD): the few
// registers that spill are the staging pass's, and the occupancy gained hides
// the staging latency (measured on MI355X: Joseph adjoint and backprojection
// of 16 images of 256^2 over 90 angles in 62 and 41 us, against 69 and 48 us
// at the unconstrained 98 VGPRs).  One- and two-group workgroups of one
// pixel per thread are held to seven waves (72 VGPRs, 24 bytes spilled for one
// group): there few listed angles leave each item short and latency-bound
// (measured on MI355X: a 512^2 image with 16 copies over 5 listed angles, the
// backprojection and the Joseph adjoint 45.4 -> 42.8 and 48.6 -> 41.3 us)
template <int KIND, int GA, int PPT>
__global__ void __launch_bounds__(256 * GA / PPT) __attribute__((amdgpu_waves_per_eu(GA == 4 ? 8 : PPT == 1 ? 7 : 1))) k_gather(const JobList<GatherJob> L)
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

// Host walk of the window bins a tile's pixels read, from the kernel's own
// fixed-point formulas: for image size n, every 16 x 16 tile, the angles of
// 7- and 360-angle tables, and 2 or ceil(sqrt 2 n) + 1 detectors.  Positions
// are integer-linear in (dx, dy), so a tile's extreme bins are at its
// corners.  out[0..2] = lowest bin read, highest bin read (the interpolation
// neighbour k + 1 included), and the window length.
void gather_lds_reads(int n, long long out[3])
{
    constexpr int TILE = 16, WIN = 2 * TILE;
    const double pi = 3.14159265358979323846, two32 = 4294967296.0;
    const double cN = 0.5 * (n - 1);
    long long lo = 1LL << 60, hi = -1;
    for (int na : {7, 360}) {
        for (int a = 0; a < na; a++) {
            const double th = pi * (double)a / (double)na, c = std::cos(th), s = std::sin(th);
            const long long C = std::llround(c * two32), S = std::llround(s * two32);
            for (int nd : {2, (int)std::ceil(std::sqrt(2.0) * n) + 1}) {
                const double cD = 0.5 * (nd - 1);
                for (int i0 = 0; i0 < n; i0 += TILE) {
                    for (int j0 = 0; j0 < n; j0 += TILE) {
                        const double X0 = j0 - cN, Y0 = i0 - cN;
                        const double org = X0 * c + Y0 * s + cD;
                        const double tmin = org + std::fmin(0.0, (TILE - 1) * c) + std::fmin(0.0, (TILE - 1) * s);
                        const double k0 = std::floor(tmin) - 1.0;
                        const double tw = org - k0;
                        const int tf = (int)tw;
                        const long long T = ((long long)tf << 32) + (long long)std::rint(std::ldexp(tw - tf, 32));
                        for (int dy : {0, TILE - 1}) {
                            for (int dx : {0, TILE - 1}) {
                                const long long k = (T + dy * S + dx * C) >> 32;
                                lo = std::min(lo, k);
                                hi = std::max(hi, k + 1);
                            }
                        }
                    }
                }
            }
        }
    }
    out[0] = lo;
    out[1] = hi;
    out[2] = WIN;
}

// Default gather shape for up to m listed angles: one angle group of one pixel
// per thread while few angles leave each item latency-bound, two groups of
// four pixels per thread in between, four groups once there are enough angles
// to share (measured on MI355X, a 512^2 image with 16 copies: backprojection /
// Joseph adjoint at 10 angles 48.3 / 48.2 us with one group against 54.6 /
// 51.4 with four; at 20 angles 59.0 / 58.7 with two against 60.9 / 59.5; at
// 50 angles 91.0 / 96.8 with four against 95.3 / 102.7 with two).
int gather_groups_auto(int m) { return m < 12 ? 1 : m < 32 ? 24 : 44; }

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

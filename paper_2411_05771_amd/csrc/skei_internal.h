// Internal declarations shared by the HIP translation units of libskei_ct.
// Not part of the public C ABI (include/skei_ct.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "skei_ct.h"

namespace skei {

// Per full-scan angle constants, computed in double precision on the host and
// rounded once to float.  "Major" is the axis Joseph's method steps along
// (image rows when |cos| >= |sin|, columns otherwise); "minor" is the axis it
// interpolates along.  With c_m / c_M the direction cosines of the minor and
// major axes, the minor coordinate of ray k at major index M is
//     u(k, M) = base + k * inv_m + M * du ,
// i.e. u = (s_k - (M - cN) c_M) / c_m + cN.
struct AngleRow {
    int64_t base_fx;  // base, inv_m and du in 32.32 fixed point (exact ray stepping)
    int64_t inv_fx;
    int64_t du_fx;
    int64_t c_fx, s_fx;   // cos theta, sin theta in 32.32 (pixel-driven positions)
    double scale;     // 1 / |c_m|   (Joseph step length), double
    double cd, sd;    // cos theta, sin theta in double (pixel-driven positions)
    float c, s;       // cos theta, sin theta
    float w;          // |c_m| = max(|cos|, |sin|)
    float inv_w2;     // 1 / w^2
    float du;         // -c_M / c_m               (float copies for range estimates)
    float base;       // -cD / c_m + cN (1 + c_M / c_m)
    float inv_m;      // 1 / c_m
    int rows;         // 1: major axis = image rows
};
static_assert(sizeof(AngleRow) == 96, "AngleRow layout");

// LDS line padding used by the ray-driven kernels: every staged image line
// carries PAD zeros on each side so that clamped tap positions read zeros.
constexpr int kLinePad = 4;

// Angles staged per LDS pass by the pixel-driven gathers.
constexpr int kAngleChunk = 64;

// Accelerator complex dies (XCDs) of the device; each has its own L2.
// Workgroup L of a launch is dispatched to XCD L % kXcds.
constexpr int kXcds = 8;

int check_launch();   // maps hipGetLastError to SKEI_OK / SKEI_ELAUNCH

// ------------------------------------------------------------------ jobs
// Every kernel runs a list of jobs; a job is one operator application on one
// problem (its own geometry, images, sketch and buffers), cut into `items`
// work items of one workgroup each.  The arithmetic of an item depends only
// on its job, never on the other jobs of the launch or on how items are
// dispatched, so a problem's results are bitwise the same alone and batched.

// Joseph forward projection (KIND fwd) or B_S^T (KIND bpT) over listed angles.
//   fwd, resid = 0: y[b][r][k] = (A_S x[b])[r][k]
//   fwd, resid = 1: y[b][r][k] = yfull[b][idx[r]][k] - (A_S x[b])[r][k]   (in double);
//   bpT:            y[b][r][k] = (B_S^T x[b])[r][k]  (unscaled)
// xT (optional): the images transposed (xT[b][j][i] = x[b][i][j]); when given,
// column-stepping angles stage rows of xT instead of gathering columns of x.
// An item is G consecutive listed angles x one of nseg detector segments of
// one image.
struct RayJob {
    const float *x, *xT;
    const int32_t *idx;
    const AngleRow *tab;
    void *y;                 // float or double, by launch
    const float *yfull;
    int n, n_det, m, n_angles;
    int G, nseg, seg, ngroups;
    int R, pitch, resid, pad_;
    long long items;
};

// Pixel-driven gathers over listed angles (KIND joseph-adjoint or
// backprojection): out = scale * op(in), or out = other - scale * op(in) when
// `other` is given (then partial[item] = sum out^2 if partial is given);
// outT (optional) receives out transposed.  An item is a 16 x 16 pixel tile.
struct GatherJob {
    const float *in;
    const int32_t *idx;
    const AngleRow *tab;
    float *out;
    const float *other;
    double *partial;
    float *outT;
    int n, n_det, m;
    float scale;
    long long items;
};

// Ram-Lak filter along detector rows: q = scale * H p.  An item is one row.
// With `partial` set the job instead sums the squares of each row of p:
// partial[row] = sum_k p[row][k]^2, in double, in a fixed order.  With `loss`
// set it is one item that forms the EI loss from the partial sums (see
// fixed_order_loss): loss = w0 * sum(s0[0..n0)) + w1 * sum(s1[0..n1)).
struct RampJob {
    const void *p;           // float or double, by launch
    float *q;
    double *partial;
    const double *hodd;
    int n_det;
    float scale;
    long long rows;          // rows of a sum-of-squares job
    long long items;
    const double *s0, *s1;   // loss job
    long long n0, n1;
    double w0, w1;
    double *loss;
};

// out[b][c] = T_c x[b] (and outT = its transpose), or, with cs == nullptr, the
// plain copy / transpose of x (copies = 1).  An item is a 16 x 16 output tile.
struct RotJob {
    const float *x;
    const float *cs;
    float *out, *outT;
    int n, copies;
    long long items;
};

// g[b] = alpha * sum_c T_c^T h[b][c] + beta * add[b]; then, when x_upd is
// given, x_upd[b] -= step * g[b].  An item is 64 pixels.
struct RotAdjJob {
    const float *h;
    const float *cs;
    const float *add;
    float *g;
    float *x_upd;
    int n, copies;
    float alpha, beta, step;
    int pad_;
    long long items;
};

// out = w0 * sum(p0[0..n0)) + w1 * sum(p1[0..n1)), fixed order.  One item.
struct RedJob {
    const double *p0, *p1;
    double *out;
    long long n0, n1;
    double w0, w1;
    long long items;
};

// Persistent-launch cursors (device memory), one per XCD range.  A stage
// alternates between two sets: each launch draws from one and zeroes the
// other, which the next launch of the stage (stream-ordered after it) uses.
struct WorkQueue {
    unsigned int next[kXcds];
    unsigned int pad_[8];
};

constexpr int kInlineJobs = 2;

// A launch's job list.
//   inline mode (jobs == nullptr): up to kInlineJobs jobs passed by value;
//     their concatenated items are cut into 8 contiguous ranges of about
//     equal cost, and workgroup L takes item L / 8 of range L % 8.
//   table modes: jobs / first (first global item of each job, njobs + 1
//     entries) / xr (kXcds + 1 boundaries of the XCD ranges) in device memory.
//     wq == nullptr: one workgroup per item, XCD x runs its range in order.
//     wq != nullptr: persistent workgroups run a static share of their XCD's
//     range, then draw its remainder and the other XCDs' remainders one item
//     at a time from per-XCD cursors.
template <typename Job>
struct JobList {
    Job inl[kInlineJobs];
    long long inl_first[kInlineJobs + 1];
    long long inl_xr[kXcds + 1];   // inline mode: XCD ranges of the items
    int ninl;
    int njobs;
    const Job *jobs;
    const long long *first;
    const long long *xr;
    WorkQueue *wq;
    WorkQueue *wq_next;      // zeroed by this launch for the next one
    long long total;
    long long grid_static;   // table mode without queue: 8 * largest XCD range
    int persistent_grid;     // table mode with queue: workgroups to launch (0 = auto)
};

// Estimated cost of one item of a job (arbitrary units, only ratios matter);
// used to cut work lists into XCD ranges of about equal cost.
inline double item_cost(const RayJob &j) { return (double)j.G * j.seg * j.n + 4.0 * j.n * j.n / (j.R > 0 ? j.R : 1); }
inline double item_cost(const GatherJob &j) { return 256.0 * (j.m + 8); }
inline double item_cost(const RampJob &j)
{
    return j.loss ? (double)(j.n0 + j.n1) : j.partial ? 4.0 * j.n_det : (double)j.n_det * (j.n_det / 2 + 4);
}
inline double item_cost(const RotJob &j) { return j.cs ? 256.0 * 4 : 256.0; }
inline double item_cost(const RotAdjJob &j) { return 64.0 * 9 * j.copies; }
inline double item_cost(const RedJob &j) { return (double)(j.n0 + j.n1); }

// Cuts the concatenated items of `count` jobs (first[i] = first item of job
// i, first[count] = total) where the running cost first reaches x/8 of the
// total: xr[0..8] with xr[0] = 0 and xr[8] = total.  Returns the largest
// range.
template <typename Job>
inline long long xcd_ranges(const Job *jobs, int count, const long long *first, long long *xr)
{
    const long long total = first[count];
    double total_cost = 0.0;
    for (int i = 0; i < count; i++) total_cost += item_cost(jobs[i]) * (double)jobs[i].items;
    for (int x = 0; x <= kXcds; x++) xr[x] = total;
    xr[0] = 0;
    double run = 0.0;
    int x = 1;
    for (int i = 0; i < count && x < kXcds; i++) {
        const double c = item_cost(jobs[i]);
        const long long cnt = jobs[i].items;
        while (x < kXcds) {
            const double target = total_cost * x / kXcds;
            if (run + c * (double)cnt < target) break;
            long long k = c > 0 ? (long long)((target - run) / c + 0.999999) : 0;
            k = k < 0 ? 0 : (k > cnt ? cnt : k);
            xr[x++] = first[i] + k;
        }
        run += c * (double)cnt;
    }
    long long widest = 0;
    for (int q = 1; q <= kXcds; q++) {
        if (xr[q] < xr[q - 1]) xr[q] = xr[q - 1];
        if (xr[q] - xr[q - 1] > widest) widest = xr[q] - xr[q - 1];
    }
    return widest;
}

template <typename Job>
inline JobList<Job> inline_jobs(const Job *jobs, int count)
{
    JobList<Job> L{};
    L.ninl = count;
    long long t = 0;
    for (int i = 0; i < count; i++) {
        L.inl[i] = jobs[i];
        L.inl_first[i] = t;
        t += jobs[i].items;
    }
    L.inl_first[count] = t;
    L.total = t;
    L.grid_static = kXcds * xcd_ranges(jobs, count, L.inl_first, L.inl_xr);
    return L;
}

// ------------------------------------------------------------- launchers
// All enqueue on `st` and return SKEI_OK, SKEI_ERANGE (a launch shape the
// kernels do not support) or SKEI_ELAUNCH.

enum RayKind : int { kRayFwd = 0, kRayBpT = 1 };
enum GatherKind : int { kGatherJosephAdj = 0, kGatherBackproject = 1 };

// Launch shape of a ray kernel: rays per thread (1..4), lines per unrolled
// march unit (16, 8 or 4) and LDS bytes.
struct RayShape {
    int rpt;
    int unroll;
    int waves;   // per workgroup: 3, 4, 6 or 8 (6 and 8 with at most 2 rays per thread)
    size_t shm;
};

// The shape one launch needs for jobs of shapes a and b.
inline RayShape merge_shapes(const RayShape &a, const RayShape &b)
{
    RayShape r;
    r.rpt = a.rpt > b.rpt ? a.rpt : b.rpt;
    r.unroll = a.unroll < b.unroll ? a.unroll : b.unroll;   // units nest: 4 | 8 | 16
    // jobs of a launch share the wave count (0 = unset; a mismatch fails the launch)
    r.waves = a.waves == 0 ? b.waves : b.waves == 0 ? a.waves : a.waves == b.waves ? a.waves : -1;
    r.shm = a.shm > b.shm ? a.shm : b.shm;
    return r;
}

// Ray kernels: sh.rpt >= ceil(G * seg / 256), sh.shm >= 2 * R * pitch * 4 and
// R a multiple of sh.unroll for every job; out_double selects y's element type.
int ray_run(int kind, bool out_double, const RayShape &sh, const JobList<RayJob> &L, hipStream_t st);
// Gathers with GA angle groups per pixel (1, 2 or 4; results do not depend on it).
int gather_run(int kind, int ga, const JobList<GatherJob> &L, hipStream_t st);
// Ramp: block >= ramp_block(n_det) and shm >= ramp_shm(n_det) for every job.
int ramp_run(bool in_double, int block, size_t shm, const JobList<RampJob> &L, hipStream_t st);
int rotate_run(const JobList<RotJob> &L, hipStream_t st);
int rotate_adj_run(const JobList<RotAdjJob> &L, hipStream_t st);
int reduce_run(const JobList<RedJob> &L, hipStream_t st);

// Launch shape of the ray-driven kernels (0 = automatic choice):
//   group: listed angles per workgroup (they share every staged image chunk)
//   lines: image lines per march unit (an LDS chunk holds two)
//   split: detector segments per angle
struct RayTune {
    int group = 0, lines = 0, split = 0;
    int waves = 0;   // waves per workgroup (3, 4, 6 or 8; 0 = 3 or 4, whichever leaves fewer ray slots empty)
    int units = 2;   // march units per LDS chunk (2 or 4)
};

// Ray job of one operator application and the launch shape it needs.
// rpt_cap > 0 sizes G and the segments to fill at most rpt_cap * 256 rays per
// workgroup (tune.group / tune.split still win).
int make_ray_job(const struct ::skei_geom *g, const float *x, const float *xT, int batch, const int32_t *idx,
                 int m, void *y, const float *yfull, const RayTune &tune, int rpt_cap,
                 RayJob &job, RayShape &shape);

GatherJob make_gather_job(const struct ::skei_geom *g, const float *in, int batch, const int32_t *idx, int m,
                          float scale, float *out, const float *other, double *partial, float *outT);
size_t gather_items(int n, int batch);
int gather_groups_auto(int m);   // default GA for m listed angles

RampJob make_ramp_job(const struct ::skei_geom *g, const void *p, long long rows, float scale, float *q);
// Row sums of squares of p [rows][N_det] (float) into partial[rows]; runs in a ramp launch.
RampJob make_row_sumsq_job(const struct ::skei_geom *g, const float *p, long long rows, double *partial);
// The EI loss from its partial sums, as one item of a ramp launch.
RampJob make_loss_job(const RedJob &r);
int ramp_block(int n_det);      // threads per row
size_t ramp_shm(int n_det);     // LDS bytes per row
// Dense sketch of sinogram rows (k_sketch.hip): out = G y per image, or
// G^T y with transpose; G is m x n_rows row-major.
int launch_sketch_rows(const float *G, int m, int n_rows, const float *y, int batch, int row_len, bool transpose,
                       float *out, hipStream_t st);
// Host walks of the LDS reads of the ramp and ray kernels (bounds self-checks).
void ramp_lds_reads(int n_det, long long out[5]);
void ray_lds_reads(int n, long long out[3]);
void gather_lds_reads(int n, long long out[3]);

RotJob make_rot_job(const float *x, int batch, int copies, int n, const float *cs, float *out, float *outT);
RotAdjJob make_rot_adj_job(const float *h, int batch, int copies, int n, const float *cs, float alpha,
                           const float *add, float beta, float *g);

// Convenience wrappers: one job, inline mode.
int launch_radon_fwd(const skei_geom *g, const float *x, const float *xT, int batch, const int32_t *idx, int m,
                     float *y, const float *yfull, const RayTune &tune, hipStream_t st);
int launch_bp_T(const skei_geom *g, const float *x, const float *xT, int batch, const int32_t *idx, int m,
                float *qf, double *qd, const RayTune &tune, hipStream_t st);
int launch_gather(int kind, const skei_geom *g, const float *in, int batch, const int32_t *idx, int m, float scale,
                  float *out, const float *other, double *partial, float *outT, hipStream_t st);
int launch_ramp(const skei_geom *g, const float *pf, const double *pd, long long rows, float scale, float *q,
                hipStream_t st);
int launch_rotate(const float *x, int batch, int copies, int n, const float *cs, float *out, float *outT,
                  hipStream_t st);
int launch_rotate_adj(const float *h, int batch, int copies, int n, const float *cs, float alpha,
                      const float *add, float beta, float *g, hipStream_t st);

// Deterministic reductions.
size_t sumsq_partials(size_t len);
int launch_sumsq(const float *a, const float *b, size_t len, double *partial, hipStream_t st);
int launch_reduce2(const double *p0, size_t n0, double w0, const double *p1, size_t n1, double w1,
                   double *out, hipStream_t st);

}  // namespace skei

struct skei_geom {
    int n, n_angles, n_det;
    int device;
    skei::RayTune tune_fwd, tune_bpt;
    skei::AngleRow *tab;   // device [n_angles]
    double *hodd;          // device [n_hodd]: h(2e+1) = -1 / (pi (2e+1))^2
    int n_hodd;
};

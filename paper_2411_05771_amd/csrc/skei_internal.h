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
    double scale;     // 1 / |c_m|   (Joseph step length), double
    float c, s;       // cos theta, sin theta
    float w;          // |c_m| = max(|cos|, |sin|)
    float inv_w2;     // 1 / w^2
    float du;         // -c_M / c_m               (float copies for range estimates)
    float base;       // -cD / c_m + cN (1 + c_M / c_m)
    float inv_m;      // 1 / c_m
    int rows;         // 1: major axis = image rows
};
static_assert(sizeof(AngleRow) == 64, "AngleRow layout");

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
//                   partial[item] = sum of y^2 over the item's rays
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
    double *partial;
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
struct RampJob {
    const void *p;           // float or double, by launch
    float *q;
    const double *hodd;
    int n_det;
    float scale;
    long long items;
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

// Persistent-launch cursors (device memory).  They are zero between launches:
// the last workgroup to finish a launch resets them.
struct WorkQueue {
    unsigned int next[kXcds];
    unsigned int done;
    unsigned int pad_[7];
};

constexpr int kInlineJobs = 2;

// A launch's job list.
//   inline mode (jobs == nullptr): up to kInlineJobs jobs passed by value;
//     workgroup L takes item (L % 8) * per + L / 8 of the concatenated items
//     (XCD-major: each XCD gets one contiguous range).
//   table modes: jobs / first (first global item of each job, njobs + 1
//     entries) / xr (kXcds + 1 boundaries of the XCD ranges) in device memory.
//     wq == nullptr: one workgroup per item, XCD x runs its range in order.
//     wq != nullptr: persistent workgroups draw `chunk` items at a time from
//     their XCD's queue and then from the other XCDs' queues.
template <typename Job>
struct JobList {
    Job inl[kInlineJobs];
    long long inl_first[kInlineJobs + 1];
    int ninl;
    int njobs;
    const Job *jobs;
    const long long *first;
    const long long *xr;
    WorkQueue *wq;
    long long total;
    long long grid_static;   // table mode without queue: 8 * largest XCD range
    int persistent_grid;     // table mode with queue: workgroups to launch (0 = auto)
    int chunk;               // table mode with queue: items per draw (0 = 1)
};

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
    return L;
}

// ------------------------------------------------------------- launchers
// All enqueue on `st` and return SKEI_OK, SKEI_ERANGE (a launch shape the
// kernels do not support) or SKEI_ELAUNCH.

enum RayKind : int { kRayFwd = 0, kRayBpT = 1 };
enum GatherKind : int { kGatherJosephAdj = 0, kGatherBackproject = 1 };

// Ray kernels: rpt = rays per thread (1..8) >= ceil(G * seg / 256) for every
// job; shm = LDS bytes >= 2 * R * pitch * 4 for every job; out_double selects
// the element type of y.
int ray_run(int kind, bool out_double, int rpt, size_t shm, const JobList<RayJob> &L, hipStream_t st);
// Gathers with GA angle groups per pixel (1, 2 or 4; results do not depend on it).
int gather_run(int kind, int ga, const JobList<GatherJob> &L, hipStream_t st);
// Ramp: rpt >= ceil(n_det / block) for every job, block a multiple of 64,
// shm >= (3 n_det + 2) * sizeof(element) for every job.
int ramp_run(bool in_double, int rpt, int block, size_t shm, const JobList<RampJob> &L, hipStream_t st);
int rotate_run(const JobList<RotJob> &L, hipStream_t st);
int rotate_adj_run(const JobList<RotAdjJob> &L, hipStream_t st);
int reduce_run(const JobList<RedJob> &L, hipStream_t st);

// Launch shape of the ray-driven kernels (0 = automatic choice):
//   group: listed angles per workgroup (they share every staged image chunk)
//   lines: image lines per LDS chunk
//   split: detector segments per angle
struct RayTune {
    int group = 0, lines = 0, split = 0;
};

// Ray job of one operator application; returns the rays per thread it needs
// (rpt) and its LDS bytes.  rpt_cap > 0 sizes G and the segments to fill at
// most rpt_cap * 256 rays per workgroup (tune.group / tune.split still win).
struct RayShape {
    int rpt;
    size_t shm;
};
int make_ray_job(const struct ::skei_geom *g, const float *x, const float *xT, int batch, const int32_t *idx,
                 int m, void *y, const float *yfull, double *partial, const RayTune &tune, int rpt_cap,
                 RayJob &job, RayShape &shape);
// Upper bound of a ray job's items for any tuning (partial-sum buffers).
size_t ray_items_max(const struct ::skei_geom *g, int batch, int m, const RayTune &tune);

GatherJob make_gather_job(const struct ::skei_geom *g, const float *in, int batch, const int32_t *idx, int m,
                          float scale, float *out, const float *other, double *partial, float *outT);
size_t gather_items(int n, int batch);
int gather_groups_auto(int m);   // default GA for m listed angles

RampJob make_ramp_job(const struct ::skei_geom *g, const void *p, long long rows, float scale, float *q);
void ramp_shape(int n_det, int &rpt, int &block);   // per-row launch shape
size_t ramp_shm(int n_det, bool in_double);

RotJob make_rot_job(const float *x, int batch, int copies, int n, const float *cs, float *out, float *outT);
RotAdjJob make_rot_adj_job(const float *h, int batch, int copies, int n, const float *cs, float alpha,
                           const float *add, float beta, float *g);

// Convenience wrappers: one job, inline mode.
int launch_radon_fwd(const skei_geom *g, const float *x, const float *xT, int batch, const int32_t *idx, int m,
                     float *y, const float *yfull, double *partial, const RayTune &tune, hipStream_t st);
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

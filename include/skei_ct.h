/*
 * skei_ct.h -- C ABI of the MI355X (gfx950) sketched-EI CT operator library.
 *
 * The library evaluates the operators that every sketched equivariant-imaging
 * (EI) loss evaluation applies (Xu, Li, Tang, arXiv 2411.05771):
 *
 *   A      discrete Radon transform of a 2-D parallel-beam CT scan
 *          (Sec. 4.1.1; y ~ A x of Sec. 2.1), computed with Joseph's method;
 *   A_S    the sketched operator S A of Sec. 3.1, where the sketch S selects
 *          whole projection angles (the interleaved angle subsets of
 *          Sec. 4.2.1) and is passed as a list of angle indices;
 *   A^T    the exact transpose of A (and A_S^T = A^T S^T);
 *   fbp    filtered backprojection, the stable approximation of A^dagger
 *          named in Sec. 2.1 and Sec. 4.1.1, and fbp_S = (S A)^dagger ~
 *          (pi/m) B_S H of Sec. 3.1 -- Ram-Lak filter H, pixel-driven
 *          linear-interpolation backprojection B_S;
 *   T_phi  the image rotations that form the transformation group of
 *          Sec. 4.1.3, by bilinear resampling;
 *   the sketched test-time EI loss of Eq. (skeilossttt) / Algorithm 2 with
 *   the reconstruction network taken as the identity, and its gradient with
 *   respect to the image.
 *
 * Geometry (fixed by this library; the paper states none of it).  Image
 * pixel (i, j) has centre X = j - (N-1)/2, Y = i - (N-1)/2 (row i <-> Y);
 * detector k sits at s_k = k - (N_det-1)/2 with unit spacing; full-scan
 * angle a is theta_a = a*pi/N_theta; ray (a, k) is {X cos + Y sin = s_k}.
 *
 * Conventions shared by every call:
 *   - Arrays are caller-owned, contiguous, row-major DEVICE memory on the
 *     device that was current when the geometry was created: float32 data,
 *     int32 angle lists.  Images are [batch][N][N]; sinograms are
 *     [batch][m][N_det] with row r holding angle angle_idx[r].
 *   - Angle lists hold indices into the full scan, each in [0, N_theta);
 *     repeats are allowed and rows follow list order.  Entries are NOT
 *     checked on the device: an out-of-range entry is undefined behaviour
 *     (the Python layer validates lists when it builds them).
 *   - Outputs are overwritten, never accumulated.  Inputs and outputs must
 *     not overlap.
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is
 *     the default stream).  No call synchronises the host.
 *   - A skei_geom is immutable after creation; calls on different streams
 *     may share it.
 *   - Return value: SKEI_OK (0) or a negative SKEI_E* code; on error nothing
 *     has been enqueued.  skei_strerror() gives the text.
 *   - Results are deterministic: no atomics, fixed summation order, so the
 *     same inputs give bitwise the same outputs whatever else is in flight.
 */
#ifndef SKEI_CT_H
#define SKEI_CT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SKEI_OK = 0,
    SKEI_EINVAL = -1,   /* null pointer, non-positive size, bad combination   */
    SKEI_ENOMEM = -2,   /* device allocation failed (geometry / plans only)   */
    SKEI_ELAUNCH = -3,  /* a HIP launch or runtime call failed                */
    SKEI_ERANGE = -4,   /* size beyond what the kernels support               */
    SKEI_ESPACE = -5,   /* caller workspace smaller than the *_bytes() query  */
    SKEI_ESCRATCH = -6  /* need beyond the static scratch of a no-allocation  */
                        /* entry point                                        */
};

typedef struct skei_geom skei_geom;

/* Library version string and error text (static storage). */
const char *skei_version(void);
const char *skei_strerror(int code);

/* ------------------------------------------------------------------ */
/* Geometry (Sec. 4.1.1: N x N image, N_theta uniformly spaced angles */
/* in [0, pi), N_det unit-spaced detector bins).                      */
/* Builds the per-angle table (cos, sin, Joseph stepping constants)   */
/* in double precision on the host, rounds it once to float32 and     */
/* uploads it, together with the Ram-Lak taps, to the current device. */
/* Limits: 2 <= N <= 2032, 1 <= N_theta <= 65536, 2 <= N_det <= 2048.  */
/* The returned object owns that device memory; destroy frees it.     */
/* ------------------------------------------------------------------ */
int skei_geom_create(int n, int n_angles, int n_det, skei_geom **out);
int skei_geom_destroy(skei_geom *g);
int skei_geom_info(const skei_geom *g, int *n, int *n_angles, int *n_det);

/* Launch shape of the ray-driven kernels (forward projector, B_S^T) used by
 * later calls on this geometry: `group` listed angles per workgroup (1..8),
 * `lines` image lines per march unit (an LDS chunk holds two), `split`
 * detector segments per angle;
 * 0 keeps the built-in choice.  Results do not depend on these (bitwise);
 * only speed does.  Not to be changed while calls on the geometry run. */
enum { SKEI_OP_FWD = 0, SKEI_OP_BPT = 1 };
int skei_geom_set_tuning(skei_geom *g, int op, int group, int lines, int split);

/* y = A_S x   (Sec. 3.1 sketched forward operator; Joseph's method).
 * x [batch][N][N] -> y [batch][m][N_det].  Row r is the Joseph line sum
 * of every image along the rays of angle angle_idx[r]: step over the
 * image rows (|cos| >= |sin|) or columns, interpolate linearly between the
 * two nearest pixel centres and scale by the step length 1/max(|cos|,|sin|). */
int skei_radon_fwd(const skei_geom *g, const float *x, int batch,
                   const int32_t *angle_idx, int m, float *y, void *stream);

/* r = S y - A_S x   (the measurement-consistency residual of the EI loss,
 * Eq. (skeilossttt) / Algorithm 2, with S the listed angles).
 * x [batch][N][N], y_full [batch][N_theta][N_det] (the whole measured
 * sinogram) -> r [batch][m][N_det] with r[b][i][k] = y_full[b][angle_idx[i]][k]
 * minus row i of skei_radon_fwd(x).  The projection is accumulated and the
 * difference taken in double precision before r is rounded to float32: the
 * residual is far smaller than y, so rounding A_S x to float first would
 * cost most of its significant digits.  Same launch shapes and errors as
 * skei_radon_fwd; y_full must not overlap r. */
int skei_radon_resid(const skei_geom *g, const float *x, const float *y_full, int batch,
                     const int32_t *angle_idx, int m, float *r, void *stream);

/* Dense measurement-space sketches (the Gaussian / Rademacher sketches of
 * Sec. 2.3 and of the proof of Theorem 1), mixing whole projections:
 * S = G (x) I_{N_det} for a dense G in R^{m x n_rows} (row-major, device
 * float32, e.g. i.i.d. N(0, 1/m) or +-1/sqrt(m) entries so that
 * E[S^T S] = I).  A dense sketch of the operator is then A_S = S A, with
 * A_S x = skei_sketch_rows(G, A x) and A_S^T r = A^T skei_sketch_rows_T(G, r).
 *   skei_sketch_rows:   y [batch][n_rows][row_len] -> out [batch][m][row_len],
 *                       out[b][i][c] = sum_a G[i][a] y[b][a][c];
 *   skei_sketch_rows_T: r [batch][m][row_len] -> out [batch][n_rows][row_len],
 *                       out[b][a][c] = sum_i G[i][a] r[b][i][c].
 * Computed on the matrix cores in float32 with float32 accumulation, in a
 * fixed order (deterministic).  batch <= 65535.  Inputs and outputs must not
 * overlap. */
int skei_sketch_rows(const float *G, int m, int n_rows, const float *y, int batch, int row_len,
                     float *out, void *stream);
int skei_sketch_rows_T(const float *G, int m, int n_rows, const float *r, int batch, int row_len,
                       float *out, void *stream);

/* x = A_S^T y   (exact transpose of skei_radon_fwd, computed per pixel as a
 * gather over the m listed angles: no atomics).
 * y [batch][m][N_det] -> x [batch][N][N]. */
int skei_radon_adj(const skei_geom *g, const float *y, int batch,
                   const int32_t *angle_idx, int m, float *x, void *stream);

/* q = H p   (Ram-Lak filter, unit spacing: h(0)=1/4, h(odd n)=-1/(pi n)^2,
 * h(even n)=0), a linear convolution along each detector row with zero
 * padding, accumulated in double precision.  p, q: [rows][N_det]. */
int skei_ramp(const skei_geom *g, const float *p, int rows, float *q, void *stream);

/* x = B_S q   (pixel-driven backprojection without the pi/m factor: each
 * pixel takes the linear interpolation of row r at its projection
 * X cos + Y sin, zero off the detector, summed over the listed angles).
 * q [batch][m][N_det] -> x [batch][N][N]. */
int skei_backproject(const skei_geom *g, const float *q, int batch,
                     const int32_t *angle_idx, int m, float *x, void *stream);

/* q = B_S^T x   (exact transpose of skei_backproject, ray-driven gather).
 * x [batch][N][N] -> q [batch][m][N_det]. */
int skei_backproject_T(const skei_geom *g, const float *x, int batch,
                       const int32_t *angle_idx, int m, float *q, void *stream);

/* FBP as A^dagger (Sec. 2.1, Sec. 4.1.1) and its sketched form fbp_S of
 * Sec. 3.1:  x = fbp_S y = (pi/m) B_S H y;   y' = fbp_S^T x = (pi/m) H B_S^T x.
 * `work` is caller device scratch of at least skei_fbp_workspace_bytes()
 * bytes (it holds the filtered sinogram); work_bytes is its size. */
size_t skei_fbp_workspace_bytes(const skei_geom *g, int batch, int m);
int skei_fbp(const skei_geom *g, const float *y, int batch, const int32_t *angle_idx, int m,
             float *x, void *work, size_t work_bytes, void *stream);
int skei_fbp_adj(const skei_geom *g, const float *x, int batch, const int32_t *angle_idx, int m,
                 float *y, void *work, size_t work_bytes, void *stream);

/* Rotations T_phi (Sec. 4.1.3 group of rotations), bilinear, zero fill:
 *   out[b][c](p) = x[b](R(-phi_c) p)   about the image centre, i.e. the
 *   output pixel at (X, Y) samples x at (cos X + sin Y, -sin X + cos Y).
 * cos_sin: device float [copies][2] = (cos phi_c, sin phi_c), a point of the
 *   unit circle up to float rounding: the transpose visits the 3 x 3 output
 *   pixels around each input pixel's preimage, which holds every output that
 *   can reach it only while |cos| + |sin| <= sqrt(2).  Other pairs give an
 *   unspecified (but in-bounds) result; they are not checked.
 * skei_rotate:     x [batch][N][N] -> out [batch][copies][N][N].
 * skei_rotate_adj: h [batch][copies][N][N] -> g [batch][N][N],
 *                  g[b] = sum_c T_{phi_c}^T h[b][c]  (exact transpose; gather). */
int skei_rotate(const float *x, int batch, int copies, int n, const float *cos_sin,
                float *out, void *stream);
int skei_rotate_adj(const float *h, int batch, int copies, int n, const float *cos_sin,
                    float *g, void *stream);

/* Sum of squared differences  *out = sum_i (a_i - b_i)^2  (b may be NULL:
 * sum a_i^2), reduced in double precision in a fixed order.  `out` is one
 * device double.  `work` must hold skei_sumsq_workspace_bytes(len). */
size_t skei_sumsq_workspace_bytes(size_t len);
int skei_sumsq_diff(const float *a, const float *b, size_t len, double *out,
                    void *work, size_t work_bytes, void *stream);

/* ------------------------------------------------------------------ */
/* Sketched test-time EI loss and gradient (Eq. skeilossttt, Alg. 2), */
/* network = identity, for an image batch x [batch][N][N]:            */
/*   r_MC[b]  = y[b][mc_idx] - A_mc x[b]                               */
/*   z[b][c]  = T_c x[b],   r[b][c] = z[b][c] - fbp_S(A_S z[b][c])      */
/*   loss     = sum_b ||r_MC[b]||^2 + (lambda/C) sum_{b,c} ||r[b][c]||^2 */
/*   grad[b]  = -2 A_mc^T r_MC[b]                                       */
/*              + (2 lambda / C) sum_c T_c^T (r[b][c] - A_S^T fbp_S^T r) */
/* y is the full measured sinogram [batch][N_theta][N_det]; the MC     */
/* term reads its rows mc_idx[0..m_mc) (all angles for the unsketched  */
/* MC term, the sketch itself for Alg. 2's sketched MC term).          */
/* loss: one device double.  grad: device [batch][N][N] or NULL (loss  */
/* only).  `work`: skei_ei_workspace_bytes() bytes of device scratch.  */
/* ------------------------------------------------------------------ */
size_t skei_ei_workspace_bytes(const skei_geom *g, int batch, int m_mc, int m, int copies);
int skei_ei_loss_grad(const skei_geom *g, const float *x, const float *y, int batch,
                      const int32_t *mc_idx, int m_mc, const int32_t *angle_idx, int m,
                      int copies, const float *cos_sin, float lambda,
                      double *loss, float *grad, void *work, size_t work_bytes, void *stream);

/* No-allocation variant of skei_ei_loss_grad, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, results
 * (bitwise) and kernels as skei_ei_loss_grad, without `work`: the
 * workspace is a static device array of skei_ei_noalloc_scratch_bytes()
 * bytes (64 MiB) inside the library, one per device, held from the first
 * use on that device until the process ends.  The call allocates nothing:
 * no hipMalloc/hipFree, no allocating library routine.  Its first call on
 * a device looks up the array's device address (hipGetSymbolAddress) and
 * caches it.  Limits and errors: SKEI_ESCRATCH (nothing enqueued) when
 * skei_ei_workspace_bytes() of the arguments exceeds the array, e.g. the
 * 256 x 256 / 360-angle / 363-detector step with 16 copies and m = 90
 * needs about 29 MB and fits; a 1024 x 1024 one with 16 copies does not.
 * Every call on a device shares that device's array and leaves its
 * contents behind (the step writes every piece before reading it, so
 * nothing needs clearing): calls that overlap in time on one device, on
 * any streams, race and must be serialised by the caller. */
size_t skei_ei_noalloc_scratch_bytes(void);
int skei_ei_loss_grad_noalloc(const skei_geom *g, const float *x, const float *y, int batch,
                              const int32_t *mc_idx, int m_mc, const int32_t *angle_idx, int m,
                              int copies, const float *cos_sin, float lambda,
                              double *loss, float *grad, void *stream);

/* ------------------------------------------------------------------ */
/* Batched EI plans: many EI problems of different sizes (own geometry, */
/* batch, sketch, copies) evaluated together, one launch per stage for  */
/* all of them.  Each problem computes exactly what skei_ei_loss_grad   */
/* computes for it, bitwise: results do not depend on the other         */
/* problems, the dispatch mode or the launch shapes.                    */
/*                                                                      */
/* A plan binds the problems' device pointers and a caller workspace of */
/* skei_ei_plan_workspace_bytes() bytes (the scratch of every problem   */
/* that brings none of its own) at creation; it owns a small device     */
/* table (work lists and queue cursors) that destroy frees.             */
/* Runs of one plan must not overlap (they share the queue cursors);    */
/* different plans may run concurrently on different streams.  Problems */
/* with grad == NULL get the loss only.                                 */
/* ------------------------------------------------------------------ */
typedef struct skei_ei_problem {
    const skei_geom *geom;
    int batch;
    float *x;                   /* [batch][N][N]; updated when step != 0 */
    const float *y;             /* [batch][N_theta][N_det]               */
    const int32_t *mc_idx;      /* MC angle list, m_mc entries           */
    int m_mc;
    const int32_t *angle_idx;   /* sketch, m entries                     */
    int m;
    int copies;
    const float *cos_sin;       /* [copies][2]                           */
    float lambda;
    double *loss;               /* one device double                     */
    float *grad;                /* [batch][N][N] or NULL                 */
    float step;                 /* gradient step: after the gradient is  */
                                /* formed, x -= step * grad (0: x is     */
                                /* left alone; needs grad)               */
    void *work;                 /* this problem's own scratch of         */
    size_t work_bytes;          /* skei_ei_problem_workspace_bytes()     */
                                /* bytes, or NULL: carved from the plan  */
                                /* workspace                             */
} skei_ei_problem;

/* Scratch one problem needs (for skei_ei_problem.work). */
size_t skei_ei_problem_workspace_bytes(const skei_ei_problem *problem);

typedef struct skei_ei_plan skei_ei_plan;

size_t skei_ei_plan_workspace_bytes(const skei_ei_problem *problems, int count);
int skei_ei_plan_create(const skei_ei_problem *problems, int count, void *work, size_t work_bytes,
                        skei_ei_plan **out);
int skei_ei_plan_destroy(skei_ei_plan *plan);
int skei_ei_plan_run(skei_ei_plan *plan, void *stream);

/* Dispatch of one stage (SKEI_STAGE_*) of a plan:
 *   SKEI_DISPATCH_PERSISTENT: one resident wave of workgroups that draw work
 *     items from per-XCD queues, then steal from the other XCDs' queues;
 *   SKEI_DISPATCH_STATIC: one workgroup per work item, XCD-major ranges.
 * `shape`: for the ray-driven stages (FWD, BP_T) rays per thread (1..4)
 * plus 100 x the image lines per march unit (0 = built-in, 4, 8 or 16; an
 * LDS chunk holds two units), plus 10000 for workgroups of three waves
 * instead of four, plus 20000 for LDS chunks of four units, plus 40000 for
 * six waves or 80000 for eight waves (one or two rays per thread);
 * for the gathers (BP_RESID, ADJ) angle groups per pixel (1, 2, 4) with one
 * pixel per thread, or 10 x groups + 4 (14, 24, 44) with four pixels per
 * thread; 0 keeps the default; ignored by the other stages.  Synchronises the device when
 * the shape changes (the work list is rebuilt). */
enum { SKEI_DISPATCH_PERSISTENT = 0, SKEI_DISPATCH_STATIC = 1 };
int skei_ei_plan_configure(skei_ei_plan *plan, int stage, int dispatch, int shape);
int skei_ei_plan_get_config(const skei_ei_plan *plan, int stage, int *dispatch, int *shape);

/* Autotuner: for every stage, times each (dispatch, shape) candidate on the
 * plan's own problems (hipEvents, median of `reps` launches on `stream`) and
 * keeps the fastest.  Choices are cached per stage under a signature of the
 * stage's work list (sizes, not pointers) -- in memory, and in the text file
 * `cache_path` when it is not NULL (read first, appended to).  It first runs
 * the whole step once so that every candidate is timed on real intermediate
 * values.  Problems' images are never changed: the fused gradient step
 * (skei_ei_problem.step) is left out of every run the tuner makes, and the
 * losses and gradients it leaves behind are those of the unchanged images.
 * Synchronises. */
int skei_ei_plan_autotune(skei_ei_plan *plan, void *stream, int reps, const char *cache_path);

/* Profiling probe for skei_ei_loss_grad and skei_ei_plan_run: when set, the
 * next calls record hipEvent_t `ev_begin` / `ev_end` on their stream
 * immediately before and after the launch of stage `stage` (SKEI_STAGE_*),
 * so a caller can time one kernel inside the fused step with
 * hipEventElapsedTime.  Pass stage < 0 (or null events) to clear.
 * Process-wide setting; not for concurrent callers.
 * Stages of one EI step, in launch order:
 *   ROTATE     z = T x (and z^T), x^T
 *   FWD        A_S z and the MC residual y[mc] - A_mc x (one launch)
 *   RAMP       H A_S z
 *   BP_RESID   r = z - (pi/m) B_S H A_S z
 *   REDUCE     the loss
 *   BP_T       B_S^T r
 *   RAMP_T     (pi/m) H B_S^T r
 *   ADJ        r - A_S^T (...) and A_mc^T r_MC (one launch)
 *   ROTATE_ADJ the gradient */
enum {
    SKEI_STAGE_ROTATE = 0, SKEI_STAGE_FWD = 1, SKEI_STAGE_RAMP = 2, SKEI_STAGE_BP_RESID = 3,
    SKEI_STAGE_REDUCE = 4, SKEI_STAGE_BP_T = 5, SKEI_STAGE_RAMP_T = 6, SKEI_STAGE_ADJ = 7,
    SKEI_STAGE_ROTATE_ADJ = 8, SKEI_STAGE_COUNT = 9
};
int skei_probe_set(int stage, void *ev_begin, void *ev_end);

/* Layout self-check (host only, no device work): walks every LDS read a
 * kernel makes, from the kernel's own layout formulas, for one size.
 *   SKEI_LDS_RAMP, size = N_det (2..2048): out[0..4] = lowest element read,
 *     highest read by a thread that owns an output, highest read by any
 *     thread, last element of the staged row, elements allocated (doubles).
 *   SKEI_LDS_RAY, size = N (2..2032): out[0..2] = lowest and highest
 *     position read within a staged image line, and the line pitch (floats).
 *   SKEI_LDS_GATHER, size = N (2..2032): out[0..2] = lowest and highest
 *     window bin read by the pixel-driven gathers (the interpolation
 *     neighbour included) over every 16 x 16 tile and the angles of 7- and
 *     360-angle tables, and the window length (bins).
 * Returns SKEI_EINVAL / SKEI_ERANGE for a bad kernel or size. */
enum { SKEI_LDS_RAMP = 0, SKEI_LDS_RAY = 1, SKEI_LDS_GATHER = 2 };
int skei_lds_read_bounds(int kernel, int size, long long *out);

#ifdef __cplusplus
}
#endif
#endif /* SKEI_CT_H */

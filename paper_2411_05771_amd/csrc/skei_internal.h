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

// Residual / reduction modes shared by kernels.
enum Mode : int {
    kPlain = 0,      // out = op(in)
    kResidSub = 1,   // out = other - op(in)        (and partial sums of out^2)
};

int check_launch();   // maps hipGetLastError to SKEI_OK / SKEI_ELAUNCH

// ---------------------------------------------------------------- launchers
// All take device pointers and enqueue on `st`.  Shapes are validated by the
// C ABI layer before these are called.

// Launch shape of the ray-driven kernels (0 = automatic choice):
//   group: listed angles per workgroup (they share every staged image chunk)
//   lines: image lines per LDS chunk
//   split: detector segments per angle
struct RayTune {
    int group = 0, lines = 0, split = 0;
};

// Ray-driven Joseph projection (and its MC-residual form):
//   plain:   y[b][r][k] = (A_S x[b])[r][k]
//   resid:   y[b][r][k] = yfull[b][idx[r]][k] - (A_S x[b])[r][k]  (difference taken in double);
//            partial[] = per-workgroup sums of y^2
// xT (optional, may be null): the images transposed, [batch][N][N] with
// xT[b][j][i] = x[b][i][j]; when given, column-stepping angles stage rows of xT
// (contiguous DMA) instead of gathering columns of x.
int launch_radon_fwd(const skei_geom *g, const float *x, const float *xT, int batch, const int32_t *idx, int m,
                     float *y, const float *yfull, double *partial, const RayTune &tune, hipStream_t st);
size_t radon_fwd_partials(const skei_geom *g, int batch, int m, const RayTune &tune);

// Ray-driven B_S^T (unscaled), written as float (qf) or double (qd; exactly one non-null).
int launch_bp_T(const skei_geom *g, const float *x, const float *xT, int batch, const int32_t *idx, int m,
                float *qf, double *qd, const RayTune &tune, hipStream_t st);

// xT[b] = transpose(x[b]) for square N x N images.
int launch_transpose(const float *x, int batch, int n, float *xT, hipStream_t st);

// Pixel-driven gathers over the listed angles.
//   joseph: A_S^T y   ;  bp: scale * B_S q
//   resid:  out = other - op(in)   (partial[] per-block sum of out^2 when partial != nullptr)
int launch_radon_adj(const skei_geom *g, const float *y, int batch, const int32_t *idx, int m,
                     float *x, const float *other, hipStream_t st);
int launch_backproject(const skei_geom *g, const float *q, int batch, const int32_t *idx, int m,
                       float scale, float *x, const float *other, double *partial, hipStream_t st,
                       float *xT = nullptr);
size_t gather_partials(const skei_geom *g, int batch);

// Ram-Lak ramp along rows, double accumulation, times `scale`; the input is
// float (pf) or double (pd; exactly one non-null).
int launch_ramp(const skei_geom *g, const float *pf, const double *pd, int rows, float scale, float *q,
                hipStream_t st);

// Rotation and its transpose (copies summed).  rotate_adj optionally fuses
// g = alpha * sum_c T_c^T h[b][c] + beta * add[b].
// outT (optional): also write every output image transposed.
int launch_rotate(const float *x, int batch, int copies, int n, const float *cs, float *out, hipStream_t st,
                  float *outT = nullptr);
int launch_rotate_adj(const float *h, int batch, int copies, int n, const float *cs, float alpha,
                      const float *add, float beta, float *g, hipStream_t st);

// Deterministic reductions.
size_t sumsq_partials(size_t len);
int launch_sumsq(const float *a, const float *b, size_t len, double *partial, hipStream_t st);
// out = w0 * sum(p0[0..n0)) + w1 * sum(p1[0..n1))  (p1 may be null), fixed order, one block.
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

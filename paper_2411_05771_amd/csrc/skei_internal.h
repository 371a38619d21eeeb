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
    float c, s;      // cos theta, sin theta
    float inv_m;     // 1 / c_m
    float du;        // -c_M / c_m
    float base;      // -cD / c_m + cN (1 + c_M / c_m)
    float scale;     // 1 / |c_m|   (Joseph step length)
    float w;         // |c_m| = max(|cos|, |sin|)
    float inv_w2;    // 1 / w^2
    int rows;        // 1: major axis = image rows
    int pad_[7];
};
static_assert(sizeof(AngleRow) == 64, "AngleRow layout");

// LDS line padding used by the ray-driven kernels: every staged image line
// carries PAD zeros on each side so that clamped tap positions read zeros.
constexpr int kLinePad = 4;

// Pixel tile of the pixel-driven gathers and the detector window they stage.
constexpr int kTile = 16;
constexpr int kWin = 32;
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

// Ray-driven Joseph projection (and its MC-residual form):
//   plain:   y[b][r][k] = (A_S x[b])[r][k]
//   resid:   y[b][r][k] = yfull[b][idx[r]][k] - (A_S x[b])[r][k]; partial[] = per-block sum of y^2
int launch_radon_fwd(const skei_geom *g, const float *x, int batch, const int32_t *idx, int m,
                     float *y, const float *yfull, double *partial, int lines_per_chunk, hipStream_t st);
size_t radon_fwd_partials(const skei_geom *g, int batch, int m);

// Ray-driven B_S^T (unscaled).
int launch_bp_T(const skei_geom *g, const float *x, int batch, const int32_t *idx, int m,
                float *q, int lines_per_chunk, hipStream_t st);

// Pixel-driven gathers over the listed angles.
//   joseph: A_S^T y   ;  bp: scale * B_S q
//   resid:  out = other - op(in)   (partial[] per-block sum of out^2 when partial != nullptr)
int launch_radon_adj(const skei_geom *g, const float *y, int batch, const int32_t *idx, int m,
                     float *x, const float *other, hipStream_t st);
int launch_backproject(const skei_geom *g, const float *q, int batch, const int32_t *idx, int m,
                       float scale, float *x, const float *other, double *partial, hipStream_t st);
size_t gather_partials(const skei_geom *g, int batch);

// Ram-Lak ramp along rows, double accumulation, times `scale`.
int launch_ramp(const skei_geom *g, const float *p, int rows, float scale, float *q, hipStream_t st);

// Rotation and its transpose (copies summed).  rotate_adj optionally fuses
// g = alpha * sum_c T_c^T h[b][c] + beta * add[b].
int launch_rotate(const float *x, int batch, int copies, int n, const float *cs, float *out, hipStream_t st);
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
    skei::AngleRow *tab;   // device [n_angles]
    double *hodd;          // device [n_hodd]: h(2e+1) = -1 / (pi (2e+1))^2
    int n_hodd;
};

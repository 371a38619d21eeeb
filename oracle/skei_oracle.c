/*
 * skei_oracle.c -- plain, slow, double-precision CPU oracle for the sketched
 * EI CT operator path (Xu, Li, Tang, "Equivariant Test-Time Training with
 * Operator Sketching for Imaging Inverse Problems", arXiv 2411.05771).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load
 * or call this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code, header, table or
 * constant with the HIP path.
 *
 * What it computes (every operator is linear, outputs are overwritten):
 *   - Sec. 4.1.1 (sparse-view CT set-up) models CT by a discrete Radon
 *     transform over uniformly spaced angles and uses FBP as the stable
 *     stand-in for A^dagger (Sec. 2.1, problem set-up).  The paper names no
 *     discretisation; this oracle takes Joseph's method (Joseph, IEEE TMI
 *     1(3), 1982) for A, its literal transpose for A^T, the Ram-Lak filter
 *     with unit detector spacing
 *     (Kak & Slaney, Principles of Computerized Tomographic Imaging, ch. 3)
 *     and pixel-driven linear-interpolation backprojection scaled by pi/m
 *     for FBP.
 *   - Sec. 3.1 (sketched EI) defines the sketch S_k as a row selector:
 *     A_S = S A and y_S = S y.  Sec. 4.2.1 draws S_k as interleaved angle
 *     subsets, so a sketch here is a list of angle indices; output rows
 *     follow list order.
 *   - Sec. 4.1.3 takes the transformation group to be image rotations;
 *     T_phi here is bilinear resampling about the image centre, zero fill.
 *   - Eq. (skeilossttt) and Algorithm 2 give the sketched test-time EI loss;
 *     with the network replaced by the identity its value and its gradient
 *     with respect to the image are composed here from the operators above.
 *
 * Geometry (a reading of the paper, which states none of it):
 *   pixel (i, j): centre X_j = j - cN, Y_i = i - cN, cN = (N-1)/2, row i <-> Y;
 *   detector k:   s_k = k - cD, cD = (N_det-1)/2, unit spacing;
 *   angle a:      theta_a = a*pi/N_theta, ray (a,k) = {X cos + Y sin = s_k}.
 *
 * Layouts: image [batch][N][N], sinogram [batch][m][N_det], row-major,
 * float64 throughout.  Parallel loops (OpenMP) only split independent
 * outputs; every output is summed in the same order whatever the thread
 * count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Joseph steps along rows when |cos| >= |sin|.  The comparison is made on the
 * integer angle index so that the 45- and 135-degree ties resolve the same
 * way on every machine (both branches agree there in exact arithmetic). */
static int steps_along_rows(int a, int n_angles)
{
    return 4 * a <= n_angles || 4 * a >= 3 * n_angles;
}

static double angle_of(int a, int n_angles) { return M_PI * (double)a / (double)n_angles; }

/* ---------------------------------------------------------------------- */
/* Forward projection A_S (Joseph's method).                               */
/* For a ray that is closer to the x axis, step over every image row,       */
/* find where the ray crosses the row's centre line, interpolate linearly   */
/* between the two nearest pixel centres of that row, and multiply the sum  */
/* by the step length 1/|cos|.  Otherwise step over columns.  Pixels off    */
/* the image count as zero.                                                 */
/* ---------------------------------------------------------------------- */
static double joseph_ray(const double *img, int n, int n_angles, int a, double s_k)
{
    const double th = angle_of(a, n_angles), c = cos(th), s = sin(th);
    const double cN = 0.5 * (n - 1);
    double acc = 0.0;
    if (steps_along_rows(a, n_angles)) {
        for (int i = 0; i < n; i++) {
            const double Y = i - cN;
            const double u = (s_k - Y * s) / c + cN;      /* column coordinate */
            const double fl = floor(u), f = u - fl;
            const int j = (int)fl;
            if (j >= 0 && j < n) acc += (1.0 - f) * img[(size_t)i * n + j];
            if (j + 1 >= 0 && j + 1 < n) acc += f * img[(size_t)i * n + j + 1];
        }
        return acc / fabs(c);
    }
    for (int j = 0; j < n; j++) {
        const double X = j - cN;
        const double v = (s_k - X * c) / s + cN;          /* row coordinate */
        const double fl = floor(v), f = v - fl;
        const int i = (int)fl;
        if (i >= 0 && i < n) acc += (1.0 - f) * img[(size_t)i * n + j];
        if (i + 1 >= 0 && i + 1 < n) acc += f * img[(size_t)(i + 1) * n + j];
    }
    return acc / fabs(s);
}

void oracle_radon_fwd(const double *x, int batch, int n, int n_angles, int n_det,
                      const int32_t *idx, int m, double *y)
{
    const double cD = 0.5 * (n_det - 1);
#pragma omp parallel for collapse(2) schedule(static)
    for (int b = 0; b < batch; b++)
        for (int r = 0; r < m; r++) {
            const double *img = x + (size_t)b * n * n;
            double *row = y + ((size_t)b * m + r) * n_det;
            for (int k = 0; k < n_det; k++) row[k] = joseph_ray(img, n, n_angles, idx[r], k - cD);
        }
}

/* ---------------------------------------------------------------------- */
/* Adjoint A_S^T: the literal transpose of the loop above -- the same walk, */
/* scattering y/|cos| (or y/|sin|) into the two pixels instead of gathering.*/
/* ---------------------------------------------------------------------- */
static void joseph_ray_scatter(double *img, int n, int n_angles, int a, double s_k, double val)
{
    const double th = angle_of(a, n_angles), c = cos(th), s = sin(th);
    const double cN = 0.5 * (n - 1);
    if (steps_along_rows(a, n_angles)) {
        const double g = val / fabs(c);
        for (int i = 0; i < n; i++) {
            const double Y = i - cN;
            const double u = (s_k - Y * s) / c + cN;
            const double fl = floor(u), f = u - fl;
            const int j = (int)fl;
            if (j >= 0 && j < n) img[(size_t)i * n + j] += (1.0 - f) * g;
            if (j + 1 >= 0 && j + 1 < n) img[(size_t)i * n + j + 1] += f * g;
        }
        return;
    }
    const double g = val / fabs(s);
    for (int j = 0; j < n; j++) {
        const double X = j - cN;
        const double v = (s_k - X * c) / s + cN;
        const double fl = floor(v), f = v - fl;
        const int i = (int)fl;
        if (i >= 0 && i < n) img[(size_t)i * n + j] += (1.0 - f) * g;
        if (i + 1 >= 0 && i + 1 < n) img[(size_t)(i + 1) * n + j] += f * g;
    }
}

void oracle_radon_adj(const double *y, int batch, int n, int n_angles, int n_det,
                      const int32_t *idx, int m, double *x)
{
    const double cD = 0.5 * (n_det - 1);
#pragma omp parallel for schedule(static)
    for (int b = 0; b < batch; b++) {
        double *img = x + (size_t)b * n * n;
        memset(img, 0, sizeof(double) * (size_t)n * n);
        for (int r = 0; r < m; r++)
            for (int k = 0; k < n_det; k++)
                joseph_ray_scatter(img, n, n_angles, idx[r], k - cD, y[((size_t)b * m + r) * n_det + k]);
    }
}

/* ---------------------------------------------------------------------- */
/* Ram-Lak filter H, spatial domain, unit detector spacing:                 */
/*   h(0) = 1/4,  h(n) = -1/(pi^2 n^2) for odd n,  h(n) = 0 for even n != 0  */
/* applied as a linear (zero-padded, never circular) convolution along each */
/* detector row: q[k] = sum_j h(k - j) p[j].                                */
/* ---------------------------------------------------------------------- */
double oracle_ramlak_tap(int n)
{
    if (n == 0) return 0.25;
    if (n % 2 == 0) return 0.0;
    return -1.0 / (M_PI * M_PI * (double)n * (double)n);
}

void oracle_ramp(const double *p, int rows, int n_det, double *q)
{
#pragma omp parallel for schedule(static)
    for (int r = 0; r < rows; r++) {
        const double *in = p + (size_t)r * n_det;
        double *out = q + (size_t)r * n_det;
        for (int k = 0; k < n_det; k++) {
            double acc = 0.0;
            for (int j = 0; j < n_det; j++) acc += oracle_ramlak_tap(k - j) * in[j];
            out[k] = acc;
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Pixel-driven backprojection B_S (no scale): each pixel centre projects   */
/* onto t = X cos + Y sin + cD on the detector axis of every listed angle,  */
/* and takes the linear interpolation of that row at t (zero off the        */
/* detector).  B_S^T is its literal transpose (scatter).                    */
/* ---------------------------------------------------------------------- */
void oracle_backproject(const double *q, int batch, int n, int n_angles, int n_det,
                        const int32_t *idx, int m, double *x)
{
    const double cN = 0.5 * (n - 1), cD = 0.5 * (n_det - 1);
#pragma omp parallel for collapse(2) schedule(static)
    for (int b = 0; b < batch; b++)
        for (int i = 0; i < n; i++) {
            for (int j = 0; j < n; j++) {
                const double X = j - cN, Y = i - cN;
                double acc = 0.0;
                for (int r = 0; r < m; r++) {
                    const double th = angle_of(idx[r], n_angles);
                    const double t = X * cos(th) + Y * sin(th) + cD;
                    const double fl = floor(t), f = t - fl;
                    const int k = (int)fl;
                    const double *row = q + ((size_t)b * m + r) * n_det;
                    if (k >= 0 && k < n_det) acc += (1.0 - f) * row[k];
                    if (k + 1 >= 0 && k + 1 < n_det) acc += f * row[k + 1];
                }
                x[((size_t)b * n + i) * n + j] = acc;
            }
        }
}

void oracle_backproject_T(const double *x, int batch, int n, int n_angles, int n_det,
                          const int32_t *idx, int m, double *q)
{
    const double cN = 0.5 * (n - 1), cD = 0.5 * (n_det - 1);
#pragma omp parallel for collapse(2) schedule(static)
    for (int b = 0; b < batch; b++)
        for (int r = 0; r < m; r++) {
            double *row = q + ((size_t)b * m + r) * n_det;
            memset(row, 0, sizeof(double) * (size_t)n_det);
            const double th = angle_of(idx[r], n_angles);
            for (int i = 0; i < n; i++)
                for (int j = 0; j < n; j++) {
                    const double X = j - cN, Y = i - cN;
                    const double t = X * cos(th) + Y * sin(th) + cD;
                    const double fl = floor(t), f = t - fl;
                    const int k = (int)fl;
                    const double v = x[((size_t)b * n + i) * n + j];
                    if (k >= 0 && k < n_det) row[k] += (1.0 - f) * v;
                    if (k + 1 >= 0 && k + 1 < n_det) row[k + 1] += f * v;
                }
        }
}

/* fbp_S = (pi/m) B_S H   and its transpose (pi/m) H B_S^T (H is symmetric). */
void oracle_fbp(const double *y, int batch, int n, int n_angles, int n_det,
                const int32_t *idx, int m, double *x)
{
    double *q = malloc(sizeof(double) * (size_t)batch * m * n_det);
    oracle_ramp(y, batch * m, n_det, q);
    oracle_backproject(q, batch, n, n_angles, n_det, idx, m, x);
    const double scale = M_PI / (double)m;
    for (size_t p = 0; p < (size_t)batch * n * n; p++) x[p] *= scale;
    free(q);
}

void oracle_fbp_adj(const double *x, int batch, int n, int n_angles, int n_det,
                    const int32_t *idx, int m, double *y)
{
    double *g = malloc(sizeof(double) * (size_t)batch * m * n_det);
    oracle_backproject_T(x, batch, n, n_angles, n_det, idx, m, g);
    oracle_ramp(g, batch * m, n_det, y);
    const double scale = M_PI / (double)m;
    for (size_t p = 0; p < (size_t)batch * m * n_det; p++) y[p] *= scale;
    free(g);
}

/* ---------------------------------------------------------------------- */
/* Rotation T_phi: out(p) = x(R(-phi) p) by bilinear interpolation between  */
/* pixel centres, zero outside.  With cos/sin of phi (c, s):                */
/*   u = c X + s Y + cN  (column),  v = -s X + c Y + cN  (row).             */
/* out[b][cp] = T_{phi_cp} x[b];  the transpose sums over the copies:       */
/* g[b] = sum_cp T_{phi_cp}^T h[b][cp].                                     */
/* ---------------------------------------------------------------------- */
void oracle_rotate(const double *x, int batch, int copies, int n, const double *cos_sin, double *out)
{
    const double cN = 0.5 * (n - 1);
#pragma omp parallel for collapse(2) schedule(static)
    for (int b = 0; b < batch; b++)
        for (int cp = 0; cp < copies; cp++) {
            const double c = cos_sin[2 * cp], s = cos_sin[2 * cp + 1];
            const double *img = x + (size_t)b * n * n;
            double *o = out + ((size_t)b * copies + cp) * n * n;
            for (int i = 0; i < n; i++)
                for (int j = 0; j < n; j++) {
                    const double X = j - cN, Y = i - cN;
                    const double u = c * X + s * Y + cN, v = -s * X + c * Y + cN;
                    const double fu = floor(u), fv = floor(v);
                    const double au = u - fu, av = v - fv;
                    const int j0 = (int)fu, i0 = (int)fv;
                    double acc = 0.0;
                    for (int di = 0; di < 2; di++)
                        for (int dj = 0; dj < 2; dj++) {
                            const int ii = i0 + di, jj = j0 + dj;
                            if (ii < 0 || ii >= n || jj < 0 || jj >= n) continue;
                            const double w = (di ? av : 1.0 - av) * (dj ? au : 1.0 - au);
                            acc += w * img[(size_t)ii * n + jj];
                        }
                    o[(size_t)i * n + j] = acc;
                }
        }
}

void oracle_rotate_adj(const double *h, int batch, int copies, int n, const double *cos_sin, double *g)
{
    const double cN = 0.5 * (n - 1);
#pragma omp parallel for schedule(static)
    for (int b = 0; b < batch; b++) {
        double *img = g + (size_t)b * n * n;
        memset(img, 0, sizeof(double) * (size_t)n * n);
        for (int cp = 0; cp < copies; cp++) {
            const double c = cos_sin[2 * cp], s = cos_sin[2 * cp + 1];
            const double *hin = h + ((size_t)b * copies + cp) * n * n;
            for (int i = 0; i < n; i++)
                for (int j = 0; j < n; j++) {
                    const double X = j - cN, Y = i - cN;
                    const double u = c * X + s * Y + cN, v = -s * X + c * Y + cN;
                    const double fu = floor(u), fv = floor(v);
                    const double au = u - fu, av = v - fv;
                    const int j0 = (int)fu, i0 = (int)fv;
                    const double val = hin[(size_t)i * n + j];
                    for (int di = 0; di < 2; di++)
                        for (int dj = 0; dj < 2; dj++) {
                            const int ii = i0 + di, jj = j0 + dj;
                            if (ii < 0 || ii >= n || jj < 0 || jj >= n) continue;
                            const double w = (di ? av : 1.0 - av) * (dj ? au : 1.0 - au);
                            img[(size_t)ii * n + jj] += w * val;
                        }
                }
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Sketched test-time EI loss with the network taken as the identity        */
/* (Eq. skeilossttt; Algorithm 2, one iteration), for an image batch x:     */
/*                                                                          */
/*   r_MC[b]    = y[b][mc_idx] - A_{mc_idx} x[b]                            */
/*   z[b][c]    = T_c x[b]                                                  */
/*   r[b][c]    = z[b][c] - fbp_S(A_S z[b][c])                              */
/*   L          = sum_b ( ||r_MC[b]||^2 + (lambda/C) sum_c ||r[b][c]||^2 )  */
/*   dL/dx[b]   = -2 A_mc^T r_MC[b]                                         */
/*                + (2 lambda/C) sum_c T_c^T ( r[b][c] - A_S^T fbp_S^T r )  */
/*                                                                          */
/* y is the full measured sinogram [batch][n_angles][n_det]; the MC term    */
/* reads the rows listed in mc_idx (all angles for the unsketched MC term,  */
/* or the sketch itself for the sketched MC term of Algorithm 2).  Sums of  */
/* squares are plain l2^2 (no mean).  grad may be NULL.                     */
/* ---------------------------------------------------------------------- */
static double sumsq(const double *v, size_t len)
{
    double acc = 0.0;
    for (size_t p = 0; p < len; p++) acc += v[p] * v[p];
    return acc;
}

double oracle_ei_loss_grad(const double *x, const double *y, int batch, int n, int n_angles, int n_det,
                           const int32_t *mc_idx, int m_mc, const int32_t *idx, int m,
                           int copies, const double *cos_sin, double lambda, double *grad)
{
    const size_t img = (size_t)n * n;
    double loss = 0.0;
    double *axv = malloc(sizeof(double) * (size_t)m_mc * n_det);
    double *rmc = malloc(sizeof(double) * (size_t)m_mc * n_det);
    double *z = malloc(sizeof(double) * (size_t)copies * img);
    double *ys = malloc(sizeof(double) * (size_t)copies * m * n_det);
    double *w = malloc(sizeof(double) * (size_t)copies * img);
    double *t1 = malloc(sizeof(double) * (size_t)copies * m * n_det);
    double *t2 = malloc(sizeof(double) * (size_t)copies * img);
    double *g1 = malloc(sizeof(double) * img);
    for (int b = 0; b < batch; b++) {
        const double *xb = x + (size_t)b * img;
        const double *yb = y + (size_t)b * n_angles * n_det;
        /* measurement consistency */
        oracle_radon_fwd(xb, 1, n, n_angles, n_det, mc_idx, m_mc, axv);
        for (int r = 0; r < m_mc; r++)
            for (int k = 0; k < n_det; k++)
                rmc[(size_t)r * n_det + k] = yb[(size_t)mc_idx[r] * n_det + k] - axv[(size_t)r * n_det + k];
        double l_mc = sumsq(rmc, (size_t)m_mc * n_det);
        /* sketched equivariance term */
        oracle_rotate(xb, 1, copies, n, cos_sin, z);
        oracle_radon_fwd(z, copies, n, n_angles, n_det, idx, m, ys);
        oracle_fbp(ys, copies, n, n_angles, n_det, idx, m, w);
        for (size_t p = 0; p < (size_t)copies * img; p++) w[p] = z[p] - w[p];   /* w <- r */
        double l_ei = sumsq(w, (size_t)copies * img);
        loss += l_mc + lambda / copies * l_ei;
        if (!grad) continue;
        double *gb = grad + (size_t)b * img;
        oracle_radon_adj(rmc, 1, n, n_angles, n_det, mc_idx, m_mc, gb);
        for (size_t p = 0; p < img; p++) gb[p] *= -2.0;
        oracle_fbp_adj(w, copies, n, n_angles, n_det, idx, m, t1);
        oracle_radon_adj(t1, copies, n, n_angles, n_det, idx, m, t2);
        for (size_t p = 0; p < (size_t)copies * img; p++) t2[p] = w[p] - t2[p];
        oracle_rotate_adj(t2, 1, copies, n, cos_sin, g1);
        const double scale = 2.0 * lambda / copies;
        for (size_t p = 0; p < img; p++) gb[p] += scale * g1[p];
    }
    free(axv); free(rmc); free(z); free(ys); free(w); free(t1); free(t2); free(g1);
    return loss;
}

// C ABI entry points (include/skei_ct.h): argument validation, workspace
// carving and kernel launch sequences.  Nothing here allocates device memory.
#include <cmath>
#include <cstdint>

#include "skei_internal.h"

using namespace skei;

namespace {

constexpr double kPi = 3.14159265358979323846;

inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

int check_geom_op(const skei_geom *g, const void *in, int batch, const int32_t *idx, int m, const void *out)
{
    if (!g || !in || !out || !idx) return SKEI_EINVAL;
    if (batch <= 0 || m <= 0) return SKEI_EINVAL;
    if (batch > 65535 || m > 2147483647 / 2) return SKEI_ERANGE;
    return SKEI_OK;
}

// Carves a caller workspace into 256-byte aligned pieces.
struct Carver {
    char *p;
    size_t left;
    bool ok = true;
    template <typename T>
    T *take(size_t count)
    {
        const size_t b = align256(count * sizeof(T));
        if (!p || b > left) {
            ok = false;
            return nullptr;
        }
        T *r = reinterpret_cast<T *>(p);
        p += b;
        left -= b;
        return r;
    }
};

struct EiSizes {
    size_t img, sino, mc, part_mc, part_ei, total;
};

EiSizes ei_sizes(const skei_geom *g, int batch, int m_mc, int m, int copies)
{
    EiSizes s;
    const size_t nn = (size_t)g->n * g->n;
    const size_t bc = (size_t)batch * copies;
    s.img = bc * nn;
    s.sino = bc * (size_t)m * g->n_det;
    s.mc = (size_t)batch * m_mc * g->n_det;
    s.part_mc = radon_fwd_partials(g, batch, m_mc, g->tune_fwd);
    s.part_ei = gather_partials(g, (int)bc);
    s.total = align256(s.img * 4) * 4            // z (later d), zT, r, rT
              + align256(nn * batch * 4)         // xT
              + align256(s.sino * 8)             // ys (A_S z as float, later B_S^T r as double)
              + align256(s.sino * 4)             // qs (H ys, later (pi/m) H B_S^T r)
              + align256(s.mc * 4)               // r_MC
              + align256(nn * batch * 4)         // A_mc^T r_MC
              + align256(s.part_mc * 8) + align256(s.part_ei * 8);
    return s;
}

struct Probe {
    int stage = -1;
    hipEvent_t b = nullptr, e = nullptr;
};
Probe g_probe;

// Launch stage `stage` of the EI step through `fn`, bracketed by the probe's
// events when the probe targets it.
template <typename F>
int staged(int stage, hipStream_t st, F &&fn)
{
    const bool on = g_probe.stage == stage && g_probe.b && g_probe.e;
    if (on && hipEventRecord(g_probe.b, st) != hipSuccess) return SKEI_ELAUNCH;
    const int rc = fn();
    if (rc) return rc;
    if (on && hipEventRecord(g_probe.e, st) != hipSuccess) return SKEI_ELAUNCH;
    return SKEI_OK;
}

}  // namespace

extern "C" {

int skei_probe_set(int stage, void *ev_begin, void *ev_end)
{
    if (stage >= SKEI_STAGE_COUNT) return SKEI_EINVAL;
    g_probe.stage = stage;
    g_probe.b = static_cast<hipEvent_t>(ev_begin);
    g_probe.e = static_cast<hipEvent_t>(ev_end);
    return SKEI_OK;
}

int skei_radon_fwd(const skei_geom *g, const float *x, int batch, const int32_t *angle_idx, int m, float *y,
                   void *stream)
{
    int rc = check_geom_op(g, x, batch, angle_idx, m, y);
    if (rc) return rc;
    return launch_radon_fwd(g, x, nullptr, batch, angle_idx, m, y, nullptr, nullptr, g->tune_fwd, S(stream));
}

int skei_radon_adj(const skei_geom *g, const float *y, int batch, const int32_t *angle_idx, int m, float *x,
                   void *stream)
{
    int rc = check_geom_op(g, y, batch, angle_idx, m, x);
    if (rc) return rc;
    return launch_radon_adj(g, y, batch, angle_idx, m, x, nullptr, S(stream));
}

int skei_ramp(const skei_geom *g, const float *p, int rows, float *q, void *stream)
{
    if (!g || !p || !q || rows <= 0) return SKEI_EINVAL;
    return launch_ramp(g, p, nullptr, rows, 1.0f, q, S(stream));
}

int skei_backproject(const skei_geom *g, const float *q, int batch, const int32_t *angle_idx, int m, float *x,
                     void *stream)
{
    int rc = check_geom_op(g, q, batch, angle_idx, m, x);
    if (rc) return rc;
    return launch_backproject(g, q, batch, angle_idx, m, 1.0f, x, nullptr, nullptr, S(stream));
}

int skei_backproject_T(const skei_geom *g, const float *x, int batch, const int32_t *angle_idx, int m, float *q,
                       void *stream)
{
    int rc = check_geom_op(g, x, batch, angle_idx, m, q);
    if (rc) return rc;
    return launch_bp_T(g, x, nullptr, batch, angle_idx, m, q, nullptr, g->tune_bpt, S(stream));
}

size_t skei_fbp_workspace_bytes(const skei_geom *g, int batch, int m)
{
    if (!g || batch <= 0 || m <= 0) return 0;
    // fbp keeps the filtered sinogram (float); fbp_adj keeps B_S^T x in double
    // (so that the high-pass ramp does not amplify its rounding) and the
    // transposed images (contiguous staging for column-stepping angles)
    return align256((size_t)batch * m * g->n_det * sizeof(double)) +
           align256((size_t)batch * g->n * g->n * sizeof(float));
}

int skei_fbp(const skei_geom *g, const float *y, int batch, const int32_t *angle_idx, int m, float *x, void *work,
             size_t work_bytes, void *stream)
{
    int rc = check_geom_op(g, y, batch, angle_idx, m, x);
    if (rc) return rc;
    if (!work) return SKEI_EINVAL;
    if (work_bytes < skei_fbp_workspace_bytes(g, batch, m)) return SKEI_ESPACE;
    float *q = static_cast<float *>(work);
    rc = launch_ramp(g, y, nullptr, batch * m, 1.0f, q, S(stream));
    if (rc) return rc;
    return launch_backproject(g, q, batch, angle_idx, m, (float)(kPi / m), x, nullptr, nullptr, S(stream));
}

int skei_fbp_adj(const skei_geom *g, const float *x, int batch, const int32_t *angle_idx, int m, float *y,
                 void *work, size_t work_bytes, void *stream)
{
    int rc = check_geom_op(g, x, batch, angle_idx, m, y);
    if (rc) return rc;
    if (!work) return SKEI_EINVAL;
    if (work_bytes < skei_fbp_workspace_bytes(g, batch, m)) return SKEI_ESPACE;
    double *t = static_cast<double *>(work);
    float *xT = reinterpret_cast<float *>(static_cast<char *>(work) +
                                          align256((size_t)batch * m * g->n_det * sizeof(double)));
    rc = launch_transpose(x, batch, g->n, xT, S(stream));
    if (rc) return rc;
    rc = launch_bp_T(g, x, xT, batch, angle_idx, m, nullptr, t, g->tune_bpt, S(stream));
    if (rc) return rc;
    return launch_ramp(g, nullptr, t, batch * m, (float)(kPi / m), y, S(stream));
}

int skei_rotate(const float *x, int batch, int copies, int n, const float *cos_sin, float *out, void *stream)
{
    if (!x || !cos_sin || !out || batch <= 0 || copies <= 0 || n < 2) return SKEI_EINVAL;
    if ((size_t)batch * copies > 65535 || n > 16384) return SKEI_ERANGE;
    return launch_rotate(x, batch, copies, n, cos_sin, out, S(stream));
}

int skei_rotate_adj(const float *h, int batch, int copies, int n, const float *cos_sin, float *g, void *stream)
{
    if (!h || !cos_sin || !g || batch <= 0 || copies <= 0 || n < 2) return SKEI_EINVAL;
    if (batch > 65535 || n > 16384) return SKEI_ERANGE;
    return launch_rotate_adj(h, batch, copies, n, cos_sin, 1.0f, nullptr, 0.0f, g, S(stream));
}

size_t skei_sumsq_workspace_bytes(size_t len) { return align256(sumsq_partials(len) * sizeof(double)); }

int skei_sumsq_diff(const float *a, const float *b, size_t len, double *out, void *work, size_t work_bytes,
                    void *stream)
{
    if (!a || !out || !work || len == 0) return SKEI_EINVAL;
    if (work_bytes < skei_sumsq_workspace_bytes(len)) return SKEI_ESPACE;
    double *part = static_cast<double *>(work);
    int rc = launch_sumsq(a, b, len, part, S(stream));
    if (rc) return rc;
    return launch_reduce2(part, sumsq_partials(len), 1.0, nullptr, 0, 0.0, out, S(stream));
}

size_t skei_ei_workspace_bytes(const skei_geom *g, int batch, int m_mc, int m, int copies)
{
    if (!g || batch <= 0 || m_mc <= 0 || m <= 0 || copies <= 0) return 0;
    return ei_sizes(g, batch, m_mc, m, copies).total;
}

int skei_ei_loss_grad(const skei_geom *g, const float *x, const float *y, int batch, const int32_t *mc_idx,
                      int m_mc, const int32_t *angle_idx, int m, int copies, const float *cos_sin, float lambda,
                      double *loss, float *grad, void *work, size_t work_bytes, void *stream)
{
    if (!g || !x || !y || !mc_idx || !angle_idx || !cos_sin || !loss || !work) return SKEI_EINVAL;
    if (batch <= 0 || m_mc <= 0 || m <= 0 || copies <= 0) return SKEI_EINVAL;
    if ((size_t)batch * copies > 65535) return SKEI_ERANGE;
    const EiSizes sz = ei_sizes(g, batch, m_mc, m, copies);
    if (work_bytes < sz.total) return SKEI_ESPACE;
    Carver cv{static_cast<char *>(work), work_bytes};
    float *z = cv.take<float>(sz.img);
    float *zT = cv.take<float>(sz.img);
    float *r = cv.take<float>(sz.img);
    float *rT = cv.take<float>(sz.img);
    float *xT = cv.take<float>((size_t)g->n * g->n * batch);
    double *ysd = cv.take<double>(sz.sino);
    float *ys = reinterpret_cast<float *>(ysd);
    float *qs = cv.take<float>(sz.sino);
    float *rmc = cv.take<float>(sz.mc);
    float *amc = cv.take<float>((size_t)g->n * g->n * batch);
    double *pmc = cv.take<double>(sz.part_mc);
    double *pei = cv.take<double>(sz.part_ei);
    if (!cv.ok) return SKEI_ESPACE;

    const hipStream_t st = S(stream);
    const int bc = batch * copies;
    const float pim = (float)(kPi / m);
    int rc;
    // forward: z = T x ; ys = A_S z ; qs = H ys ; r = z - (pi/m) B_S qs ; r_MC = y[mc] - A_mc x
    if ((rc = staged(SKEI_STAGE_ROTATE, st, [&] { return launch_rotate(x, batch, copies, g->n, cos_sin, z, st, zT); })))
        return rc;
    if ((rc = staged(SKEI_STAGE_FWD_SKETCH, st,
                     [&] { return launch_radon_fwd(g, z, zT, bc, angle_idx, m, ys, nullptr, nullptr, g->tune_fwd, st); })))
        return rc;
    if ((rc = staged(SKEI_STAGE_RAMP, st, [&] { return launch_ramp(g, ys, nullptr, bc * m, 1.0f, qs, st); }))) return rc;
    if ((rc = staged(SKEI_STAGE_BP_RESID, st,
                     [&] { return launch_backproject(g, qs, bc, angle_idx, m, pim, r, z, pei, st, rT); })))
        return rc;
    if ((rc = staged(SKEI_STAGE_FWD_MC, st,
                     [&] {
                         int rc2 = launch_transpose(x, batch, g->n, xT, st);
                         if (rc2) return rc2;
                         return launch_radon_fwd(g, x, xT, batch, mc_idx, m_mc, rmc, y, pmc, g->tune_fwd, st);
                     })))
        return rc;
    if ((rc = staged(SKEI_STAGE_REDUCE, st, [&] {
             return launch_reduce2(pmc, sz.part_mc, 1.0, pei, sz.part_ei, (double)lambda / copies, loss, st);
         })))
        return rc;
    if (!grad) return SKEI_OK;
    // backward: ys = B_S^T r ; qs = (pi/m) H ys ; z = r - A_S^T qs ;
    //           amc = A_mc^T r_MC ; grad = (2 lambda / C) sum_c T_c^T z - 2 amc
    if ((rc = staged(SKEI_STAGE_BP_T, st, [&] { return launch_bp_T(g, r, rT, bc, angle_idx, m, nullptr, ysd, g->tune_bpt, st); })))
        return rc;
    if ((rc = staged(SKEI_STAGE_RAMP_T, st, [&] { return launch_ramp(g, nullptr, ysd, bc * m, pim, qs, st); }))) return rc;
    if ((rc = staged(SKEI_STAGE_ADJ_SKETCH, st,
                     [&] { return launch_radon_adj(g, qs, bc, angle_idx, m, z, r, st); })))
        return rc;
    if ((rc = staged(SKEI_STAGE_ADJ_MC, st,
                     [&] { return launch_radon_adj(g, rmc, batch, mc_idx, m_mc, amc, nullptr, st); })))
        return rc;
    return staged(SKEI_STAGE_ROTATE_ADJ, st, [&] {
        return launch_rotate_adj(z, batch, copies, g->n, cos_sin, 2.0f * lambda / copies, amc, -2.0f, grad, st);
    });
}

}  // extern "C"

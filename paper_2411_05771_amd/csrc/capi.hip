// C ABI entry points (include/skei_ct.h): argument validation, workspace
// carving and kernel launch sequences.  Nothing here allocates device memory.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>

#include "ei_step.h"
#include "skei_internal.h"

using namespace skei;

namespace {

constexpr double kPi = 3.14159265358979323846;

inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

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

struct Probe {
    int stage = -1;
    hipEvent_t b = nullptr, e = nullptr;
};
Probe g_probe;

}  // namespace

namespace skei {

int probe_begin(int stage, hipStream_t st)
{
    const bool on = g_probe.stage == stage && g_probe.b && g_probe.e;
    if (on && hipEventRecord(g_probe.b, st) != hipSuccess) return SKEI_ELAUNCH;
    return SKEI_OK;
}

int probe_end(int stage, hipStream_t st)
{
    const bool on = g_probe.stage == stage && g_probe.b && g_probe.e;
    if (on && hipEventRecord(g_probe.e, st) != hipSuccess) return SKEI_ELAUNCH;
    return SKEI_OK;
}

namespace {

struct EiSizes {
    size_t img, sino, mc, part_mc, part_ei;
};

EiSizes ei_sizes(const skei_geom *g, int batch, int m_mc, int m, int copies)
{
    EiSizes s;
    const size_t nn = (size_t)g->n * g->n;
    const size_t bc = (size_t)batch * copies;
    s.img = bc * nn;
    s.sino = bc * (size_t)m * g->n_det;
    s.mc = (size_t)batch * m_mc * g->n_det;
    s.part_mc = (size_t)batch * m_mc;   // one per r_MC row
    s.part_ei = gather_items(g->n, (int)bc);
    return s;
}

}  // namespace

size_t ei_workspace_bytes(const skei_geom *g, int batch, int m_mc, int m, int copies)
{
    const EiSizes s = ei_sizes(g, batch, m_mc, m, copies);
    const size_t nn = (size_t)g->n * g->n;
    return align256(s.img * 4) * 4          // z (later d), zT, r, rT
           + align256(nn * batch * 4)       // xT
           + align256(s.sino * 8)           // ys (A_S z as float, later B_S^T r as double)
           + align256(s.sino * 4)           // qs (H ys, later (pi/m) H B_S^T r)
           + align256(s.mc * 4)             // r_MC
           + align256(nn * batch * 4)       // A_mc^T r_MC
           + align256(s.part_mc * 8) + align256(s.part_ei * 8);
}

bool ei_carve(const skei_geom *g, int batch, int m_mc, int m, int copies, void *work, size_t bytes, EiBuffers &b)
{
    const EiSizes sz = ei_sizes(g, batch, m_mc, m, copies);
    const size_t nn = (size_t)g->n * g->n;
    Carver cv{static_cast<char *>(work), bytes};
    b.z = cv.take<float>(sz.img);
    b.zT = cv.take<float>(sz.img);
    b.r = cv.take<float>(sz.img);
    b.rT = cv.take<float>(sz.img);
    b.xT = cv.take<float>(nn * batch);
    b.ysd = cv.take<double>(sz.sino);
    b.ys = reinterpret_cast<float *>(b.ysd);
    b.qs = cv.take<float>(sz.sino);
    b.rmc = cv.take<float>(sz.mc);
    b.amc = cv.take<float>(nn * batch);
    b.pmc = cv.take<double>(sz.part_mc);
    b.pei = cv.take<double>(sz.part_ei);
    b.n_pmc = sz.part_mc;
    b.n_pei = sz.part_ei;
    return cv.ok;
}

int ei_problem_jobs(const skei_ei_problem &p, const EiBuffers &b, const RayChoice &fwd, const RayChoice &bpt,
                    EiJobs &J)
{
    const skei_geom *g = p.geom;
    const int n = g->n, batch = p.batch, copies = p.copies, m = p.m, m_mc = p.m_mc;
    const int bc = batch * copies;
    const float pim = (float)(kPi / m);
    int rc;
    // forward: z = T x ; ys = A_S z ; r_MC = y[mc] - A_mc x ; qs = H ys ;
    //          r = z - (pi/m) B_S qs ; loss
    J.rot[0] = make_rot_job(p.x, batch, copies, n, p.cos_sin, b.z, b.zT);
    J.rot[1] = make_rot_job(p.x, batch, 1, n, nullptr, nullptr, b.xT);
    RayTune tf = g->tune_fwd, tb = g->tune_bpt;
    // built-in march units when the geometry is not tuned (the autotuner's
    // MI355X choices at 256 x 256): 8 lines, two units per LDS chunk for the
    // forward; 4 lines, four units per chunk for B^T up to 512 (8 lines and
    // two units above, for occupancy)
    if (tf.lines == 0) tf.lines = 8;
    if (tb.lines == 0) {
        tb.lines = n <= 512 ? 4 : 8;
        tb.units = n <= 512 ? 4 : 2;
    }
    if (!fwd.own) {
        tf = RayTune{};
        tf.lines = fwd.lines;
        tf.waves = fwd.waves;
        tf.units = fwd.units;
    }
    if (!bpt.own) {
        tb = RayTune{};
        tb.lines = bpt.lines;
        tb.waves = bpt.waves;
        tb.units = bpt.units;
    }
    // Without a tuning of the geometry, the ray jobs take the plans' default
    // rays per thread (one angle per item for N_det up to the slots): items
    // holding several angles measured markedly slower than one-angle items.
    const long long rows_f = (long long)bc * m + (long long)batch * m_mc, rows_b = (long long)bc * m;
    const int rpt_f = fwd.own && tf.group == 0 && tf.split == 0 ? ray_rpt_default(g->n_det, rows_f, false) : fwd.rpt;
    const int rpt_b = bpt.own && tb.group == 0 && tb.split == 0 ? ray_rpt_default(g->n_det, rows_b, true) : bpt.rpt;
    if ((rc = make_ray_job(g, b.z, b.zT, bc, p.angle_idx, m, b.ys, nullptr, tf, rpt_f, J.fwd[0],
                           J.fwd_shape[0])))
        return rc;
    tf.waves = J.fwd_shape[0].waves;   // both jobs of the launch share the workgroup size
    if ((rc = make_ray_job(g, p.x, b.xT, batch, p.mc_idx, m_mc, b.rmc, p.y, tf, rpt_f, J.fwd[1],
                           J.fwd_shape[1])))
        return rc;
    // ||r_MC||^2 as row sums in a fixed order (in the ramp launch): the loss
    // is bitwise the same under every launch shape
    const long long mc_rows = (long long)batch * m_mc;
    if ((size_t)mc_rows > b.n_pmc) return SKEI_ERANGE;
    J.ramp[0] = make_ramp_job(g, b.ys, (long long)bc * m, 1.0f, b.qs);
    J.ramp[1] = make_row_sumsq_job(g, b.rmc, mc_rows, b.pmc);
    J.bp = make_gather_job(g, b.qs, bc, p.angle_idx, m, pim, b.r, b.z, b.pei, b.rT);
    J.red = RedJob{};
    J.red.p0 = b.pmc;
    J.red.n0 = mc_rows;
    J.red.w0 = 1.0;
    J.red.p1 = b.pei;
    J.red.n1 = J.bp.items;
    J.red.w1 = (double)p.lambda / copies;
    J.red.out = p.loss;
    J.red.items = 1;
    // backward: ysd = B_S^T r ; qs = (pi/m) H ysd ; z = r - A_S^T qs ;
    //           amc = A_mc^T r_MC ; grad = (2 lambda / C) sum_c T_c^T z - 2 amc
    J.grad = p.grad != nullptr;
    if ((rc = make_ray_job(g, b.r, b.rT, bc, p.angle_idx, m, b.ysd, nullptr, tb, rpt_b, J.bpt,
                           J.bpt_shape)))
        return rc;
    J.rampT = make_ramp_job(g, b.ysd, (long long)bc * m, pim, b.qs);
    J.adj[0] = make_gather_job(g, b.qs, bc, p.angle_idx, m, 1.0f, b.z, b.r, nullptr, nullptr);
    J.adj[1] = make_gather_job(g, b.rmc, batch, p.mc_idx, m_mc, 1.0f, b.amc, nullptr, nullptr, nullptr);
    J.radj = make_rot_adj_job(b.z, batch, copies, n, p.cos_sin, 2.0f * p.lambda / copies, b.amc, -2.0f, p.grad);
    if (p.step != 0.0f && p.grad) {
        J.radj.x_upd = p.x;
        J.radj.step = p.step;
    }
    return SKEI_OK;
}

// Scratch of the no-allocation EI entry point: a file-scope device array,
// so the call itself allocates nothing (for callers that cannot allocate:
// graph capture, tight serving loops).  Each device that loads the library
// holds its own copy until the process ends.  In host code `scratch` is
// only a stand-in for the symbol; its device address on the current device
// comes from hipGetSymbolAddress, looked up once per device and cached.
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

int noalloc_scratch(void **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SKEI_ELAUNCH;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SKEI_ELAUNCH;
        addr[dev] = ptr;
    }
    *out = addr[dev];
    return SKEI_OK;
}

int ei_loss_grad_impl(const skei_geom *g, const float *x, const float *y, int batch, const int32_t *mc_idx,
                      int m_mc, const int32_t *angle_idx, int m, int copies, const float *cos_sin, float lambda,
                      double *loss, float *grad, void *work, size_t work_bytes, void *stream)
{
    if (!g || !x || !y || !mc_idx || !angle_idx || !cos_sin || !loss || !work) return SKEI_EINVAL;
    if (batch <= 0 || m_mc <= 0 || m <= 0 || copies <= 0) return SKEI_EINVAL;
    if ((size_t)batch * copies > 65535) return SKEI_ERANGE;
    EiBuffers b;
    if (!ei_carve(g, batch, m_mc, m, copies, work, work_bytes, b)) return SKEI_ESPACE;
    const skei_ei_problem p{g,      batch, const_cast<float *>(x), y,    mc_idx, m_mc, angle_idx, m, copies, cos_sin,
                            lambda, loss,  grad,                   0.0f, nullptr, 0};
    EiJobs J;
    int rc = ei_problem_jobs(p, b, RayChoice{}, RayChoice{}, J);
    if (rc) return rc;

    const hipStream_t st = S(stream);
    const RayShape fwd_sh = merge_shapes(J.fwd_shape[0], J.fwd_shape[1]);
    if ((rc = staged(SKEI_STAGE_ROTATE, st, [&] { return rotate_run(inline_jobs(J.rot, 2), st); }))) return rc;
    // the MC job's items (full scan, the residual's precise sums) are the
    // longest: listed first, they start first and do not form the tail
    const RayJob fwd_jobs[2] = {J.fwd[1], J.fwd[0]};
    if ((rc = staged(SKEI_STAGE_FWD, st, [&] { return ray_run(kRayFwd, false, fwd_sh, inline_jobs(fwd_jobs, 2), st); })))
        return rc;
    if ((rc = staged(SKEI_STAGE_RAMP, st,
                     [&] { return ramp_run(false, ramp_block(g->n_det), ramp_shm(g->n_det), inline_jobs(J.ramp, 2), st); })))
        return rc;
    if ((rc = staged(SKEI_STAGE_BP_RESID, st,
                     [&] { return gather_run(kGatherBackproject, gather_groups_auto(m), inline_jobs(&J.bp, 1), st); })))
        return rc;
    // with a gradient, the loss is formed by one item of the RAMP_T launch
    // (same fixed order) and REDUCE launches nothing
    if ((rc = staged(SKEI_STAGE_REDUCE, st,
                     [&] { return grad ? SKEI_OK : reduce_run(inline_jobs(&J.red, 1), st); })))
        return rc;
    if (!grad) return SKEI_OK;
    const RampJob rampT[2] = {make_loss_job(J.red), J.rampT};   // the loss item starts first
    if ((rc = staged(SKEI_STAGE_BP_T, st,
                     [&] { return ray_run(kRayBpT, true, J.bpt_shape, inline_jobs(&J.bpt, 1), st); })))
        return rc;
    if ((rc = staged(SKEI_STAGE_RAMP_T, st,
                     [&] { return ramp_run(true, ramp_block(g->n_det), ramp_shm(g->n_det), inline_jobs(rampT, 2), st); })))
        return rc;
    if ((rc = staged(SKEI_STAGE_ADJ, st, [&] {
             const GatherJob adj_jobs[2] = {J.adj[1], J.adj[0]};   // the full-scan MC items first
             return gather_run(kGatherJosephAdj, gather_groups_auto(std::max(m, m_mc)), inline_jobs(adj_jobs, 2), st);
         })))
        return rc;
    return staged(SKEI_STAGE_ROTATE_ADJ, st, [&] { return rotate_adj_run(inline_jobs(&J.radj, 1), st); });
}

}  // namespace skei

extern "C" {

int skei_lds_read_bounds(int kernel, int size, long long *out)
{
    if (!out || size < 2) return SKEI_EINVAL;
    if (kernel == SKEI_LDS_RAMP) {
        if (size > 2048) return SKEI_ERANGE;
        ramp_lds_reads(size, out);
        return SKEI_OK;
    }
    if (kernel == SKEI_LDS_RAY) {
        if (size > 2032) return SKEI_ERANGE;
        ray_lds_reads(size, out);
        return SKEI_OK;
    }
    if (kernel == SKEI_LDS_GATHER) {
        if (size > 2032) return SKEI_ERANGE;
        gather_lds_reads(size, out);
        return SKEI_OK;
    }
    return SKEI_EINVAL;
}

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
    return launch_radon_fwd(g, x, nullptr, batch, angle_idx, m, y, nullptr, g->tune_fwd, S(stream));
}

int skei_radon_resid(const skei_geom *g, const float *x, const float *y_full, int batch, const int32_t *angle_idx,
                     int m, float *r, void *stream)
{
    int rc = check_geom_op(g, x, batch, angle_idx, m, r);
    if (rc) return rc;
    if (!y_full) return SKEI_EINVAL;
    return launch_radon_fwd(g, x, nullptr, batch, angle_idx, m, r, y_full, g->tune_fwd, S(stream));
}

int skei_sketch_rows(const float *G, int m, int n_rows, const float *y, int batch, int row_len, float *out,
                     void *stream)
{
    if (!G || !y || !out || m <= 0 || n_rows <= 0 || batch <= 0 || row_len <= 0) return SKEI_EINVAL;
    if (batch > 65535 || (long long)m * n_rows > 0x7fffffffLL) return SKEI_ERANGE;
    return launch_sketch_rows(G, m, n_rows, y, batch, row_len, false, out, S(stream));
}

int skei_sketch_rows_T(const float *G, int m, int n_rows, const float *r, int batch, int row_len, float *out,
                       void *stream)
{
    if (!G || !r || !out || m <= 0 || n_rows <= 0 || batch <= 0 || row_len <= 0) return SKEI_EINVAL;
    if (batch > 65535 || (long long)m * n_rows > 0x7fffffffLL) return SKEI_ERANGE;
    return launch_sketch_rows(G, m, n_rows, r, batch, row_len, true, out, S(stream));
}

int skei_radon_adj(const skei_geom *g, const float *y, int batch, const int32_t *angle_idx, int m, float *x,
                   void *stream)
{
    int rc = check_geom_op(g, y, batch, angle_idx, m, x);
    if (rc) return rc;
    return launch_gather(kGatherJosephAdj, g, y, batch, angle_idx, m, 1.0f, x, nullptr, nullptr, nullptr, S(stream));
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
    return launch_gather(kGatherBackproject, g, q, batch, angle_idx, m, 1.0f, x, nullptr, nullptr, nullptr, S(stream));
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
    return launch_gather(kGatherBackproject, g, q, batch, angle_idx, m, (float)(kPi / m), x, nullptr, nullptr, nullptr,
                         S(stream));
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
    rc = launch_rotate(x, batch, 1, g->n, nullptr, nullptr, xT, S(stream));
    if (rc) return rc;
    rc = launch_bp_T(g, x, xT, batch, angle_idx, m, nullptr, t, g->tune_bpt, S(stream));
    if (rc) return rc;
    return launch_ramp(g, nullptr, t, batch * m, (float)(kPi / m), y, S(stream));
}

int skei_rotate(const float *x, int batch, int copies, int n, const float *cos_sin, float *out, void *stream)
{
    if (!x || !cos_sin || !out || batch <= 0 || copies <= 0 || n < 2) return SKEI_EINVAL;
    if ((size_t)batch * copies > 65535 || n > 16384) return SKEI_ERANGE;
    return launch_rotate(x, batch, copies, n, cos_sin, out, nullptr, S(stream));
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
    return ei_workspace_bytes(g, batch, m_mc, m, copies);
}

int skei_ei_loss_grad(const skei_geom *g, const float *x, const float *y, int batch, const int32_t *mc_idx,
                      int m_mc, const int32_t *angle_idx, int m, int copies, const float *cos_sin, float lambda,
                      double *loss, float *grad, void *work, size_t work_bytes, void *stream)
{
    return ei_loss_grad_impl(g, x, y, batch, mc_idx, m_mc, angle_idx, m, copies, cos_sin, lambda, loss, grad, work,
                             work_bytes, stream);
}

size_t skei_ei_noalloc_scratch_bytes(void) { return kNoallocScratchBytes; }

int skei_ei_loss_grad_noalloc(const skei_geom *g, const float *x, const float *y, int batch, const int32_t *mc_idx,
                              int m_mc, const int32_t *angle_idx, int m, int copies, const float *cos_sin,
                              float lambda, double *loss, float *grad, void *stream)
{
    if (!g || batch <= 0 || m_mc <= 0 || m <= 0 || copies <= 0) return SKEI_EINVAL;
    if (ei_workspace_bytes(g, batch, m_mc, m, copies) > kNoallocScratchBytes) return SKEI_ESCRATCH;
    void *work = nullptr;
    int rc = noalloc_scratch(&work);
    if (rc) return rc;
    return ei_loss_grad_impl(g, x, y, batch, mc_idx, m_mc, angle_idx, m, copies, cos_sin, lambda, loss, grad, work,
                             kNoallocScratchBytes, stream);
}

}  // extern "C"

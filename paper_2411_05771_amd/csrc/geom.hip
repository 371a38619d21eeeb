// Geometry object: per-angle Joseph constants and Ram-Lak taps on the device.
//
// The angle grid is theta_a = a*pi/N_theta (Sec. 4.1.1: uniformly spaced
// angles).  Every constant is computed in double precision here and rounded
// once to float, so the kernels never accumulate angle or position error
// across steps: positions are always recomputed from indices with one FMA.
#include <cmath>
#include <cstdio>
#include <mutex>
#include <new>
#include <vector>

#include "skei_internal.h"
#include "work.h"

namespace skei {

int check_launch()
{
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SKEI_OK : SKEI_ELAUNCH;
}

int resident_workgroups(const void *kernel, int block, size_t shm)
{
    struct Entry {
        const void *k;
        int block, dev;
        size_t shm;
        int n;
    };
    static std::mutex mu;
    static std::vector<Entry> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    std::lock_guard<std::mutex> lock(mu);
    for (const Entry &e : cache)
        if (e.k == kernel && e.block == block && e.shm == shm && e.dev == dev) return e.n;
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, shm) != hipSuccess) return -1;
    const int n = cus * (per_cu < 1 ? 1 : per_cu);
    cache.push_back(Entry{kernel, block, dev, shm, n});
    return n;
}

}  // namespace skei

extern "C" {

const char *skei_version(void) { return "skei_ct 0.1 gfx950"; }

const char *skei_strerror(int code)
{
    switch (code) {
    case SKEI_OK: return "ok";
    case SKEI_EINVAL: return "invalid argument (null pointer, non-positive size or bad combination)";
    case SKEI_ENOMEM: return "device allocation failed";
    case SKEI_ELAUNCH: return "HIP launch or runtime call failed";
    case SKEI_ERANGE: return "size beyond the supported range";
    case SKEI_ESPACE: return "workspace smaller than required";
    case SKEI_ESCRATCH: return "workspace need exceeds the static scratch of the no-allocation entry point";
    default: return "unknown error";
    }
}

int skei_geom_create(int n, int n_angles, int n_det, skei_geom **out)
{
    if (!out) return SKEI_EINVAL;
    *out = nullptr;
    if (n < 2 || n_angles < 1 || n_det < 2) return SKEI_EINVAL;
    if (n > 2032 || n_angles > 65536 || n_det > 2048) return SKEI_ERANGE;

    const double pi = 3.14159265358979323846;
    const double cN = 0.5 * (n - 1), cD = 0.5 * (n_det - 1);
    std::vector<skei::AngleRow> tab(n_angles);
    for (int a = 0; a < n_angles; a++) {
        const double th = pi * (double)a / (double)n_angles;
        const double c = std::cos(th), s = std::sin(th);
        // Joseph steps along rows when |cos| >= |sin|; decided on the integer
        // index so that the 45/135-degree ties are machine independent.
        const bool rows = 4 * a <= n_angles || 4 * a >= 3 * n_angles;
        const double cm = rows ? c : s, cM = rows ? s : c;
        skei::AngleRow r{};
        const double base = -cD / cm + cN * (1.0 + cM / cm);
        const double two32 = 4294967296.0;
        r.base_fx = (int64_t)std::llround(base * two32);
        r.inv_fx = (int64_t)std::llround(two32 / cm);
        r.du_fx = (int64_t)std::llround(-cM / cm * two32);
        r.c_fx = (int64_t)std::llround(c * two32);
        r.s_fx = (int64_t)std::llround(s * two32);
        r.cd = c;
        r.sd = s;
        r.c = (float)c;
        r.s = (float)s;
        r.inv_m = (float)(1.0 / cm);
        r.du = (float)(-cM / cm);
        r.base = (float)base;
        r.scale = 1.0 / std::fabs(cm);
        r.w = (float)std::fabs(cm);
        r.inv_w2 = (float)(1.0 / (cm * cm));
        r.rows = rows ? 1 : 0;
        tab[a] = r;
    }
    // Ram-Lak taps at odd offsets, h(2e+1) = -1/(pi (2e+1))^2; h(0) = 1/4 and
    // the even taps are zero (Kak & Slaney ch. 3, unit detector spacing).
    // odd taps h(1), h(3), ... : every offset below N_det, rounded up to a
    // multiple of 16 taps (the filter kernel steps 4 groups of 4 taps)
    const int n_hodd = ((n_det / 2 + 1) + 15) / 16 * 16;
    std::vector<double> hodd(n_hodd);
    for (int e = 0; e < n_hodd; e++) {
        const double d = pi * (double)(2 * e + 1);
        hodd[e] = -1.0 / (d * d);
    }

    skei_geom *g = new (std::nothrow) skei_geom{};
    if (!g) return SKEI_ENOMEM;
    g->n = n;
    g->n_angles = n_angles;
    g->n_det = n_det;
    g->n_hodd = n_hodd;
    if (hipGetDevice(&g->device) != hipSuccess) {
        delete g;
        return SKEI_ELAUNCH;
    }
    if (hipMalloc((void **)&g->tab, sizeof(skei::AngleRow) * n_angles) != hipSuccess) {
        delete g;
        return SKEI_ENOMEM;
    }
    if (hipMalloc((void **)&g->hodd, sizeof(double) * n_hodd) != hipSuccess) {
        (void)hipFree(g->tab);
        delete g;
        return SKEI_ENOMEM;
    }
    if (hipMemcpy(g->tab, tab.data(), sizeof(skei::AngleRow) * n_angles, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g->hodd, hodd.data(), sizeof(double) * n_hodd, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(g->tab);
        (void)hipFree(g->hodd);
        delete g;
        return SKEI_ELAUNCH;
    }
    *out = g;
    return SKEI_OK;
}

int skei_geom_destroy(skei_geom *g)
{
    if (!g) return SKEI_EINVAL;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(g->device);
    (void)hipFree(g->tab);
    (void)hipFree(g->hodd);
    (void)hipSetDevice(cur);
    delete g;
    return SKEI_OK;
}

int skei_geom_set_tuning(skei_geom *g, int op, int group, int lines, int split)
{
    if (!g || group < 0 || group > 8 || lines < 0 || lines > 64 || split < 0 || split > 64) return SKEI_EINVAL;
    skei::RayTune t;
    t.group = group;
    t.lines = lines;
    t.split = split;
    if (op == SKEI_OP_FWD)
        g->tune_fwd = t;
    else if (op == SKEI_OP_BPT)
        g->tune_bpt = t;
    else
        return SKEI_EINVAL;
    return SKEI_OK;
}

int skei_geom_info(const skei_geom *g, int *n, int *n_angles, int *n_det)
{
    if (!g) return SKEI_EINVAL;
    if (n) *n = g->n;
    if (n_angles) *n_angles = g->n_angles;
    if (n_det) *n_det = g->n_det;
    return SKEI_OK;
}

}  // extern "C"

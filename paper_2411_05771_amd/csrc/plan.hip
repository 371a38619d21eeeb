// Batched EI plans (skei_ei_plan_*): the EI step of many problems of
// different sizes, one launch per stage for all of them, and the autotuner
// that picks each stage's dispatch mode and launch shape.
//
// Every problem's jobs come from ei_problem_jobs, exactly as for the
// one-problem entry point.  A stage's jobs are concatenated problem by
// problem into one work list; the list is cut into kXcds contiguous ranges of
// about equal estimated cost, one per XCD, so the items of one image stay on
// one L2.  Persistent dispatch launches one resident wave of workgroups that
// drain their XCD's range through an atomic cursor and then steal from the
// other ranges; static dispatch launches one workgroup per item.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "ei_step.h"
#include "skei_internal.h"

using namespace skei;

namespace {

constexpr int kStages = SKEI_STAGE_COUNT;

struct StageCfg {
    int dispatch = SKEI_DISPATCH_STATIC;
    int shape = 0;
};

struct StageTable {
    int njobs = 0;
    long long total = 0;
    long long grid_static = 0;
    size_t off_jobs = 0, off_first = 0, off_xr = 0;
    // launch parameters
    RayShape ray{0, 16, 0, 0};   // ray stages (merged over the problems)
    size_t shm = 0;           // ramp stages
    int ga = 0;        // gather stages
    int ramp_block = 0;
};

bool is_ray_stage(int s) { return s == SKEI_STAGE_FWD || s == SKEI_STAGE_BP_T; }

// Ray-stage shape codes (skei_ei_plan_configure): the wave count and chunk
// flags live in the ten-thousands digits as bits (1: three waves, 2: chunks
// of four units, 4: six waves, 8: eight waves); 0 waves = automatic.
int ray_code_waves(int shape)
{
    const int f = shape / 10000;
    return f & 1 ? 3 : f & 4 ? 6 : f & 8 ? 8 : shape > 0 ? 4 : 0;
}
bool ray_code_units4(int shape) { return (shape / 10000) & 2; }
bool ray_code_valid(int shape)
{
    const int rpt = shape % 100, lines = shape % 10000 / 100, f = shape / 10000;
    const int wave_bits = (f & 1) + ((f >> 2) & 1) + ((f >> 3) & 1);
    if (shape < 0 || f >= 16 || rpt > 4 || wave_bits > 1) return false;
    if ((f & 12) && rpt > 2) return false;   // six or eight waves: at most 2 rays per thread
    return lines == 0 || lines == 4 || lines == 8 || lines == 16;
}
int ray_code(const RayShape &r, int cfg_shape)
{
    return r.rpt + 100 * (cfg_shape % 10000 / 100) + (r.waves == 3 ? 10000 : 0) + (ray_code_units4(cfg_shape) ? 20000 : 0) +
           (r.waves == 6 ? 40000 : 0) + (r.waves == 8 ? 80000 : 0);
}
bool is_gather_stage(int s) { return s == SKEI_STAGE_BP_RESID || s == SKEI_STAGE_ADJ; }

// Host image of the device table: appends `bytes` at a 256-byte boundary.
size_t reserve(std::vector<char> &img, size_t bytes)
{
    const size_t off = align256(img.size());
    img.resize(off + bytes);
    return off;
}

template <typename Job>
void lay_out(const std::vector<Job> &jobs, StageTable &t, std::vector<char> &img)
{
    t.njobs = (int)jobs.size();
    std::vector<long long> first(jobs.size() + 1, 0);
    for (size_t i = 0; i < jobs.size(); i++) first[i + 1] = first[i] + jobs[i].items;
    t.total = first.back();
    std::vector<long long> xr(kXcds + 1);
    const long long widest = jobs.empty() ? 0 : xcd_ranges(jobs.data(), (int)jobs.size(), first.data(), xr.data());
    if (jobs.empty()) std::fill(xr.begin(), xr.end(), 0LL);
    t.grid_static = (long long)kXcds * widest;
    t.off_jobs = reserve(img, sizeof(Job) * std::max<size_t>(jobs.size(), 1));
    if (!jobs.empty()) std::memcpy(img.data() + t.off_jobs, jobs.data(), sizeof(Job) * jobs.size());
    t.off_first = reserve(img, sizeof(long long) * first.size());
    std::memcpy(img.data() + t.off_first, first.data(), sizeof(long long) * first.size());
    t.off_xr = reserve(img, sizeof(long long) * xr.size());
    std::memcpy(img.data() + t.off_xr, xr.data(), sizeof(long long) * xr.size());
}

// Stage-tuning cache: signature -> config.
struct TuneCache {
    std::mutex mu;
    std::unordered_map<std::string, StageCfg> map;
    std::vector<std::string> loaded_files;
};
TuneCache &tune_cache()
{
    static TuneCache c;
    return c;
}

}  // namespace

struct skei_ei_plan {
    int device = 0;
    std::vector<skei_ei_problem> probs;
    std::vector<EiBuffers> bufs;
    StageCfg cfg[kStages];
    StageTable tab[kStages];
    bool any_grad = false;
    char *dev = nullptr;
    size_t dev_bytes = 0;
    WorkQueue *queues = nullptr;   // two sets per stage, at the start of dev
    int parity[kStages] = {};      // the set the next launch of a stage uses
    bool tuning = false;           // while true the fused x -= step * grad is left out
};

// One angle per item fills a workgroup with up to 3 x 256 rays; below 256 rows
// (512 for B^T) a launch of such items leaves most CUs idle, and splitting
// each row over more workgroups wins (measured on MI355X, a 512^2 image with
// 16 copies, 726 detectors, per stage: forward / B^T at 5 angles 81.0 / 100.5
// -> 66.6 / 64.2 us with one ray per thread; at 20 angles the forward is best
// at two rays, 89.0 -> 80.9 us, and B^T at one, 107.8 -> 83.8 us; from 50
// angles up the three-ray default is best)
int skei::ray_rpt_default(int n_det, long long rows, bool transpose)
{
    const int def = n_det > 400 ? 3 : 2;
    if (rows < 256 || (transpose && rows < 512)) return 1;
    if (rows < 512) return std::min(def, 2);
    return def;
}

namespace {

int plan_build(skei_ei_plan *P)
{
    // default rays per thread: 2 fills a workgroup with one angle of up to
    // 512 detectors; wider detector rows pack better at 3; launches with few
    // (image, angle) rows take fewer (ray_rpt_default)
    int max_nd = 1;
    long long rows_f = 0, rows_b = 0;
    for (const skei_ei_problem &p : P->probs) {
        max_nd = std::max(max_nd, p.geom->n_det);
        rows_f += (long long)p.batch * p.copies * p.m + (long long)p.batch * p.m_mc;
        if (p.grad) rows_b += (long long)p.batch * p.copies * p.m;
    }
    // ray-stage shape code: rays per thread + 100 x march unit height, + 10000
    // for three-wave workgroups, + 20000 for LDS chunks of four units, + 40000
    // for six-wave and + 80000 for eight-wave workgroups (both run best with
    // the higher occupancy of 8-line chunks by default; the default wave
    // count is the first problem's automatic choice)
    auto choice = [&](int shape, int def_lines, int def_rpt) {
        RayChoice c;
        c.own = false;
        c.rpt = shape % 100 > 0 ? shape % 100 : def_rpt;
        c.lines = shape % 10000 > 0 ? shape % 10000 / 100 : def_lines;
        c.waves = ray_code_waves(shape);
        c.units = ray_code_units4(shape) ? 4 : 2;
        return c;
    };
    RayChoice fwd_c = choice(P->cfg[SKEI_STAGE_FWD].shape, 8, ray_rpt_default(max_nd, rows_f, false));
    RayChoice bpt_c = choice(P->cfg[SKEI_STAGE_BP_T].shape, 8, ray_rpt_default(max_nd, rows_b, true));
    std::vector<RotJob> rot;
    std::vector<RayJob> fwd, bpt;
    std::vector<RampJob> ramp, rampT, loss;
    std::vector<GatherJob> bp, adj;
    std::vector<RedJob> red;
    std::vector<RotAdjJob> radj;
    StageTable t[kStages];
    int max_m_bp = 1, max_m_adj = 1;
    for (size_t i = 0; i < P->probs.size(); i++) {
        const skei_ei_problem &p = P->probs[i];
        EiJobs J;
        int rc = ei_problem_jobs(p, P->bufs[i], fwd_c, bpt_c, J);
        if (rc) return rc;
        // an automatic wave count is fixed by the first problem for all
        if (fwd_c.waves == 0) fwd_c.waves = J.fwd_shape[0].waves;
        if (bpt_c.waves == 0 && J.grad) bpt_c.waves = J.bpt_shape.waves;
        rot.push_back(J.rot[0]);
        rot.push_back(J.rot[1]);
        fwd.push_back(J.fwd[1]);   // the full-scan MC job's long items first
        fwd.push_back(J.fwd[0]);
        for (int k = 0; k < 2; k++) {
            t[SKEI_STAGE_FWD].ray = merge_shapes(t[SKEI_STAGE_FWD].ray, J.fwd_shape[k]);
        }
        ramp.push_back(J.ramp[0]);
        ramp.push_back(J.ramp[1]);
        bp.push_back(J.bp);
        max_m_bp = std::max(max_m_bp, p.m);
        if (!J.grad) red.push_back(J.red);   // else the loss is an item of the RAMP_T launch
        if (J.grad) {
            bpt.push_back(J.bpt);
            t[SKEI_STAGE_BP_T].ray = merge_shapes(t[SKEI_STAGE_BP_T].ray, J.bpt_shape);
            rampT.push_back(J.rampT);
            loss.push_back(make_loss_job(J.red));
            adj.push_back(J.adj[1]);   // the full-scan MC job's long items first
            adj.push_back(J.adj[0]);
            max_m_adj = std::max(max_m_adj, std::max(p.m, p.m_mc));
            if (P->tuning) {   // timing runs must not move the caller's image
                J.radj.x_upd = nullptr;
                J.radj.step = 0.0f;
            }
            radj.push_back(J.radj);
        }
    }
    // ramp launch shape: rows of up to the widest detector, 256 threads
    for (int s : {SKEI_STAGE_RAMP, SKEI_STAGE_RAMP_T}) {
        t[s].ramp_block = ramp_block(max_nd);
        t[s].shm = ramp_shm(max_nd);
    }
    const int gbp = P->cfg[SKEI_STAGE_BP_RESID].shape, gadj = P->cfg[SKEI_STAGE_ADJ].shape;
    t[SKEI_STAGE_BP_RESID].ga = gbp > 0 ? gbp : gather_groups_auto(max_m_bp);
    t[SKEI_STAGE_ADJ].ga = gadj > 0 ? gadj : gather_groups_auto(max_m_adj);

    std::vector<char> img;
    reserve(img, sizeof(WorkQueue) * 2 * kStages);   // zero cursors
    lay_out(rot, t[SKEI_STAGE_ROTATE], img);
    lay_out(fwd, t[SKEI_STAGE_FWD], img);
    lay_out(ramp, t[SKEI_STAGE_RAMP], img);
    lay_out(bp, t[SKEI_STAGE_BP_RESID], img);
    lay_out(red, t[SKEI_STAGE_REDUCE], img);
    lay_out(bpt, t[SKEI_STAGE_BP_T], img);
    rampT.insert(rampT.begin(), loss.begin(), loss.end());   // the loss items start first
    lay_out(rampT, t[SKEI_STAGE_RAMP_T], img);
    lay_out(adj, t[SKEI_STAGE_ADJ], img);
    lay_out(radj, t[SKEI_STAGE_ROTATE_ADJ], img);

    // (re)upload: nothing of this plan may be in flight
    if (hipSetDevice(P->device) != hipSuccess) return SKEI_ELAUNCH;
    if (hipDeviceSynchronize() != hipSuccess) return SKEI_ELAUNCH;
    if (img.size() > P->dev_bytes) {
        if (P->dev) hipFree(P->dev);
        P->dev = nullptr;
        P->dev_bytes = 0;
        void *d = nullptr;
        if (hipMalloc(&d, img.size()) != hipSuccess) return SKEI_ENOMEM;
        P->dev = static_cast<char *>(d);
        P->dev_bytes = img.size();
    }
    if (hipMemcpy(P->dev, img.data(), img.size(), hipMemcpyHostToDevice) != hipSuccess) return SKEI_ELAUNCH;
    P->queues = reinterpret_cast<WorkQueue *>(P->dev);
    for (int s = 0; s < kStages; s++) {
        P->tab[s] = t[s];
        P->parity[s] = 0;
    }
    return SKEI_OK;
}

template <typename Job>
JobList<Job> table_list(const skei_ei_plan *P, int s)
{
    const StageTable &t = P->tab[s];
    JobList<Job> L{};
    L.njobs = t.njobs;
    L.jobs = reinterpret_cast<const Job *>(P->dev + t.off_jobs);
    L.first = reinterpret_cast<const long long *>(P->dev + t.off_first);
    L.xr = reinterpret_cast<const long long *>(P->dev + t.off_xr);
    const bool pers = P->cfg[s].dispatch == SKEI_DISPATCH_PERSISTENT;
    L.wq = pers ? P->queues + 2 * s + P->parity[s] : nullptr;
    L.wq_next = pers ? P->queues + 2 * s + (1 - P->parity[s]) : nullptr;
    L.total = t.total;
    L.grid_static = t.grid_static;
    return L;
}

int launch_stage(const skei_ei_plan *P, int s, hipStream_t st)
{
    const StageTable &t = P->tab[s];
    switch (s) {
    case SKEI_STAGE_ROTATE: return rotate_run(table_list<RotJob>(P, s), st);
    case SKEI_STAGE_FWD: return ray_run(kRayFwd, false, t.ray, table_list<RayJob>(P, s), st);
    case SKEI_STAGE_RAMP: return ramp_run(false, t.ramp_block, t.shm, table_list<RampJob>(P, s), st);
    case SKEI_STAGE_BP_RESID: return gather_run(kGatherBackproject, t.ga, table_list<GatherJob>(P, s), st);
    case SKEI_STAGE_REDUCE: return reduce_run(table_list<RedJob>(P, s), st);
    case SKEI_STAGE_BP_T: return ray_run(kRayBpT, true, t.ray, table_list<RayJob>(P, s), st);
    case SKEI_STAGE_RAMP_T: return ramp_run(true, t.ramp_block, t.shm, table_list<RampJob>(P, s), st);
    case SKEI_STAGE_ADJ: return gather_run(kGatherJosephAdj, t.ga, table_list<GatherJob>(P, s), st);
    case SKEI_STAGE_ROTATE_ADJ: return rotate_adj_run(table_list<RotAdjJob>(P, s), st);
    default: return SKEI_EINVAL;
    }
}

int run_stage(skei_ei_plan *P, int s, hipStream_t st)
{
    if (P->tab[s].total <= 0) return SKEI_OK;
    const int rc = launch_stage(P, s, st);
    if (rc == SKEI_OK && P->cfg[s].dispatch == SKEI_DISPATCH_PERSISTENT) P->parity[s] ^= 1;
    return rc;
}

int check_problem(const skei_ei_problem &p)
{
    if (!p.geom || !p.x || !p.y || !p.mc_idx || !p.angle_idx || !p.cos_sin || !p.loss) return SKEI_EINVAL;
    if (p.batch <= 0 || p.m_mc <= 0 || p.m <= 0 || p.copies <= 0) return SKEI_EINVAL;
    if ((size_t)p.batch * p.copies > 65535) return SKEI_ERANGE;
    if (p.step != 0.0f && !p.grad) return SKEI_EINVAL;
    return SKEI_OK;
}

// Signature of a stage's work: the sizes of every problem, not its pointers.
std::string stage_signature(const skei_ei_plan *P, int s)
{
    std::string sig = "s" + std::to_string(s);
    unsigned long long h = 1469598103934665603ULL;
    auto mix = [&](long long v) {
        for (int i = 0; i < 8; i++) {
            h ^= (unsigned long long)((v >> (8 * i)) & 0xff);
            h *= 1099511628211ULL;
        }
    };
    for (const skei_ei_problem &p : P->probs) {
        mix(p.geom->n);
        mix(p.geom->n_angles);
        mix(p.geom->n_det);
        mix(p.batch);
        mix(p.m_mc);
        mix(p.m);
        mix(p.copies);
        mix(p.grad != nullptr);
    }
    char buf[32];
    std::snprintf(buf, sizeof buf, ":%016llx", h);
    return sig + buf;
}

void cache_load(const char *path)
{
    TuneCache &c = tune_cache();
    std::lock_guard<std::mutex> lock(c.mu);
    for (const std::string &f : c.loaded_files)
        if (f == path) return;
    c.loaded_files.push_back(path);
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char key[128];
    int d, sh;
    while (std::fscanf(f, "%127s %d %d", key, &d, &sh) == 3) c.map[key] = StageCfg{d, sh};
    std::fclose(f);
}

void cache_store(const char *path, const std::string &key, const StageCfg &cfg)
{
    TuneCache &c = tune_cache();
    std::lock_guard<std::mutex> lock(c.mu);
    c.map[key] = cfg;
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d\n", key.c_str(), cfg.dispatch, cfg.shape);
    std::fclose(f);
}

bool cache_find(const std::string &key, StageCfg &cfg)
{
    TuneCache &c = tune_cache();
    std::lock_guard<std::mutex> lock(c.mu);
    auto it = c.map.find(key);
    if (it == c.map.end()) return false;
    cfg = it->second;
    return true;
}

}  // namespace

extern "C" {

size_t skei_ei_problem_workspace_bytes(const skei_ei_problem *p)
{
    if (!p || check_problem(*p)) return 0;
    return align256(ei_workspace_bytes(p->geom, p->batch, p->m_mc, p->m, p->copies));
}

size_t skei_ei_plan_workspace_bytes(const skei_ei_problem *problems, int count)
{
    if (!problems || count <= 0) return 0;
    size_t total = 0;
    for (int i = 0; i < count; i++) {
        const skei_ei_problem &p = problems[i];
        if (check_problem(p)) return 0;
        if (!p.work) total += skei_ei_problem_workspace_bytes(&p);
    }
    return total;
}

int skei_ei_plan_create(const skei_ei_problem *problems, int count, void *work, size_t work_bytes,
                        skei_ei_plan **out)
{
    if (!problems || count <= 0 || !out) return SKEI_EINVAL;
    *out = nullptr;
    for (int i = 0; i < count; i++) {
        int rc = check_problem(problems[i]);
        if (rc) return rc;
    }
    const size_t need = skei_ei_plan_workspace_bytes(problems, count);
    if (need > 0 && (!work || work_bytes < need)) return work ? SKEI_ESPACE : SKEI_EINVAL;
    skei_ei_plan *P = new (std::nothrow) skei_ei_plan;
    if (!P) return SKEI_ENOMEM;
    // default: static dispatch (measured ahead of persistent on every stage of
    // the EI and uneven workloads; the autotuner still tries both)
    for (int s = 0; s < kStages; s++) P->cfg[s].dispatch = SKEI_DISPATCH_STATIC;
    if (hipGetDevice(&P->device) != hipSuccess) {
        delete P;
        return SKEI_ELAUNCH;
    }
    char *w = static_cast<char *>(work);
    for (int i = 0; i < count; i++) {
        const skei_ei_problem &p = problems[i];
        const size_t b = skei_ei_problem_workspace_bytes(&p);
        EiBuffers eb;
        const bool own = p.work != nullptr;
        if ((own && p.work_bytes < b) ||
            !ei_carve(p.geom, p.batch, p.m_mc, p.m, p.copies, own ? p.work : w, own ? p.work_bytes : b, eb)) {
            delete P;
            return SKEI_ESPACE;
        }
        if (!own) w += b;
        P->probs.push_back(p);
        P->bufs.push_back(eb);
        P->any_grad |= p.grad != nullptr;
    }
    int rc = plan_build(P);
    if (rc) {
        skei_ei_plan_destroy(P);
        return rc;
    }
    *out = P;
    return SKEI_OK;
}

int skei_ei_plan_destroy(skei_ei_plan *plan)
{
    if (!plan) return SKEI_EINVAL;
    if (plan->dev) {
        int cur = 0;
        hipGetDevice(&cur);
        hipSetDevice(plan->device);
        hipDeviceSynchronize();
        hipFree(plan->dev);
        hipSetDevice(cur);
    }
    delete plan;
    return SKEI_OK;
}

int skei_ei_plan_run(skei_ei_plan *plan, void *stream)
{
    if (!plan) return SKEI_EINVAL;
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    for (int s = 0; s < kStages; s++) {
        if (s > SKEI_STAGE_REDUCE && !plan->any_grad) break;
        int rc = staged(s, st, [&] { return run_stage(plan, s, st); });
        if (rc) return rc;
    }
    return SKEI_OK;
}

int skei_ei_plan_configure(skei_ei_plan *plan, int stage, int dispatch, int shape)
{
    if (!plan || stage < 0 || stage >= kStages) return SKEI_EINVAL;
    if (dispatch != SKEI_DISPATCH_PERSISTENT && dispatch != SKEI_DISPATCH_STATIC) return SKEI_EINVAL;
    if (is_ray_stage(stage) && !ray_code_valid(shape)) return SKEI_EINVAL;
    if (is_gather_stage(stage) && !(shape == 0 || shape == 1 || shape == 2 || shape == 4 || shape == 14 ||
                                     shape == 24 || shape == 44))
        return SKEI_EINVAL;
    if (!is_ray_stage(stage) && !is_gather_stage(stage)) shape = 0;
    const bool rebuild = plan->cfg[stage].shape != shape;
    const StageCfg old = plan->cfg[stage];
    plan->cfg[stage] = StageCfg{dispatch, shape};
    if (rebuild) {
        int rc = plan_build(plan);
        if (rc) {
            plan->cfg[stage] = old;
            plan_build(plan);
            return rc;
        }
    }
    return SKEI_OK;
}

int skei_ei_plan_get_config(const skei_ei_plan *plan, int stage, int *dispatch, int *shape)
{
    if (!plan || stage < 0 || stage >= kStages) return SKEI_EINVAL;
    if (dispatch) *dispatch = plan->cfg[stage].dispatch;
    if (shape) {
        const StageTable &t = plan->tab[stage];
        *shape = is_ray_stage(stage) ? ray_code(t.ray, plan->cfg[stage].shape) : is_gather_stage(stage) ? t.ga : 0;
    }
    return SKEI_OK;
}

int skei_ei_plan_autotune(skei_ei_plan *plan, void *stream, int reps, const char *cache_path)
{
    if (!plan || reps <= 0) return SKEI_EINVAL;
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (cache_path) cache_load(cache_path);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return SKEI_ELAUNCH;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return SKEI_ELAUNCH;
    }
    // Every candidate is timed on real intermediate values: one whole run
    // first fills the plan's buffers.  The fused gradient step is left out of
    // that run and of every timed launch, so x is unchanged by tuning.
    plan->tuning = true;
    int rc = plan_build(plan);
    for (int s = 0; s < kStages && rc == SKEI_OK; s++) {
        if (s > SKEI_STAGE_REDUCE && !plan->any_grad) break;
        rc = run_stage(plan, s, st);
    }
    for (int s = 0; s < kStages && rc == SKEI_OK; s++) {
        if (plan->tab[s].total <= 0) continue;
        const std::string key = stage_signature(plan, s);
        StageCfg best;
        if (cache_find(key, best)) {
            rc = skei_ei_plan_configure(plan, s, best.dispatch, best.shape);
            continue;
        }
        std::vector<int> shapes{0};
        if (is_ray_stage(s))
            shapes = {1,     2,     3,     4,     802,   803,   402,   403,   10002, 10802, 10003, 10004,
                      10803, 30402, 30802, 20402, 20403, 40401, 40801, 40802, 80401, 80801};
        if (is_gather_stage(s)) shapes = {1, 2, 4, 14, 24, 44};
        float best_ms = 3.0e38f;
        best = plan->cfg[s];
        for (int d : {SKEI_DISPATCH_PERSISTENT, SKEI_DISPATCH_STATIC}) {
            for (int sh : shapes) {
                if ((rc = skei_ei_plan_configure(plan, s, d, sh))) {
                    if (rc != SKEI_ERANGE) break;
                    rc = SKEI_OK;   // a shape the problems do not fit (e.g. too many rays per thread): skip it
                    continue;
                }
                if ((rc = run_stage(plan, s, st))) break;   // warm-up
                std::vector<float> ms;
                for (int r = 0; r < reps && rc == SKEI_OK; r++) {
                    if (hipEventRecord(e0, st) != hipSuccess) rc = SKEI_ELAUNCH;
                    if (!rc) rc = run_stage(plan, s, st);
                    if (!rc && hipEventRecord(e1, st) != hipSuccess) rc = SKEI_ELAUNCH;
                    if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = SKEI_ELAUNCH;
                    float t = 0.0f;
                    if (!rc && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = SKEI_ELAUNCH;
                    ms.push_back(t);
                }
                if (rc) break;
                std::sort(ms.begin(), ms.end());
                const float med = ms[ms.size() / 2];
                if (med < best_ms) {
                    best_ms = med;
                    best = StageCfg{d, sh};
                }
            }
            if (rc) break;
        }
        if (rc) break;
        rc = skei_ei_plan_configure(plan, s, best.dispatch, best.shape);
        if (!rc) cache_store(cache_path, key, best);
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    plan->tuning = false;
    const int rb = plan_build(plan);   // the chosen shapes, with the gradient step restored
    return rc ? rc : rb;
}

}  // extern "C"

// The EI loss/gradient step as per-stage job lists, shared by the one-problem
// entry point (skei_ei_loss_grad) and batched plans (skei_ei_plan_*): both
// build every problem's jobs with ei_problem_jobs, so a problem computes the
// same thing, bitwise, alone or batched.
#pragma once

#include "skei_internal.h"

namespace skei {

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Device buffers of one problem's step, carved from a workspace.
struct EiBuffers {
    float *z, *zT, *r, *rT, *xT;   // [B*C][N][N] x4, [B][N][N]
    double *ysd;                   // [B*C][m][N_det] doubles (its first half doubles as float ys)
    float *ys, *qs;                // [B*C][m][N_det]
    float *rmc;                    // [B][m_mc][N_det]
    float *amc;                    // [B][N][N]
    double *pmc, *pei;             // partial sums of squares
    size_t n_pmc, n_pei;           // their capacities
};

size_t ei_workspace_bytes(const skei_geom *g, int batch, int m_mc, int m, int copies);
// false when `bytes` is too small.
bool ei_carve(const skei_geom *g, int batch, int m_mc, int m, int copies, void *work, size_t bytes, EiBuffers &b);

// All jobs of one problem's step.  Two-job stages (ROTATE, FWD, RAMP, ADJ)
// hold the sketch/copies job first and the MC / plain-image job second.
struct EiJobs {
    RotJob rot[2];
    RayJob fwd[2];
    RayShape fwd_shape[2];
    RampJob ramp[2];   // H ys, and the row sums of squares of r_MC
    GatherJob bp;
    RedJob red;
    RayJob bpt;
    RayShape bpt_shape;
    RampJob rampT;
    GatherJob adj[2];
    RotAdjJob radj;
    bool grad;
};

// Launch shape of a ray stage's jobs: rays-per-thread cap (0 = per-problem
// automatic shape), march unit height (0 = the built-in choice), waves per
// workgroup and units per LDS chunk.  `own` = use the geometry's tuning (skei_geom_set_tuning) instead.
struct RayChoice {
    int rpt = 0, lines = 0, waves = 4, units = 2;
    bool own = true;
};
int ei_problem_jobs(const skei_ei_problem &p, const EiBuffers &b, const RayChoice &fwd, const RayChoice &bpt,
                    EiJobs &J);

// Default rays-per-thread cap of an EI ray launch over `rows` (image, listed
// angle) pairs: 3 for rows wider than 400 detectors, else 2; fewer when the
// launch has too few rows to fill the chip (transpose: the B^T stage).
int ray_rpt_default(int n_det, long long rows, bool transpose);

// Stage probe (skei_probe_set): events around the launch of one stage.
int probe_begin(int stage, hipStream_t st);
int probe_end(int stage, hipStream_t st);

template <typename F>
int staged(int stage, hipStream_t st, F &&fn)
{
    int rc = probe_begin(stage, st);
    if (rc) return rc;
    rc = fn();
    if (rc) return rc;
    return probe_end(stage, st);
}

}  // namespace skei

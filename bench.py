"""Benchmark: sketched EI loss forward+backward step on one MI355X.

Workload (the EI operator step): one 256 x 256 float32 ellipse phantom, 360
angles in [0, pi), 363 unit detectors, y = A x_true + N(0, (0.01 max)^2),
x = FBP(y) as the image under evaluation, 16 copies rotated by seeded
phi ~ U[0, 2 pi), a seeded random quarter sketch (m = 90), lambda = 1.  One
step is skei_ei_loss_grad: T, A_S, H, B_S (+ residual/loss), A (MC residual),
reduction, then B_S^T, H, A_S^T, A^T, T^T for the gradient.

value = projector rays per step / step time, in GRays/s: a step evaluates
the full-scan A and the sketched A_S on every copy once forward and once
adjoint, i.e. 2 * (N_theta + C*m) * N_det rays.

Prints ONE JSON line.  --gpus N > 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import math
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "sketched fwd+adj GRays/s and EI-loss fwd+bwd step ms at 1e-5 rel err; p50/p99 job latency"

# MI355X published peaks used for the roofline fraction.
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3          # published fp32 vector peak (packed issue)
PEAK_FP32_NONPACKED_TFLOPS = 78.6  # 256 CU x 64 lanes x 2 flop x 2.4 GHz (packed fp32 is disabled in this build)

WORKLOADS = {
    "ei256": dict(n=256, n_angles=360, n_det=363, copies=16, m=90, batch=1, lam=1.0),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="ei256", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    return ap.parse_args()


def algorithmic_flops(stage, w, widths):
    """Algorithmic floating-point work of one launch of `stage` (2 flops per
    tap / multiply-add), from the per-unit counts of each operator."""
    n, nd, c, m, b = w["n"], w["n_det"], w["copies"], w["m"], w["batch"]
    na = w["n_angles"]
    bc = b * c
    if stage == "fwd":                 # Joseph: 2 taps per major-axis line per ray (A_S on copies + A_mc)
        return 2.0 * (2 * n) * (bc * m + b * na) * nd
    if stage == "adj":                 # 2 taps per (pixel, angle): A_S^T on copies + A_mc^T
        return 2.0 * 2 * n * n * (bc * m + b * na)
    if stage == "bp_resid":
        return 2.0 * 2 * n * n * bc * m
    if stage == "bp_T":                # 2/w pixels within unit distance per line, per ray
        return 2.0 * n * nd * bc * float(np.sum(2.0 / widths))
    if stage in ("ramp", "ramp_T"):    # symmetric form: one multiply-add per odd offset pair + centre
        return 2.0 * bc * m * nd * (nd + 1) / 2
    if stage in ("rotate", "rotate_adj"):
        return 2.0 * 4 * n * n * bc
    return 0.0


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sharded design is in DESIGN.md",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2411_05771_amd import capi, ei, ops, synth

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    w = WORKLOADS[args.workload]
    n, na, nd, c, m, b, lam = w["n"], w["n_angles"], w["n_det"], w["copies"], w["m"], w["batch"], w["lam"]
    dev = torch.device("cuda", 0)

    # ---------------------------------------------------------- inputs (seeded, resident in HBM)
    geom = ops.Geometry(n, na, nd)
    xt = torch.from_numpy(synth.phantom_batch(n, b)).to(dev)
    y_clean = ops.radon_fwd_(geom, xt, geom.full())
    z = torch.from_numpy(synth.std_noise(tuple(y_clean.shape))).to(dev, torch.float32)
    y = (y_clean + 0.01 * y_clean.max() * z).contiguous()
    x0 = ops.fbp_(geom, y, geom.full()).contiguous()
    idx = synth.random_sketch(na, m)
    cs_host = synth.cos_sin(synth.rotation_angles(c))
    cs = torch.from_numpy(cs_host.astype(np.float32)).to(dev)
    step = ei.EIStep(geom, y, geom.sketch(idx), cs, lam)
    grad = torch.empty_like(x0)
    widths = np.maximum(np.abs(np.cos(math.pi * idx / na)), np.abs(np.sin(math.pi * idx / na)))

    for _ in range(args.warmup):
        step(x0, grad)
    torch.cuda.synchronize()

    # ---------------------------------------------------------- per-stage durations (untimed pass)
    stream = torch.cuda.current_stream()
    stage_ms = {}
    for s, name in enumerate(capi.STAGES):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
        for e0, e1 in evs:
            e0.record(stream)
            e1.record(stream)
        for e0, e1 in evs:
            capi.call("skei_probe_set", s, e0._as_parameter_, e1._as_parameter_)
            step(x0, grad)
        torch.cuda.synchronize()
        stage_ms[name] = statistics.median(e0.elapsed_time(e1) for e0, e1 in evs)
    capi.call("skei_probe_set", -1, None, None)
    dominant = max(stage_ms, key=stage_ms.get)
    dom_id = capi.STAGES.index(dominant)

    # ---------------------------------------------------------- timed region
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for e0, e1 in evs:
        e0.record(stream)
        e1.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in evs:
        capi.call("skei_probe_set", dom_id, e0._as_parameter_, e1._as_parameter_)
        step(x0, grad)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    capi.call("skei_probe_set", -1, None, None)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    dom_ms = statistics.mean(e0.elapsed_time(e1) for e0, e1 in evs)

    rays_per_step = 2.0 * (na + c * m) * nd * b
    value = rays_per_step / (ms_per_step * 1e-3) / 1e9
    flops = algorithmic_flops(dominant, w, widths)
    achieved = flops / (dom_ms * 1e-3) / 1e12
    roofline = {
        "bound": "alu", "kernel": dominant, "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
        "frac_nonpacked": round(achieved / PEAK_FP32_NONPACKED_TFLOPS, 4),
        "launch_ms": round(dom_ms, 5), "traffic": traffic_for(dominant),
    }

    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "GRays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic ellipse phantoms (stand-in for CT100)",
        "config": {"workload": f"ei_step_{n}sq_{na}ang_{nd}det_{c}copies_m{m}", "n": n, "n_angles": na,
                   "n_det": nd, "copies": c, "sketch_m": m, "batch": b, "lambda": lam,
                   "rays_per_step": int(rays_per_step)},
        "ei_step_ms": round(ms_per_step, 5),
        "stage_ms": {k: round(v, 5) for k, v in stage_ms.items()},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(x0, y, idx, cs, lam, na, rays_per_step, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def traffic_for(kernel):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries, if they
    were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        ent = rec.get(kernel)
        if not ent or ent.get("source_sha") != source_sha():
            return None
        return ent.get("bytes_per_launch")
    except Exception:
        return None


def source_sha():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2411_05771_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def cpu_baseline(x0, y, idx, cs, lam, na, rays_per_step, target_s):
    """The FP64 oracle (as it stands) on the same inputs: whole EI steps,
    repeated until about `target_s` seconds of work."""
    import oracle
    xh = x0.detach().cpu().numpy().astype(np.float64)
    yh = y.detach().cpu().numpy().astype(np.float64)
    csh = cs.detach().cpu().numpy().astype(np.float64)
    reps, t_total = 0, 0.0
    while t_total < target_s and reps < 10:
        t0 = time.perf_counter()
        oracle.ei_loss_grad(xh, yh, na, idx, csh, lam)
        t_total += time.perf_counter() - t0
        reps += 1
    per_step = t_total / reps
    return {"value": round(rays_per_step / per_step / 1e9, 6), "unit": "GRays/s", "cores": oracle.num_threads(),
            "kind": "oracle", "sample": f"{reps} full EI steps of the same workload (float64, OpenMP)",
            "s_per_step": round(per_step, 4)}


if __name__ == "__main__":
    main()

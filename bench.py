"""Benchmark: sketched EI loss forward+backward step on one MI355X.

Headline workload (the EI operator step): one 256 x 256 float32 ellipse
phantom, 360 angles in [0, pi), 363 unit detectors, y = A x_true +
N(0, (0.01 max)^2), x = FBP(y) as the image under evaluation, 16 copies
rotated by seeded phi ~ U[0, 2 pi), a seeded random quarter sketch (m = 90),
lambda = 1.  One step is one run of an autotuned one-problem EI plan
(skei_ei_plan_run): T (and x^T), A_S on the copies with the MC residual
y - A x, H, r = z - (pi/m) B_S H A_S z, the loss, then B_S^T, H, A_S^T with
A^T r_MC, and T^T for the gradient -- nine launches.

value = projector rays per step / step time, in GRays/s: a step evaluates
the full-scan A and the sketched A_S on every copy once forward and once
adjoint, i.e. 2 * (N_theta + C*m) * N_det rays.

Extra legs (same JSON line): "plain_ops" -- the 64 x 64 plain operators;
"batched" -- 64 uneven problems in one plan vs one call per problem;
"serving" -- Poisson-arriving adaptation jobs under an HBM budget at a sweep
of arrival rates, continuous batching vs per-call, p50/p99 latency and
GRays/s; "cpu_baseline" and "parity" -- the FP64 oracle timed on the host
and compared with the device on oracle-made inputs.

Prints ONE JSON line.  --gpus N > 1 is refused: the path runs on one GPU.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import math
import os
import re
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
PEAK_FP32_NONPACKED_TFLOPS = 78.6  # 256 CU x 64 lanes x 2 flop x 2.4 GHz (the kernels are built with packed fp32 off)

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
    ap.add_argument("--no-batched", action="store_true", help="skip the uneven 64-problem leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-ttt", action="store_true", help="skip the test-time-training leg")
    ap.add_argument("--no-mri", action="store_true", help="skip the multicoil MRI leg")
    ap.add_argument("--headline-only", action="store_true",
                    help="time the headline EI step only (no further legs), e.g. under a profiler")
    ap.add_argument("--legs", default=None,
                    help="comma list of the further legs to run (plain_ops, paper_shaped, dense_sketch, ttt, mri, "
                         "batched, serving); default: all, minus the --no-* ones")
    ap.add_argument("--serve-jobs", type=int, default=12)
    ap.add_argument("--serve-rates", default="1,2,3,4,8", help="Poisson arrival rates swept, jobs per second")
    ap.add_argument("--serve-jobs-small", type=int, default=24)
    ap.add_argument("--serve-rates-small", default="10,20,40,80,160",
                    help="arrival rates of the small-job sweep, jobs per second")
    ap.add_argument("--budget-gb", type=float, default=1.0, help="HBM budget of the serving leg")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file (text); default: a scratch copy of the package's MI355X defaults")
    ap.add_argument("--tune-reps", type=int, default=5, help="timed launches per autotuner candidate")
    return ap.parse_args()


def algorithmic_flops(stage, w, widths, widths_mc):
    """Algorithmic floating-point work of one launch of `stage`: 2 flops per
    nonzero matrix entry applied (one multiply-add), counted from the
    operators' closed-form entries, never from what a kernel marches.

    - Joseph A (and A^T): entry (a, k), p is Lambda((s_k - s_p)/w_a)/w_a, so a
      pixel has on average 2 w_a nonzero detectors per angle: 2 w_a N^2
      entries per listed angle.
    - Pixel-driven B (and B^T): entry Lambda(s_p + c_D - k) has on average 2
      nonzero detectors per (pixel, angle): 2 N^2 entries per listed angle.
    - Ram-Lak H (symmetric form): h(0) and the odd offsets, (N_det + 1)/2
      multiply-adds per output sample.
    - Rotation T: 4 bilinear taps per output pixel.
    `widths` holds w_a of the sketch's angles, `widths_mc` those of the MC angles."""
    n, nd, c, m, b = w["n"], w["n_det"], w["copies"], w["m"], w["batch"]
    bc = b * c
    nn = float(n) * n
    if stage in ("fwd", "adj"):        # A_S on the copies + A_mc on the image (A^T: the same entries)
        return 2.0 * 2.0 * nn * (bc * float(np.sum(widths)) + b * float(np.sum(widths_mc)))
    if stage in ("bp_resid", "bp_T"):  # B_S or B_S^T on the copies
        return 2.0 * 2.0 * nn * bc * m
    if stage in ("ramp", "ramp_T"):
        return 2.0 * bc * m * nd * (nd + 1) / 2
    if stage in ("rotate", "rotate_adj"):
        return 2.0 * 4 * nn * bc
    return 0.0


def ei_inputs(geom, w, dev):
    """Seeded EI inputs made on the device: phantom, y = A x + 1 % noise, x0 = FBP(y)."""
    import torch

    from paper_2411_05771_amd import ops, synth
    xt = torch.from_numpy(synth.phantom_batch(w["n"], w["batch"])).to(dev)
    y_clean = ops.radon_fwd_(geom, xt, geom.full())
    z = torch.from_numpy(synth.std_noise(tuple(y_clean.shape))).to(dev, torch.float32)
    y = (y_clean + 0.01 * y_clean.max() * z).contiguous()
    x0 = ops.fbp_(geom, y, geom.full()).contiguous()
    return x0, y


def probe_stages(run, reps=5):
    """Median duration (ms) of every stage of `run` (HIP events around each launch)."""
    import torch

    from paper_2411_05771_amd import capi
    stream = torch.cuda.current_stream()
    out = {}
    for s, name in enumerate(capi.STAGES):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in evs:
            e0.record(stream)
            e1.record(stream)
        for e0, e1 in evs:
            capi.call("skei_probe_set", s, e0._as_parameter_, e1._as_parameter_)
            run()
        torch.cuda.synchronize()
        out[name] = statistics.median(e0.elapsed_time(e1) for e0, e1 in evs)
    capi.call("skei_probe_set", -1, None, None)
    return out


def timed_steps(run, steps, probe_stage):
    """Times exactly `steps` calls of `run` (host clock, synchronised on both
    sides) while HIP events bracket stage `probe_stage` of every step."""
    import torch

    from paper_2411_05771_amd import capi
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for e0, e1 in evs:
        e0.record(stream)
        e1.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in evs:
        capi.call("skei_probe_set", probe_stage, e0._as_parameter_, e1._as_parameter_)
        run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    capi.call("skei_probe_set", -1, None, None)
    return (t1 - t0) * 1e3 / steps, statistics.mean(e0.elapsed_time(e1) for e0, e1 in evs)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the multi-GPU sharding of the path "
              "is a design, not built", file=sys.stderr)
        sys.exit(2)
    if args.tune_cache is None:
        # the package's MI355X tuning of these workloads (autotuner output, 15
        # timed launches per candidate), copied so that new entries stay local
        import shutil
        import tempfile
        args.tune_cache = os.path.join(tempfile.mkdtemp(prefix="skei_tune_"), "tune.txt")
        shutil.copyfile(os.path.join(ROOT, "paper_2411_05771_amd", "tuned", "mi355x.txt"), args.tune_cache)
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
    x0, y = ei_inputs(geom, w, dev)
    idx = synth.random_sketch(na, m)
    cs = torch.from_numpy(synth.cos_sin(synth.rotation_angles(c)).astype(np.float32)).to(dev)
    sketch = geom.sketch(idx)
    widths = np.maximum(np.abs(np.cos(math.pi * idx / na)), np.abs(np.sin(math.pi * idx / na)))
    all_a = np.arange(na)
    widths_mc = np.maximum(np.abs(np.cos(math.pi * all_a / na)), np.abs(np.sin(math.pi * all_a / na)))

    # the product path: a one-problem EI plan, autotuned (cached per shape)
    plan = ei.EIPlan([ei.EIProblem(geom, x0, y, sketch, cs, lam)])
    tuned = plan.autotune(reps=args.tune_reps, cache_path=args.tune_cache)
    # the one-call entry point, for reference
    single = ei.EIStep(geom, y, sketch, cs, lam)
    grad = torch.empty_like(x0)

    for _ in range(args.warmup):
        plan.run()
        single(x0, grad)
    torch.cuda.synchronize()
    stage_ms = probe_stages(plan.run)
    dominant = max(stage_ms, key=stage_ms.get)
    dom_id = capi.STAGES.index(dominant)

    # ---------------------------------------------------------- timed region
    ms_per_step, dom_ms = timed_steps(plan.run, args.steps, dom_id)
    single_ms, _ = timed_steps(lambda: single(x0, grad), max(5, args.steps // 2), -1)

    rays_per_step = 2.0 * (na + c * m) * nd * b
    value = rays_per_step / (ms_per_step * 1e-3) / 1e9
    flops = algorithmic_flops(dominant, w, widths, widths_mc)
    achieved = flops / (dom_ms * 1e-3) / 1e12
    traffic, l2_hit = traffic_for(dominant, tuned[dominant][1])
    roofline = {
        "bound": "alu", "kernel": dominant, "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
        "frac_nonpacked": round(achieved / PEAK_FP32_NONPACKED_TFLOPS, 4),
        "launch_ms": round(dom_ms, 5), "flops_per_launch": flops, "traffic": traffic, "l2_hit_rate": l2_hit,
    }
    fwd_adj_ms = stage_ms["fwd"] + stage_ms["adj"]
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "GRays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic ellipse phantoms (stand-in for CT100)",
        "config": {"workload": f"ei_step_{n}sq_{na}ang_{nd}det_{c}copies_m{m}", "n": n, "n_angles": na,
                   "n_det": nd, "copies": c, "sketch_m": m, "batch": b, "lambda": lam,
                   "rays_per_step": int(rays_per_step)},
        "ei_step_ms": round(ms_per_step, 5),
        "ei_step_ms_single_call": round(single_ms, 5),
        "sketched_fwd_adj_grays": round(rays_per_step / (fwd_adj_ms * 1e-3) / 1e9, 4),
        "stage_ms": {k: round(v, 5) for k, v in stage_ms.items()},
        "tuned": {k: list(v) for k, v in tuned.items()},
        "roofline": roofline,
        # informational, not a roofline: the bytes the stage would move if every
        # tap were an HBM read (4 B per nonzero entry) over the launch time; it
        # exceeds 1 whenever the on-chip caches serve the taps
        "gather_equiv_hbm_rate_informational": round(
            gather_equiv_bytes(dominant, w, widths, widths_mc) / (dom_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
    }
    plan.close()
    if not args.headline_only:
        legs = {"plain_ops": True, "paper_shaped": True, "dense_sketch": True, "ttt": not args.no_ttt,
                "mri": not args.no_mri, "batched": not args.no_batched, "serving": not args.no_serving}
        if args.legs is not None:
            chosen = {v.strip() for v in args.legs.split(",") if v.strip()}
            unknown = chosen - set(legs)
            if unknown:
                print(f"unknown legs: {sorted(unknown)}", file=sys.stderr)
                sys.exit(2)
            legs = {k: k in chosen for k in legs}
        if legs["plain_ops"]:
            out["plain_ops"] = plain_ops_leg()
        if legs["paper_shaped"]:
            out["paper_shaped"] = paper_shaped_leg()
        if legs["dense_sketch"]:
            out["dense_sketch"] = dense_sketch_leg()
        if legs["ttt"]:
            out["ttt"] = ttt_leg()
        if legs["mri"]:
            out["mri"] = mri_leg()
        if legs["batched"]:
            out["batched"] = batched_leg(args)
        if legs["serving"]:
            out["serving"] = serving_leg(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["parity"] = cpu_baseline(w, idx, args.cpu_seconds, rays_per_step)
    print(json.dumps(out), flush=True)


def gather_equiv_bytes(stage, w, widths, widths_mc):
    """4 bytes per nonzero entry applied: the bytes the stage would move if
    every tap came from HBM (outputs are negligible beside them)."""
    return 2.0 * algorithmic_flops(stage, w, widths, widths_mc)   # 2 flops per entry -> 4 B per entry


def plain_ops_leg():
    """The plain-operator workload: one 64 x 64 ellipse phantom, 60 angles,
    91 detectors, batch 1; radon_fwd, radon_adj and Ram-Lak fbp with the
    full scan and with every 4th angle (m = 15).  Each call is timed with
    HIP events over 200 back-to-back launches (launch-latency bound at this
    size); GRays/s = m N_det / (t_fwd + t_adj).  A parity sample compares
    every output with the FP64 oracle on the same float inputs."""
    import torch

    import oracle
    from paper_2411_05771_amd import capi, ops, synth
    n, na, nd = 64, 60, 91
    dev = torch.device("cuda", 0)
    geom = ops.Geometry(n, na, nd)
    xh = synth.ellipse_phantom(n, synth.SEED_PHANTOM).astype(np.float64)
    x = torch.from_numpy(xh.astype(np.float32)).to(dev)[None].contiguous()
    stream = torch.cuda.current_stream()
    out = {"workload": "plain_ops_64sq_60ang_91det_batch1"}

    def time_us(fn, reps=200):
        for _ in range(10):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / reps

    def rel(got, want):
        return float(np.max(np.abs(got.cpu().numpy().astype(np.float64) - want)) / np.max(np.abs(want)))

    for name, idx in (("full", np.arange(na, dtype=np.int32)), ("every4", synth.interleaved_sketch(na, 4, 0))):
        sk = geom.sketch(idx)
        m = idx.size
        y = ops.radon_fwd_(geom, x, sk)
        xa = ops.radon_adj_(geom, y, sk)
        xf = ops.fbp_(geom, y, sk)
        yb, xab, xfb = torch.empty_like(y), torch.empty_like(xa), torch.empty_like(xf)
        t_f = time_us(lambda: ops.radon_fwd_(geom, x, sk, out=yb))
        t_a = time_us(lambda: ops.radon_adj_(geom, y, sk, out=xab))
        work = torch.empty(max(1, int(capi.query("skei_fbp_workspace_bytes", geom.handle, 1, m))),
                           dtype=torch.uint8, device=dev)
        t_fbp = time_us(lambda: ops.fbp_(geom, y, sk, out=xfb, work=work))
        yh = y.cpu().numpy().astype(np.float64)
        par = {"radon_fwd": rel(y, oracle.radon_fwd(xh[None], na, nd, idx)),
               "radon_adj": rel(xa, oracle.radon_adj(yh, n, na, idx)),
               "fbp": rel(xf, oracle.fbp(yh, n, na, idx))}
        out[name] = {"m": int(m), "fwd_us": round(t_f, 3), "adj_us": round(t_a, 3), "fbp_us": round(t_fbp, 3),
                     "fwd_adj_grays": round(m * nd / ((t_f + t_a) * 1e-6) / 1e9, 4),
                     "parity_relerr": {k: float(f"{v:.3e}") for k, v in par.items()}}
    return out


def paper_shaped_leg():
    """The paper's CT geometry (Sec. 4.1.1 and 4.2.1): a 512 x 512 ellipse
    phantom, 100 uniformly spaced angles, 726 detectors, interleaved sketches
    S_k = {k, k+N, k+2N, ...} with N in {1, 2, 5, 10, 20} (all, 50, 20, 10
    and 5 % of the angles).  Per N: the sketched operators' times (HIP events
    over 50 back-to-back calls), the one-call EI step with 16 rotated copies
    and the sketched MC term S y - A_S x of Algorithm 2, and the Theorem 1
    series with the network taken as the identity:
        full   = mean_c ||v_c - fbp(A v_c)||,
        sketch = mean_c mean_k ||v_c - fbp_{S_k}(A_{S_k} v_c)||  (k = 0..N-1),
    v_c = T_c fbp(y) for 4 seeded rotations; the theorem places `sketch`
    within r delta of `full` (r = max ||v_c||) with a delta the paper does not
    give, so the series is informational (the tests check its values against
    the oracle)."""
    import torch

    from paper_2411_05771_amd import ei, ops, synth
    n, na, nd = 512, 100, 726
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    geom = ops.Geometry(n, na, nd)
    w = dict(n=n, batch=1)
    x0, y = ei_inputs(geom, w, dev)
    cs = torch.from_numpy(synth.cos_sin(synth.rotation_angles(16)).astype(np.float32)).to(dev)
    v = ops.rotate_(x0, torch.from_numpy(synth.cos_sin(synth.rotation_angles(4, synth.SEED_ROTATION + 1))
                                         .astype(np.float32)).to(dev)).reshape(4, n, n).contiguous()

    def time_us(fn, reps=50):
        for _ in range(5):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / reps

    def resid(sk):
        r = v - ops.fbp_(geom, ops.radon_fwd_(geom, v, sk), sk)
        return torch.linalg.vector_norm(r.double().reshape(4, -1), dim=1)

    full = resid(geom.full())
    vnorm = torch.linalg.vector_norm(v.double().reshape(4, -1), dim=1)
    out = {"workload": "paper_ct_512sq_100ang_726det", "splits": []}
    for split in (1, 2, 5, 10, 20):
        sk = geom.sketch(synth.interleaved_sketch(na, split, 0))
        xb = torch.empty_like(x0)
        yb = torch.empty((1, sk.m, nd), device=dev)
        work = torch.empty(max(1, int(ops.capi.query("skei_fbp_workspace_bytes", geom.handle, 1, sk.m))),
                           dtype=torch.uint8, device=dev)
        ys = ops.radon_fwd_(geom, x0, sk)
        t_f = time_us(lambda: ops.radon_fwd_(geom, x0, sk, out=yb))
        t_a = time_us(lambda: ops.radon_adj_(geom, ys, sk, out=xb))
        t_fbp = time_us(lambda: ops.fbp_(geom, ys, sk, out=xb, work=work))
        step = ei.EIStep(geom, y, sk, cs, 1.0, mc=sk)
        grad = torch.empty_like(x0)
        t_ei = time_us(lambda: step(x0, grad), reps=20)
        sk_res = torch.stack([resid(geom.sketch(synth.interleaved_sketch(na, split, k))) for k in range(split)])
        out["splits"].append({
            "N": split, "m": sk.m, "fraction": round(sk.m / na, 3), "fwd_us": round(t_f, 2), "adj_us": round(t_a, 2),
            "fbp_us": round(t_fbp, 2), "ei_step_us": round(t_ei, 2),
            "theorem1_full": round(float(full.mean()), 6), "theorem1_sketch": round(float(sk_res.mean()), 6),
            "theorem1_gap_over_r": round(float((sk_res.mean() - full.mean()) / vnorm.max()), 6)})
    base = out["splits"][0]
    for e in out["splits"]:
        e["ei_step_speedup_vs_full"] = round(base["ei_step_us"] / e["ei_step_us"], 3)
    out["paper_ttt_speedup_context"] = {"hardware": "RTX 4060 Ti, whole TTT epoch incl. U-Net",
                                        "fraction_0.5": 3.59, "fraction_0.2": 7.13, "fraction_0.1": 7.65,
                                        "fraction_0.05": 8.10}
    return out


def ttt_leg():
    """Sketched equivariant test-time training (Algorithm 2) on the paper's CT
    geometry (512 x 512, 100 angles, 726 detectors): a residual BN U-Net
    (widths 32-256, seeded random weights: the pretrained CT100 model is not
    available), Adam at 5e-4, one interleaved sketch S_k and one whole-degree
    rotation per iteration.  Wall time per iteration (device-synchronised,
    10 iterations after 3 warm-up) for every split N and for adapting all
    parameters ("full") or only the BatchNorm affine ones ("bn"); and the CT
    operators' share: the same loss and backward with the network taken as
    the identity."""
    import copy

    import torch

    from paper_2411_05771_amd import ops, synth, ttt
    n, na, nd = 512, 100, 726
    dev = torch.device("cuda", 0)
    geom = ops.Geometry(n, na, nd)
    _, y = ei_inputs(geom, dict(n=n, batch=1), dev)
    torch.manual_seed(0)
    base = ttt.ResUNet(width=32, depth=4).to(dev)
    out = {"workload": "skei_ttt_512sq_100ang_726det_resunet32", **ttt.network_size(base), "modes": {}}

    class _Identity(torch.nn.Module):
        def forward(self, v):
            return v

    # the CT operators of one iteration alone: the loss and its backward with
    # the network taken as the identity (the part the library computes)
    x_in = ops.fbp_(geom, y, geom.full()).contiguous()
    rot = ttt.rotation_table(dev)
    ops_rows = []
    for split in (1, 2, 5, 10, 20):
        sk = geom.sketch(synth.interleaved_sketch(na, split, 0))
        x = x_in.clone().requires_grad_(True)

        def one():
            x.grad = None
            loss, _, _ = ttt.skei_ttt_loss(_Identity(), x, y, geom, sk, rot[36:37])
            loss.backward()
        for _ in range(3):
            one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            one()
        torch.cuda.synchronize()
        ops_rows.append({"N": split, "ms_per_iteration": round((time.perf_counter() - t0) / 20 * 1e3, 3)})
    out["operators_only"] = ops_rows
    for mode in ("full", "bn"):
        rows = []
        for split in (1, 2, 5, 10, 20):
            loop = ttt.SkEITTT(copy.deepcopy(base), geom, y, splits=split, mode=mode)
            ms = 1e3 * ttt.time_per_iteration(loop, 10, warmup=3)
            rows.append({"N": split, "fraction": round(1.0 / split, 3), "ms_per_iteration": round(ms, 3),
                         "last_loss": float(loop.losses[-1])})
        for r in rows:
            r["speedup_vs_full"] = round(rows[0]["ms_per_iteration"] / r["ms_per_iteration"], 3)
        out["modes"][mode] = rows
    out["paper_context"] = {"hardware": "RTX 4060 Ti", "time_per_epoch_s_full_ei": 9.56,
                            "time_per_epoch_s_skei_50_20_10_5pct": [2.66, 1.34, 1.25, 1.18],
                            "bn_only_full_ei": 5.45, "bn_only_skei_50_20_10_5pct": [1.46, 1.09, 1.00, 0.95]}
    return out


def mri_leg():
    """Multicoil MRI with coil sketches (Sec. 3.4, Algorithm 3) at the paper's
    setup: 128 x 128 images, 15 coils, 4x Cartesian undersampling (8 % of
    the rows around the zero frequency kept), synthetic maps, phantom and
    0.5 % noise.  Per-call time of A and A^H, and the wall time of one
    sketched EI iteration (loss, backward, Adam step; one whole-degree
    rotation per iteration), device-synchronised, for the full operator, the
    classical sketch (a random subset of Mc coils drawn every iteration, its
    operator and data formed by the library's coil selection) and the coil
    sketch (covariance, PCA to L = 15 virtual coils, R = ceil(Mc / 2) kept,
    Rademacher mixing of the rest; one fixed sketch, set-up timed apart),
    Mc in {10, 5, 2}; with the network taken as the identity (the
    operators' part) -- eagerly and as one HIP graph replayed per iteration --
    and with the residual BN U-Net (2 channels,
    widths 32-256) as F, adapted in full."""
    import torch

    from paper_2411_05771_amd import mri, synth, ttt
    dev = torch.device("cuda", 0)
    n, nc = 128, 15
    prob = mri.MRIProblem(n=n, nc=nc, accel=4, noise=0.005, device=dev)
    op, y = prob.op, prob.y
    rot = ttt.rotation_table(dev)
    g = synth.rng(synth.SEED_MRI + 50)

    def t_us(fn, reps=100):
        for _ in range(5):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return round(e0.elapsed_time(e1) * 1e3 / reps, 2)

    out = {"workload": "mri_128sq_15coils_4x", "operator_us": {
        "A": t_us(lambda: op.fwd_(prob.x0)), "A_H": t_us(lambda: op.adj_(y)), "A_pinv": t_us(lambda: op.pinv_(y))}}

    def sketch_for(kind, mc):
        if kind == "full":
            return lambda: (op, y)
        if kind == "classical":
            return lambda: mri.classical_sketch(op, y, g.choice(nc, size=mc, replace=False))
        op_s, y_s, _ = mri.coil_sketch(op, y, nc, (mc + 1) // 2, mc)
        return lambda: (op_s, y_s)

    def run(kind, mc, net):
        get = sketch_for(kind, mc)
        if net is None:
            x = prob.x0.clone().requires_grad_(True)
            opt = torch.optim.Adam([x], lr=5e-4)
        else:
            x = None
            opt = torch.optim.Adam(net.parameters(), lr=5e-4)

        def step():
            o, ys = get()
            i = int(g.integers(360))
            opt.zero_grad(set_to_none=True)
            if net is None:
                loss, _, _ = mri.mri_ei_loss(x, ys, o, rot[i:i + 1])
            else:
                loss, _, _ = mri.mri_skei_ttt_loss(net, prob.x0, ys, o, rot[i:i + 1])
            loss.backward()
            opt.step()
        return round(1e3 * mri.time_per_iteration(step, iters=30, warmup=5), 3)

    cases = [("full", nc)] + [(k, mc) for k in ("classical", "coil") for mc in (10, 5, 2)]
    setup = {}
    for mc in (10, 5, 2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mri.coil_sketch(op, y, nc, (mc + 1) // 2, mc)
        torch.cuda.synchronize()
        setup[f"coil_Mc{mc}"] = round((time.perf_counter() - t0) * 1e3, 3)
    out["coil_sketch_setup_ms"] = setup
    out["identity_ms_per_iteration"] = {f"{k}_Mc{mc}": run(k, mc, None) for k, mc in cases}

    # the same iteration (network = identity) captured once in a HIP graph and
    # replayed, for the fixed operators (the full one and the coil sketches)
    def run_graph(kind, mc):
        if kind == "classical":
            gs = mri.MRIGraphStep(prob.x0, y, op, select=mc)
            step = lambda: gs.step(rot[int(g.integers(360))].unsqueeze(0),  # noqa: E731
                                   g.choice(nc, size=mc, replace=False))
        else:
            o, ys = sketch_for(kind, mc)()
            gs = mri.MRIGraphStep(prob.x0, ys, o)
            step = lambda: gs.step(rot[int(g.integers(360))].unsqueeze(0))  # noqa: E731
        return round(1e3 * mri.time_per_iteration(step, iters=50, warmup=5), 4)
    out["identity_graph_ms_per_iteration"] = {f"{k}_Mc{mc}": run_graph(k, mc) for k, mc in cases}
    torch.manual_seed(0)
    base = ttt.ResUNet(width=32, depth=4, channels=2).to(dev)
    import copy
    out["unet_ms_per_iteration"] = {f"{k}_Mc{mc}": run(k, mc, copy.deepcopy(base)) for k, mc in cases}
    out["paper_context"] = {"hardware": "RTX 4060 Ti", "s_per_iteration_full_ei": 0.157,
                            "c_skei_10_5_2": [0.151, 0.134, 0.130], "skei_10_5_2": [0.141, 0.129, 0.127]}
    return out


def dense_sketch_leg():
    """Dense measurement-space sketches S = G (x) I (Gaussian G, Sec. 2.3) on
    the matrix cores: skei_sketch_rows / _T timed with HIP events over 100
    calls at the EI-step shape (90 x 360 mixes of 363-detector rows, 16
    images) and at a 1024^2 / 1440-angle job's shape (180 x 1440, 1449
    detectors, 16 images), against the FP32 matrix peak (157.3 TFLOP/s) and
    the 8 TB/s HBM peak; and the MC residual of one 256^2 image with a dense
    sketch, S (y - A x) (every angle projected, then mixed), against the
    angle-subsampled S y - A_S x of the same size m."""
    import torch

    from paper_2411_05771_amd import ops, synth
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()

    def time_us(fn, reps=100):
        for _ in range(5):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / reps

    out = {"gemm": []}
    for m, k, L, b in ((90, 360, 363, 16), (180, 1440, 1449, 16)):
        G = torch.from_numpy(synth.dense_sketch_matrix(m, k, "gaussian", 1).astype(np.float32)).to(dev)
        y = torch.rand((b, k, L), device=dev)
        r = torch.rand((b, m, L), device=dev)
        sy = torch.empty((b, m, L), device=dev)
        st = torch.empty((b, k, L), device=dev)
        t_s = time_us(lambda: ops.capi.call("skei_sketch_rows", ops._ptr(G), m, k, ops._ptr(y), b, L, ops._ptr(sy),
                                            ops._stream()))
        t_t = time_us(lambda: ops.capi.call("skei_sketch_rows_T", ops._ptr(G), m, k, ops._ptr(r), b, L, ops._ptr(st),
                                            ops._stream()))
        flops = 2.0 * m * k * L * b
        nbytes = 4.0 * (m * k + (k + m) * L * b)
        out["gemm"].append({"m": m, "n_rows": k, "row_len": L, "batch": b, "flops": flops, "bytes": nbytes,
                            "S_us": round(t_s, 2), "ST_us": round(t_t, 2),
                            "S_tflops": round(flops / (t_s * 1e-6) / 1e12, 2),
                            "S_frac_mfma_fp32": round(flops / (t_s * 1e-6) / 1e12 / PEAK_FP32_TFLOPS, 4),
                            "S_frac_hbm": round(nbytes / (t_s * 1e-6) / 1e9 / PEAK_HBM_GBS, 4)})
    n, na, nd, m = 256, 360, 363, 90
    geom = ops.Geometry(n, na, nd)
    x0, y = ei_inputs(geom, dict(n=n, batch=1), dev)
    ds = ops.DenseSketch(geom, synth.dense_sketch_matrix(m, na, "gaussian", 2))
    sub = geom.sketch(synth.random_sketch(na, m))
    rb = torch.empty((1, na, nd), device=dev)
    sb = torch.empty((1, m, nd), device=dev)
    t_dense = time_us(lambda: ops.sketch_rows_(ds, ops.radon_resid_(geom, x0, y, geom.full(), out=rb), out=sb))
    t_sub = time_us(lambda: ops.radon_resid_(geom, x0, y, sub, out=sb))
    out["mc_residual_256sq_m90"] = {"dense_us": round(t_dense, 2), "subsampled_us": round(t_sub, 2)}
    return out


def batched_leg(args):
    """The uneven batched workload: 64 problems (N in {128, 256, 512},
    N_theta ~ U{90..720}, N_det = ceil(sqrt 2 N) + 1, ratio in {2, 4, 8},
    8 copies), one autotuned plan vs one fused call per problem."""
    import torch

    from paper_2411_05771_amd import ei, ops, synth
    dev = torch.device("cuda", 0)
    specs = synth.uneven_problems()
    probs = []
    for p in specs:
        g = ops.Geometry(p["n"], p["n_angles"], p["n_det"])
        w = dict(n=p["n"], batch=1)
        x0, y = ei_inputs(g, w, dev)
        sk = g.sketch(synth.random_sketch(p["n_angles"], p["m"], p["sketch_seed"]))
        cs = torch.from_numpy(synth.cos_sin(synth.rotation_angles(p["copies"], p["rotation_seed"]))
                              .astype(np.float32)).to(dev)
        probs.append(ei.EIProblem(g, x0, y, sk, cs, 1.0))
    steps = [ei.EIStep(pr.geom, pr.y, pr.sk, pr.cs, 1.0) for pr in probs]

    def percall():
        for s_, pr in zip(steps, probs):
            s_(pr.x, pr.grad)
    plan = ei.EIPlan(probs)
    plan.autotune(reps=max(3, args.tune_reps // 2), cache_path=args.tune_cache)
    reps = 5
    for _ in range(2):
        plan.run()
        percall()
    plan_ms, _ = timed_steps(plan.run, reps, -1)
    call_ms, _ = timed_steps(percall, reps, -1)
    stages = probe_stages(plan.run, reps=3)
    rays = sum(2.0 * (p["n_angles"] + p["copies"] * p["m"]) * p["n_det"] for p in specs)
    # a ray marches N image lines, so rays of the 512^2 problems cost twice those
    # of 256^2: ray-lines per second compare workloads of different sizes
    ray_lines = sum(2.0 * (p["n_angles"] + p["copies"] * p["m"]) * p["n_det"] * p["n"] for p in specs)
    plan.close()
    return {"workload": "uneven_64_problems_8copies", "problems": len(specs), "plan_ms": round(plan_ms, 4),
            "per_problem_calls_ms": round(call_ms, 4), "speedup": round(call_ms / plan_ms, 3),
            "plan_grays": round(rays / (plan_ms * 1e-3) / 1e9, 4),
            "plan_g_ray_lines_per_s": round(ray_lines / (plan_ms * 1e-3) / 1e9, 1),
            "plan_stage_ms": {k: round(v, 3) for k, v in stages.items()},
            "launches_per_step": {"plan": 8, "per_problem": 8 * len(specs)}}


def serving_sweep(specs_at, rates, budget, executors, label):
    """Runs the same seeded jobs at each arrival rate with each executor."""
    from paper_2411_05771_amd import serve
    specs0 = specs_at(rates[0])
    rays = sum(serve.job_rays(s) for s in specs0)
    out = {"rays_per_point": rays, "points": []}
    host_y = None
    for rate in rates:
        specs = specs_at(rate)
        point = {"rate": rate}
        for name, kw in executors:
            ex = serve.GpuExecutor(**kw)
            if host_y is None:
                ex.prepare(specs)
                host_y = dict(ex.host_y)
            else:
                ex.host_y.update(host_y)
            rep = serve.Server(ex, budget).run(specs)
            builds = ex.plan_builds
            ex.close()
            point[name] = {"p50_s": round(rep.percentile(50), 4), "p99_s": round(rep.percentile(99), 4),
                           "makespan_s": round(rep.makespan, 3), "grays": round(rays / rep.makespan / 1e9, 4),
                           "done": len(rep.done), "rejected": len(rep.rejected), "steps": rep.iterations,
                           "max_batch": max(rep.batch_sizes) if rep.batch_sizes else 0,
                           "peak_gb": round(rep.peak_bytes / (1 << 30), 3), "plan_builds": builds}
            print(f"[serving {label}] rate {rate} {name}: {point[name]}", file=sys.stderr, flush=True)
        out["points"].append(point)
    return out


def serving_leg(args):
    """Poisson-arriving test-time adaptation jobs (16 copies, 50 iterations
    each) under an HBM budget, at a sweep of arrival rates (the same seeded
    jobs, arrival gaps scaled by the rate): continuous batching vs per-call
    launches.
      mixed: N in {256, 512, 1024}, N_theta ~ U{180..1440}, ratio in {2, 4, 8};
      small: N = 256, N_theta ~ U{180..360}, ratio in {2, 4, 8}.
    Executors: "per_call" (one plan per job, one iteration of every job per
    step), "batched" (jobs of one geometry size and repetition count share a
    plan; cheap jobs take up to 1/4 of the costliest job's iteration per
    step) and "batched_share1" (every cost class about the same device time
    per step)."""
    from paper_2411_05771_amd import synth
    budget = int(args.budget_gb * (1 << 30))
    executors = (("per_call", dict(batched=False)), ("batched", dict(batched=True)),
                 ("batched_share1", dict(batched=True, share=1.0)))
    res = {"budget_gb": args.budget_gb, "executors": [e[0] for e in executors]}
    rates = [float(r) for r in args.serve_rates.split(",")]
    res["mixed"] = dict(workload=f"poisson_{args.serve_jobs}_jobs_256_to_1024sq_180_to_1440ang_50_iters",
                        jobs=args.serve_jobs, rates_jobs_per_s=rates,
                        **serving_sweep(lambda r: synth.poisson_jobs(args.serve_jobs, rate=r), rates, budget,
                                        executors, "mixed"))
    rates_s = [float(r) for r in args.serve_rates_small.split(",")]
    small = lambda r: synth.poisson_jobs(args.serve_jobs_small, rate=r, sizes=(256,), angles=(180, 360))
    res["small"] = dict(workload=f"poisson_{args.serve_jobs_small}_jobs_256sq_180_to_360ang_50_iters",
                        jobs=args.serve_jobs_small, rates_jobs_per_s=rates_s,
                        **serving_sweep(small, rates_s, budget, executors, "small"))
    return res


def traffic_for(stage, shape):
    """HBM bytes per launch and L2 hit rate of a stage's kernel, from the
    committed rocprofv3 --pmc summary, if it was taken on the current kernel
    source and the same tuned launch shape; else (None, None)."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None, None
    try:
        rec = json.load(open(path))
        ent = rec.get(stage)
        if not ent or rec.get("source_sha") != source_sha() or ent.get("shape") != shape:
            return None, None
        return ent.get("bytes_per_launch"), ent.get("l2_hit")
    except Exception:
        return None, None


# The sources the ray kernels (the forward and B^T stages whose traffic the
# counters measured) are built from: their kernels, the job and angle-table
# layouts and the angle table's construction.
RAY_KERNEL_SOURCES = ("k_project.hip", "skei_internal.h", "work.h", "geom.hip")


_TOKENS = re.compile(r'"(?:\\.|[^"\\\n])*"|//[^\n]*|/\*.*?\*/', re.S)


def code_text(src: str) -> str:
    """The source with its comments dropped and whitespace runs folded to one
    space (string literals are kept whole), so that a comment edit leaves the
    fingerprint of the code unchanged."""
    code = _TOKENS.sub(lambda m: m.group(0) if m.group(0).startswith('"') else " ", src)
    return re.sub(r"\s+", " ", code).strip()


def source_sha():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2411_05771_amd", "csrc")
    for f in RAY_KERNEL_SOURCES:
        with open(os.path.join(csrc, f)) as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, idx, target_s, rays_per_step):
    """The FP64 oracle (as it stands) timed on whole EI steps of the workload,
    repeated until about `target_s` seconds of work; its inputs are made by
    the oracle itself (phantom, y = A x + 1 % noise, x0 = FBP(y)), and the
    same step on the device is checked against it (the parity sample)."""
    import torch

    import oracle
    from paper_2411_05771_amd import ei, ops, synth
    n, na, nd, c, lam = w["n"], w["n_angles"], w["n_det"], w["copies"], w["lam"]
    xt = synth.phantom_batch(n, w["batch"]).astype(np.float64)
    yc = oracle.radon_fwd(xt, na, nd)
    y = synth.add_relative_noise(yc, synth.std_noise(yc.shape)).astype(np.float32).astype(np.float64)
    x0 = oracle.fbp(y, n, na).astype(np.float32).astype(np.float64)
    cs = synth.cos_sin(synth.rotation_angles(c)).astype(np.float32).astype(np.float64)
    reps, t_total = 0, 0.0
    while t_total < target_s and reps < 10:
        t0 = time.perf_counter()
        want_l, want_g = oracle.ei_loss_grad(x0, y, na, idx, cs, lam)
        t_total += time.perf_counter() - t0
        reps += 1
    per_step = t_total / reps
    base = {"value": round(rays_per_step / per_step / 1e9, 6), "unit": "GRays/s", "cores": oracle.num_threads(),
            "kind": "oracle", "sample": f"{reps} full EI steps of the same workload (float64, OpenMP)",
            "s_per_step": round(per_step, 4), "cpu_model": cpu_model(), "host_cpus_visible": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0))}
    dev = torch.device("cuda", 0)
    geom = ops.Geometry(n, na, nd)
    step = ei.EIStep(geom, torch.from_numpy(y.astype(np.float32)).to(dev), geom.sketch(idx),
                     torch.from_numpy(cs.astype(np.float32)).to(dev), lam)
    loss, grad = step(torch.from_numpy(x0.astype(np.float32)).to(dev))
    g = grad.cpu().numpy().astype(np.float64).reshape(want_g.shape)
    parity = {"loss_relerr": float(abs(loss.item() - want_l) / abs(want_l)),
              "grad_relerr": float(np.max(np.abs(g - want_g)) / np.max(np.abs(want_g)))}
    return base, parity


if __name__ == "__main__":
    main()

"""Batched EI plans (skei_ei_plan_*): many problems of different sizes in one
launch per stage.

Each problem of a plan must give bitwise the loss and gradient of the
one-problem fused step (skei_ei_loss_grad) on the same inputs, whatever the
dispatch mode (persistent queues or one workgroup per item), the launch
shapes (rays per thread, angle groups per pixel) or the autotuner's choice;
and it must match the FP64 oracle to a relative max-norm error of 1e-5 in
both the loss and the gradient.

Inputs: seeded ellipse phantoms, y = A x_true + 1 % noise, x = FBP(y), a
seeded random sketch of N_theta / ratio angles and seeded rotations per
problem.  The uneven workload draws N from {128, 256, 512}, N_theta from
U{90..720}, N_det = ceil(sqrt(2) N) + 1, ratio from {2, 4, 8}, 8 copies.
"""
import numpy as np
import pytest
import torch

from gpu_util import f32, host, relerr, to_dev
from paper_2411_05771_amd import synth

pytestmark = pytest.mark.gpu


def gpu_problem(skei, ei, p, grad=True, batch=1):
    """Problem inputs made on the device (for plan-vs-single comparisons)."""
    geom = skei.Geometry(p["n"], p["n_angles"], p["n_det"])
    xt = to_dev(np.stack([synth.ellipse_phantom(p["n"], p["phantom_seed"] + i) for i in range(batch)]))
    y = skei.radon_fwd_(geom, xt, geom.full())
    y = (y + 0.01 * y.max() * to_dev(synth.std_noise(tuple(y.shape), p["noise_seed"]))).contiguous()
    x0 = skei.fbp_(geom, y, geom.full()).contiguous()
    idx = synth.random_sketch(p["n_angles"], p["m"], p["sketch_seed"])
    cs = to_dev(synth.cos_sin(synth.rotation_angles(p["copies"], p["rotation_seed"])))
    return ei.EIProblem(geom, x0, y, geom.sketch(idx), cs, 1.0, grad=grad)


def oracle_problem(skei, ei, orc, p):
    """Problem inputs made by the oracle (for oracle comparisons)."""
    if p.get("image") == "uniform":     # too small for the ellipses to cover a pixel centre
        xt = synth.uniform((1, p["n"], p["n"]), p["phantom_seed"])
    else:
        xt = synth.ellipse_phantom(p["n"], p["phantom_seed"]).astype(np.float64)[None]
    yc = orc.radon_fwd(xt, p["n_angles"], p["n_det"])
    y = f32(synth.add_relative_noise(yc, synth.std_noise(yc.shape, p["noise_seed"])))
    x0 = f32(orc.fbp(y, p["n"], p["n_angles"]))
    idx = synth.random_sketch(p["n_angles"], p["m"], p["sketch_seed"])
    cs = f32(synth.cos_sin(synth.rotation_angles(p["copies"], p["rotation_seed"])))
    geom = skei.Geometry(p["n"], p["n_angles"], p["n_det"])
    pr = ei.EIProblem(geom, to_dev(x0), to_dev(y), geom.sketch(idx), to_dev(cs), 1.0)
    return pr, (x0, y, idx, cs)


def single_call(ei, pr):
    step = ei.EIStep(pr.geom, pr.y, pr.sk, pr.cs, pr.lam, mc=pr.mc)
    loss, grad = step(pr.x, want_grad=pr.want_grad)
    return loss.clone(), (grad.clone() if pr.want_grad else None)


def assert_bitwise(plan, refs, what):
    losses, grads = plan.run()
    torch.cuda.synchronize()
    for i, (rl, rg) in enumerate(refs):
        assert torch.equal(losses[i], rl), f"{what}: loss of problem {i} differs ({losses[i].item()} vs {rl.item()})"
        if rg is not None:
            assert torch.equal(grads[i], rg), f"{what}: gradient of problem {i} differs " \
                f"(max |d| {float((grads[i] - rg).abs().max())})"


def small_mix(skei, ei):
    specs = synth.uneven_problems(count=6, sizes=(32, 48, 64, 80), angles=(20, 100), ratios=(2, 4, 8), copies=3,
                                  seed=6100)
    probs = [gpu_problem(skei, ei, p, grad=(i != 2), batch=(2 if i == 4 else 1)) for i, p in enumerate(specs)]
    return specs, probs


def test_plan_bitwise_equals_single_calls_in_every_configuration(skei):
    from paper_2411_05771_amd import capi, ei
    print("\n[plan] small mix, all dispatch modes and shapes", flush=True)
    specs, probs = small_mix(skei, ei)
    refs = [single_call(ei, pr) for pr in probs]
    plan = ei.EIPlan(probs)
    assert_bitwise(plan, refs, "default")
    for d in (capi.DISPATCH_PERSISTENT, capi.DISPATCH_STATIC):
        # ray shapes: rays per thread, + 100 x unit lines, + 10000 for three-wave workgroups,
        # + 20000 for four-unit LDS chunks, + 40000 / 80000 for six / eight waves
        for rpt, ga in ((1, 1), (2, 2), (3, 4), (4, 1), (10802, 14), (10003, 24), (1604, 44), (30402, 2), (20803, 1),
                        (40801, 1), (40402, 14), (80801, 24), (81602, 44), (60401, 2)):
            for s in capi.STAGES:
                shape = rpt if s in ("fwd", "bp_T") else ga if s in ("bp_resid", "adj") else 0
                plan.configure(s, d, shape)
            print(f"[plan] dispatch={d} rpt={rpt} ga={ga}", flush=True)
            assert_bitwise(plan, refs, f"dispatch {d} rpt {rpt} ga {ga}")
            # a second run reuses the self-resetting queue cursors
            assert_bitwise(plan, refs, f"dispatch {d} rpt {rpt} ga {ga}, second run")
    plan.close()


def test_plan_autotune_keeps_results_and_caches(skei, tmp_path):
    from paper_2411_05771_amd import capi, ei
    specs, probs = small_mix(skei, ei)
    refs = [single_call(ei, pr) for pr in probs]
    cache = str(tmp_path / "tune.txt")
    plan = ei.EIPlan(probs)
    chosen = plan.autotune(reps=3, cache_path=cache)
    print(f"\n[plan] autotuned {chosen}", flush=True)
    assert_bitwise(plan, refs, "autotuned")
    lines = open(cache).read().split("\n")
    assert len([ln for ln in lines if ln.strip()]) == len(capi.STAGES)
    plan2 = ei.EIPlan(probs)
    assert plan2.autotune(reps=3, cache_path=cache) == chosen    # served from the cache
    assert_bitwise(plan2, refs, "cached tuning")
    plan.close()
    plan2.close()


def test_plan_matches_oracle(skei, orc):
    from paper_2411_05771_amd import ei
    specs = synth.uneven_problems(count=3, sizes=(32, 48, 64), angles=(30, 90), ratios=(2, 4), copies=4, seed=6200)
    probs, want = [], []
    for p in specs:
        print(f"\n[plan-oracle] {p}", flush=True)
        pr, (x0, y, idx, cs) = oracle_problem(skei, ei, orc, p)
        probs.append(pr)
        wl, wg = orc.ei_loss_grad(x0, y, p["n_angles"], idx, cs, 1.0)
        want.append((wl, wg))
    plan = ei.EIPlan(probs)
    losses, grads = plan.run()
    for i, (wl, wg) in enumerate(want):
        e_l = abs(float(losses[i].item()) - wl) / abs(wl)
        e_g = relerr(host(grads[i]), wg)
        print(f"[plan-oracle] problem {i}: loss relerr {e_l:.2e}  grad relerr {e_g:.2e}", flush=True)
        assert e_l <= 1e-5
        assert e_g <= 1e-5
    plan.close()


def test_plan_uneven_64_problems(skei, orc):
    """The full uneven workload: 64 problems, 8 copies each, one launch per stage."""
    from paper_2411_05771_amd import ei
    specs = synth.uneven_problems()
    # the two cheapest problems and the cheapest 512 x 512 one (726 detectors)
    # are also checked against the oracle, so their inputs are made by the
    # oracle; the others are made on the device
    cost = lambda i: specs[i]["n"] ** 2 * specs[i]["n_angles"]
    sampled = sorted(range(len(specs)), key=cost)[:2]
    sampled.append(min((i for i in range(len(specs)) if specs[i]["n"] == 512), key=cost))
    probs, oracle_inputs = [], {}
    for i, p in enumerate(specs):
        if i in sampled:
            pr, inputs = oracle_problem(skei, ei, orc, p)
            oracle_inputs[i] = inputs
            probs.append(pr)
        else:
            probs.append(gpu_problem(skei, ei, p))
    print(f"\n[plan-64] {len(probs)} problems built", flush=True)
    refs = [single_call(ei, pr) for pr in probs]
    plan = ei.EIPlan(probs)
    assert_bitwise(plan, refs, "uneven 64")
    print("[plan-64] bitwise equal to single calls", flush=True)
    for i in sampled:
        p, pr = specs[i], probs[i]
        x0, y, idx, cs = oracle_inputs[i]
        wl, wg = orc.ei_loss_grad(x0, y, p["n_angles"], idx, cs, 1.0)
        e_l = abs(float(plan.losses[i].item()) - wl) / abs(wl)
        e_g = relerr(host(pr.grad), wg)
        print(f"[plan-64] problem {i} n={p['n']} n_angles={p['n_angles']} n_det={p['n_det']} m={p['m']}: "
              f"loss {e_l:.2e} grad {e_g:.2e}", flush=True)
        assert e_l <= 1e-5
        assert e_g <= 1e-5
    plan.close()


def test_plan_degenerate_problems(skei, orc):
    """A 2 x 2 image, one-angle sketches, one copy and a batch of two, mixed
    with an ordinary problem: bitwise equal to single calls, and at the
    oracle's values."""
    from paper_2411_05771_amd import ei
    base = dict(phantom_seed=synth.SEED_PHANTOM, sketch_seed=synth.SEED_SKETCH,
                rotation_seed=synth.SEED_ROTATION, noise_seed=synth.SEED_NOISE)
    specs = [dict(base, n=2, n_angles=4, n_det=3, m=1, copies=1, image="uniform"),
             dict(base, n=16, n_angles=7, n_det=23, m=1, copies=1),
             dict(base, n=40, n_angles=90, n_det=58, m=45, copies=2)]
    probs, inputs = [], []
    for p in specs:
        pr, inp = oracle_problem(skei, ei, orc, p)
        probs.append(pr)
        inputs.append(inp)
    refs = [single_call(ei, pr) for pr in probs]
    plan = ei.EIPlan(probs)
    for d in (0, 1):
        for s in ("fwd", "bp_T", "bp_resid", "adj"):
            plan.configure(s, d, 0)
        assert_bitwise(plan, refs, f"degenerate, dispatch {d}")
    for p, pr, (x0, y, idx, cs), (rl, rg) in zip(specs, probs, inputs, refs):
        wl, wg = orc.ei_loss_grad(x0, y, p["n_angles"], idx, cs, 1.0)
        e_l = abs(float(rl.item()) - wl) / abs(wl)
        e_g = relerr(host(rg), wg)
        print(f"[plan-degenerate] n={p['n']} m={p['m']} C={p['copies']}: loss {e_l:.2e} grad {e_g:.2e}",
              flush=True)
        assert e_l <= 1e-5 and e_g <= 1e-5
    plan.close()


def test_autotuned_ei_workload_plan_matches_oracle(skei, orc):
    """The EI-step workload (256^2, 360 angles, 363 detectors, 16 copies,
    random quarter sketch) through an autotuned one-problem plan -- the
    launch configuration the benchmark times -- against the oracle and,
    bitwise, against the one-call entry point."""
    from paper_2411_05771_amd import ei
    p = dict(n=256, n_angles=360, n_det=363, m=90, copies=16, phantom_seed=synth.SEED_PHANTOM,
             sketch_seed=synth.SEED_SKETCH, rotation_seed=synth.SEED_ROTATION, noise_seed=synth.SEED_NOISE)
    pr, (x0, y, idx, cs) = oracle_problem(skei, ei, orc, p)
    ref = single_call(ei, pr)
    plan = ei.EIPlan([pr])
    tuned = plan.autotune(reps=3)
    print(f"\n[plan-ei256] tuned {tuned}", flush=True)
    assert_bitwise(plan, [ref], "autotuned EI workload")
    wl, wg = orc.ei_loss_grad(x0, y, p["n_angles"], idx, cs, 1.0)
    e_l = abs(float(plan.losses[0].item()) - wl) / abs(wl)
    e_g = relerr(host(pr.grad), wg)
    print(f"[plan-ei256] loss {e_l:.2e} grad {e_g:.2e}", flush=True)
    assert e_l <= 1e-5 and e_g <= 1e-5
    plan.close()


def test_autotune_leaves_the_image_alone(skei):
    """A plan whose problem takes a fused gradient step (step != 0): tuning
    times many launches of every stage but must not move x; the next run then
    takes exactly one step, x - step * grad."""
    from paper_2411_05771_amd import ei
    p = synth.uneven_problems(count=1, sizes=(48,), angles=(40, 60), ratios=(2,), copies=3, seed=6300)[0]
    base = gpu_problem(skei, ei, p)
    x_before = base.x.clone()
    pr = ei.EIProblem(base.geom, base.x, base.y, base.sk, base.cs, 1.0, step=1e-3)
    plan = ei.EIPlan([pr])
    plan.autotune(reps=3)
    torch.cuda.synchronize()
    assert torch.equal(pr.x, x_before), "autotuning moved the image"
    ref = single_call(ei, pr)            # gradient at the unchanged image
    plan.run()
    torch.cuda.synchronize()
    assert torch.equal(pr.grad, ref[1])
    want = torch.addcmul(x_before, ref[1], torch.full_like(x_before, -1e-3))
    print(f"\n[plan-autotune] step applied, max |x - (x0 - step g)| = {float((pr.x - want).abs().max()):.2e}",
          flush=True)
    assert float((pr.x - want).abs().max()) <= 1e-6 * float(x_before.abs().max())
    assert not torch.equal(pr.x, x_before)
    plan.close()

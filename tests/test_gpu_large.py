"""Oracle parity at the largest sizes the serving workload runs.

1. The EI loss and gradient (Eq. skeilossttt, Algorithm 2 with the network
   taken as the identity) of a 1024 x 1024 job: 1440 angles, 1449 detectors
   (ceil(sqrt(2) N)), the interleaved sketch S_3 of ratio 8 (m = 180, the
   angles 3, 11, 19, ...), 16 rotated copies and the full-scan MC term --
   run through a one-problem batched plan with its own workspace, the way
   the server runs a job.  Bar: relative error <= 1e-5 in the loss and
   relative max-norm error <= 1e-5 in the gradient.
2. The rotations T_phi and their transpose (Sec. 4.1.3 group) on a
   1024 x 1024 image with 16 copies: relative max-norm error <= 1e-5 and
   adjoint gap <= 1e-6.

Inputs are made by the oracle (phantom, y = A x_true + 1 % noise,
x0 = FBP(y)); the device never makes an oracle input.
"""
import time

import numpy as np
import pytest
import torch

from gpu_util import adjoint_gap, f32, host, relerr, to_dev
from paper_2411_05771_amd import synth

pytestmark = pytest.mark.gpu


def test_ei_step_1024_job_against_oracle(skei, orc):
    from paper_2411_05771_amd import ei
    n, na, nd, ratio, k, c = 1024, 1440, 1449, 8, 3, 16
    print(f"\n[ei1024] n={n} n_angles={na} n_det={nd} ratio={ratio} (S_{k}) copies={c}", flush=True)
    t0 = time.time()
    xt = synth.ellipse_phantom(n, synth.SEED_PHANTOM + 77).astype(np.float64)[None]
    yc = orc.radon_fwd(xt, na, nd)
    y = f32(synth.add_relative_noise(yc, synth.std_noise(yc.shape, synth.SEED_NOISE + 77)))
    x0 = f32(orc.fbp(y, n, na))
    idx = synth.interleaved_sketch(na, ratio, k)
    cs = f32(synth.cos_sin(synth.rotation_angles(c, synth.SEED_ROTATION + 77)))
    want_l, want_g = orc.ei_loss_grad(x0, y, na, idx, cs, 1.0)
    print(f"[ei1024] oracle done in {time.time() - t0:.1f} s, loss {want_l:.9e}", flush=True)

    geom = skei.Geometry(n, na, nd)
    pr = ei.EIProblem(geom, to_dev(x0), to_dev(y), geom.sketch(idx), to_dev(cs), 1.0, own_workspace=True)
    plan = ei.EIPlan([pr])
    losses, grads = plan.run()
    torch.cuda.synchronize()
    e_l = abs(float(losses[0].item()) - want_l) / abs(want_l)
    e_g = relerr(host(grads[0]), want_g)
    print(f"[ei1024] loss relerr {e_l:.2e}; grad relerr {e_g:.2e}", flush=True)
    # the one-call entry point gives bitwise the same
    step = ei.EIStep(geom, pr.y, pr.sk, pr.cs, 1.0)
    l1, g1 = step(pr.x)
    assert torch.equal(l1, losses[0]) and torch.equal(g1, grads[0])
    plan.close()
    assert e_l <= 1e-5
    assert e_g <= 1e-5


def test_rotation_1024_parity_and_adjoint(skei, orc):
    n, c = 1024, 16
    print(f"\n[rotate1024] n={n} copies={c}", flush=True)
    x = f32(synth.ellipse_phantom(n, synth.SEED_PHANTOM + 5))
    cs = f32(synth.cos_sin(synth.rotation_angles(c, synth.SEED_ROTATION + 5)))
    csd = to_dev(cs)
    z = skei.rotate_(to_dev(x), csd)
    e = relerr(host(z), orc.rotate(x, cs))
    h = f32(np.random.default_rng(11).uniform(-1, 1, (c, n, n)))
    g = skei.rotate_adj_(to_dev(h), csd)
    e_adj = relerr(host(g), orc.rotate_adj(h, cs))
    gap = adjoint_gap(host(z), h, x, host(g))
    print(f"[rotate1024] rotate {e:.3e} rotate_adj {e_adj:.3e} adjoint gap {gap:.2e}", flush=True)
    assert e < 1e-5 and e_adj < 1e-5 and gap < 1e-6

"""The no-allocation EI entry point (skei_ei_loss_grad_noalloc) against the
workspace entry point (skei_ei_loss_grad), both called through the C ABI on
the same device inputs: loss and gradient must be bitwise equal (the same
kernels on the same data; the bar of the EI-step parity tests is 1e-5).

Two calls in a row share the library's static scratch: first the 256 x 256
/ 360-angle / 363-detector step with 16 copies and m = 90, then a smaller
one (64 x 64, 60 angles, 91 detectors, batch 2, 4 copies, m = 15) that
leaves the first call's data behind in the scratch, then the first again.
A step whose workspace exceeds the scratch is refused before anything is
enqueued."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2411_05771_amd import synth

pytestmark = pytest.mark.gpu


def _inputs(ops, n, na, nd, batch, copies, m, seed):
    from gpu_util import to_dev
    geom = ops.Geometry(n, na, nd)
    xt = to_dev(np.stack([synth.ellipse_phantom(n, synth.SEED_PHANTOM + seed + i) for i in range(batch)]))
    yc = ops.radon_fwd_(geom, xt, geom.full())
    z = to_dev(synth.std_noise(tuple(yc.shape), synth.SEED_NOISE + seed))
    y = (yc + 0.01 * yc.max() * z).contiguous()
    x0 = ops.fbp_(geom, y, geom.full()).contiguous()
    sk = geom.sketch(synth.random_sketch(na, m, synth.SEED_SKETCH + seed))
    cs = to_dev(synth.cos_sin(synth.rotation_angles(copies, synth.SEED_ROTATION + seed)))
    return geom, x0, y, sk, cs


def _both(ops, capi, geom, x0, y, sk, cs):
    dev = x0.device
    full = geom.full()
    b, copies = x0.shape[0], cs.shape[0]
    args = (geom.handle, ops._ptr(x0), ops._ptr(y), b, ops._ptr(full.dev), full.m, ops._ptr(sk.dev), sk.m, copies,
            ops._ptr(cs), ctypes.c_float(1.0))
    nb = int(capi.query("skei_ei_workspace_bytes", geom.handle, b, full.m, sk.m, copies))
    assert 0 < nb <= int(capi.query("skei_ei_noalloc_scratch_bytes"))
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    l_ref = torch.zeros((), dtype=torch.float64, device=dev)
    g_ref = torch.empty_like(x0)
    capi.call("skei_ei_loss_grad", *args, ops._ptr(l_ref), ops._ptr(g_ref), ops._ptr(ws), nb, ops._stream())
    l_na = torch.full((), -1.0, dtype=torch.float64, device=dev)
    g_na = torch.full_like(x0, float("nan"))
    capi.call("skei_ei_loss_grad_noalloc", *args, ops._ptr(l_na), ops._ptr(g_na), ops._stream())
    torch.cuda.synchronize()
    return l_ref, g_ref, l_na, g_na


def test_noalloc_matches_workspace_entry_point(skei):
    from paper_2411_05771_amd import capi
    ops = skei
    big = _inputs(ops, 256, 360, 363, 1, 16, 90, 0)
    small = _inputs(ops, 64, 60, 91, 2, 4, 15, 50)
    for name, case in (("256sq_16copies", big), ("64sq_batch2_4copies", small), ("256sq_again", big)):
        print(f"\n[noalloc] {name}", flush=True)
        l_ref, g_ref, l_na, g_na = _both(ops, capi, *case)
        print(f"[noalloc] {name}: loss {l_ref.item():.9e} / {l_na.item():.9e}; grad bitwise "
              f"{torch.equal(g_ref, g_na)}", flush=True)
        assert torch.equal(l_ref, l_na)
        assert torch.equal(g_ref, g_na)


def test_noalloc_refuses_beyond_scratch(skei):
    from paper_2411_05771_amd import capi
    ops = skei
    geom = ops.Geometry(1024, 1440, 1449)
    sk = geom.sketch(synth.interleaved_sketch(1440, 2, 0))
    full = geom.full()
    need = int(capi.query("skei_ei_workspace_bytes", geom.handle, 1, full.m, sk.m, 16))
    cap = int(capi.query("skei_ei_noalloc_scratch_bytes"))
    assert need > cap
    dummy = torch.zeros(16, device=geom.device)
    loss = torch.full((), -1.0, dtype=torch.float64, device=geom.device)
    rc = capi.query("skei_ei_loss_grad_noalloc", geom.handle, ops._ptr(dummy), ops._ptr(dummy), 1,
                    ops._ptr(full.dev), full.m, ops._ptr(sk.dev), sk.m, 16, ops._ptr(dummy), ctypes.c_float(1.0),
                    ops._ptr(loss), ops._ptr(dummy), ops._stream())
    torch.cuda.synchronize()
    print(f"[noalloc] need {need} B > scratch {cap} B: rc {rc} ({capi.strerror(rc)})", flush=True)
    assert rc == -6
    assert loss.item() == -1.0   # nothing ran

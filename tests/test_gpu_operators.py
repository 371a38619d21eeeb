"""GPU parity of every operator against the FP64 oracle (relative max-norm
1e-5), adjoint identities of the GPU operators (1e-6), determinism and
batch invariance.

Shapes: the 64^2 / 60-angle / 91-detector plain-operator workload, a ragged
case (image side not a multiple of 4 or 16, odd angle count so the 45-degree
tie appears, a sketch with repeats), the 256^2 / 360-angle / 363-detector EI
workload with 16 rotated copies and a random quarter sketch, a 1024^2 /
1440-angle / 1450-detector image at a 1/8 sketch (several detector passes per
thread), the 2 x 2 image, a one-angle sketch, and the largest supported image
(2032^2) and detector row (2048)."""
import numpy as np
import pytest

from gpu_util import adjoint_gap, f32, host, relerr, to_dev
from paper_2411_05771_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5
ADJ_TOL = 1e-6

CASES = {
    # name: (n, n_angles, n_det, batch, sketch)
    "plain64_full": (64, 60, 91, 1, "full"),
    "plain64_every4": (64, 60, 91, 1, "every4"),
    "ragged37": (37, 17, 53, 3, "repeats"),
    "ei256_quarter": (256, 360, 363, 16, "random"),
    "big1024_eighth": (1024, 1440, 1450, 1, "eighth"),
    # degenerate and extreme shapes: the smallest image, a one-angle sketch,
    # and the largest image and detector the library accepts
    "tiny2": (2, 4, 3, 2, "full"),
    "one_angle16": (16, 7, 23, 2, "single"),
    "max2032": (2032, 8, 2048, 1, "full"),
}


def make_case(name):
    n, na, nd, b, kind = CASES[name]
    if n < 8:   # too small for the ellipses to cover a pixel centre
        x = synth.uniform((b, n, n), synth.SEED_PHANTOM)
    else:
        x = np.stack([synth.ellipse_phantom(n, synth.SEED_PHANTOM + i) for i in range(b)]).astype(np.float64)
    if kind == "full":
        idx = np.arange(na, dtype=np.int32)
    elif kind == "every4":
        idx = synth.interleaved_sketch(na, 4, 0)
    elif kind == "repeats":
        idx = np.array([3, 0, 16, 4, 4, 12, 9, 13], dtype=np.int32)
    elif kind == "random":
        idx = synth.random_sketch(na, na // 4)
    elif kind == "single":
        idx = np.array([5], dtype=np.int32)
    else:
        idx = synth.interleaved_sketch(na, 8, 3)
    return n, na, nd, x, idx


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request, skei, orc):
    name = request.param
    n, na, nd, x, idx = make_case(name)
    print(f"\n[case {name}] n={n} n_angles={na} n_det={nd} batch={x.shape[0]} m={idx.size}", flush=True)
    geom = skei.Geometry(n, na, nd)
    sk = geom.sketch(idx)
    return dict(name=name, n=n, na=na, nd=nd, x=x, idx=idx, geom=geom, sk=sk, ops=skei, orc=orc)


def test_radon_fwd(case):
    ops, orc = case["ops"], case["orc"]
    y = ops.radon_fwd_(case["geom"], to_dev(case["x"]), case["sk"])
    want = orc.radon_fwd(f32(case["x"]), case["na"], case["nd"], case["idx"])
    e = relerr(host(y), want)
    print(f"radon_fwd relerr {e:.3e}")
    assert e < TOL


def test_radon_resid(case):
    """S y - A_S x (the MC residual of the EI loss) against the oracle.  y is
    A x plus 1 % noise, so the residual is ~100x smaller than y: the bar
    relative to max |residual| holds only if the projection and the
    difference are carried in double before the float rounding."""
    ops, orc = case["ops"], case["orc"]
    x = f32(case["x"])
    y_clean = orc.radon_fwd(x, case["na"], case["nd"])
    y_full = f32(synth.add_relative_noise(y_clean, synth.std_noise(y_clean.shape, synth.SEED_NOISE + 9)))
    r = ops.radon_resid_(case["geom"], to_dev(x), to_dev(y_full), case["sk"])
    want = y_full[:, case["idx"]] - orc.radon_fwd(x, case["na"], case["nd"], case["idx"])
    e = relerr(host(r), want)
    print(f"radon_resid relerr {e:.3e} (max|r| / max|y| = {np.abs(want).max() / np.abs(y_full).max():.2e})")
    assert e < TOL


def test_radon_adj(case):
    ops, orc = case["ops"], case["orc"]
    ysino = orc.radon_fwd(f32(case["x"]), case["na"], case["nd"], case["idx"])
    ysino = f32(ysino)
    x = ops.radon_adj_(case["geom"], to_dev(ysino), case["sk"])
    want = orc.radon_adj(ysino, case["n"], case["na"], case["idx"])
    e = relerr(host(x), want)
    print(f"radon_adj relerr {e:.3e}")
    assert e < TOL


def test_ramp_backproject_fbp(case):
    ops, orc = case["ops"], case["orc"]
    geom, sk = case["geom"], case["sk"]
    p = f32(orc.radon_fwd(f32(case["x"]), case["na"], case["nd"], case["idx"]))
    pd = to_dev(p)
    e_ramp = relerr(host(ops.ramp_(geom, pd)), orc.ramp(p))
    q = f32(orc.ramp(p))
    e_bp = relerr(host(ops.backproject_(geom, to_dev(q), sk)), orc.backproject(q, case["n"], case["na"], case["idx"]))
    e_fbp = relerr(host(ops.fbp_(geom, pd, sk)), orc.fbp(p, case["n"], case["na"], case["idx"]))
    print(f"ramp {e_ramp:.3e} backproject {e_bp:.3e} fbp {e_fbp:.3e}")
    assert e_ramp < TOL and e_bp < TOL and e_fbp < TOL


def test_backproject_T_and_fbp_adj(case):
    ops, orc = case["ops"], case["orc"]
    geom, sk = case["geom"], case["sk"]
    x = f32(case["x"])
    xd = to_dev(x)
    e_bpT = relerr(host(ops.backproject_T_(geom, xd, sk)), orc.backproject_T(x, case["na"], case["nd"], case["idx"]))
    e_fa = relerr(host(ops.fbp_adj_(geom, xd, sk)), orc.fbp_adj(x, case["na"], case["nd"], case["idx"]))
    print(f"backproject_T {e_bpT:.3e} fbp_adj {e_fa:.3e}")
    assert e_bpT < TOL and e_fa < TOL


def test_adjoint_identities_on_gpu(case):
    ops = case["ops"]
    geom, sk = case["geom"], case["sk"]
    b = case["x"].shape[0]
    g = np.random.default_rng(7)
    x = g.uniform(0, 1, (b, case["n"], case["n"]))
    y = g.uniform(0, 1, (b, sk.m, case["nd"]))
    xd, yd = to_dev(x), to_dev(y)
    x32, y32 = f32(x), f32(y)
    gaps = {
        "A": adjoint_gap(host(ops.radon_fwd_(geom, xd, sk)), y32, x32, host(ops.radon_adj_(geom, yd, sk))),
        "B": adjoint_gap(host(ops.backproject_T_(geom, xd, sk)), y32, x32, host(ops.backproject_(geom, yd, sk))),
        "fbp": adjoint_gap(host(ops.fbp_(geom, yd, sk)), x32, y32, host(ops.fbp_adj_(geom, xd, sk))),
    }
    print("adjoint gaps", {k: f"{v:.2e}" for k, v in gaps.items()})
    assert max(gaps.values()) < ADJ_TOL


def test_deterministic_and_batch_invariant(case):
    ops = case["ops"]
    geom, sk = case["geom"], case["sk"]
    xd = to_dev(case["x"])
    y1 = ops.radon_fwd_(geom, xd, sk)
    y2 = ops.radon_fwd_(geom, xd, sk)
    assert np.array_equal(host(y1), host(y2))
    a1 = ops.radon_adj_(geom, y1, sk)
    a2 = ops.radon_adj_(geom, y1.clone(), sk)
    assert np.array_equal(host(a1), host(a2))
    if xd.shape[0] > 1:
        alone = ops.radon_fwd_(geom, xd[1:2].contiguous(), sk)
        assert np.array_equal(host(alone[0]), host(y1[1]))
        alone_a = ops.radon_adj_(geom, y1[1:2].contiguous(), sk)
        assert np.array_equal(host(alone_a[0]), host(a1[1]))


def test_sketch_rows_bitwise_match_full_operator(skei):
    geom = skei.Geometry(64, 60, 91)
    x = to_dev(synth.ellipse_phantom(64, 1000))
    full = host(skei.radon_fwd_(geom, x, geom.full()))
    idx = np.array([59, 0, 17, 17, 44], dtype=np.int32)
    part = host(skei.radon_fwd_(geom, x, geom.sketch(idx)))
    assert np.array_equal(part, full[idx])


def test_rotation_parity_and_adjoint(skei, orc):
    n, copies = 256, 16
    x = f32(synth.ellipse_phantom(n, 1000))
    cs = f32(synth.cos_sin(synth.rotation_angles(copies)))
    csd = to_dev(cs)
    z = skei.rotate_(to_dev(x), csd)
    e = relerr(host(z), orc.rotate(x, cs))
    h = np.random.default_rng(3).uniform(-1, 1, (copies, n, n))
    g = skei.rotate_adj_(to_dev(h), csd)
    e_adj = relerr(host(g), orc.rotate_adj(f32(h), cs))
    gap = adjoint_gap(host(z), f32(h), x, host(g))
    print(f"rotate {e:.3e} rotate_adj {e_adj:.3e} adjoint gap {gap:.2e}")
    assert e < TOL and e_adj < TOL and gap < ADJ_TOL
    # the exact permutations: phi = 0 and pi/2
    special = to_dev(np.array([[1.0, 0.0], [0.0, 1.0]]))
    zz = host(skei.rotate_(to_dev(x), special))
    assert np.array_equal(zz[0], x) and np.array_equal(zz[1], np.rot90(x, -1))


@pytest.mark.parametrize("n,copies,batch", [(37, 5, 2), (17, 3, 1), (2, 1, 2)])
def test_rotation_ragged_tiles(skei, orc, n, copies, batch):
    """Images that are not a whole number of tiles (partial tiles, and taps
    clamped at every border), copy counts that leave some copy groups empty,
    and batches of two."""
    rng = np.random.default_rng(100 + n)
    x = f32(rng.uniform(0, 1, (batch, n, n)))
    cs = f32(synth.cos_sin(rng.uniform(0, 2 * np.pi, copies)))
    csd = to_dev(cs)
    z = skei.rotate_(to_dev(x), csd)
    e = relerr(host(z), orc.rotate(x, cs))
    h = f32(rng.uniform(0, 1, (batch, copies, n, n)))
    g = skei.rotate_adj_(to_dev(h), csd)
    e_adj = relerr(host(g), orc.rotate_adj(h, cs))
    gap = adjoint_gap(host(z), h, x, host(g))
    print(f"[rotate n={n} C={copies} B={batch}] {e:.3e} adj {e_adj:.3e} gap {gap:.2e}")
    assert e < TOL and e_adj < TOL and gap < ADJ_TOL


def test_sumsq(skei):
    a = np.random.default_rng(4).standard_normal(1_000_003)
    b = np.random.default_rng(5).standard_normal(1_000_003)
    got = float(skei.sumsq_diff_(to_dev(a), to_dev(b)).item())
    want = float(np.sum((f32(a) - f32(b)) ** 2))
    assert abs(got - want) <= 1e-12 * want


def test_invalid_arguments_raise(skei):
    from paper_2411_05771_amd import capi
    geom = skei.Geometry(32, 10, 47)
    with pytest.raises(ValueError):
        geom.sketch([0, 10])
    with pytest.raises(ValueError):
        skei.radon_fwd_(geom, to_dev(np.zeros((2, 31, 31))), geom.full())
    with pytest.raises(ValueError):
        skei.radon_fwd_(geom, to_dev(np.zeros((2, 32, 32))).cpu(), geom.full())
    with pytest.raises(capi.SkeiError):
        skei.Geometry(32, 10, 4096)

"""The multicoil MRI operator and coil sketches on the GPU (skei_mri_fwd /
skei_mri_adj / skei_coil_* through the C-ABI) against the FP64 oracle
(oracle/mri.py) on the same seeded inputs, all made on the host by synth and
the oracle (complex values rounded to complex64 first, so both sides see the
same numbers):

- A, A^H, the weighted forward A W and the pseudo-inverse D^-1 A^H at
  N = 4 ... 1024 (several line groups per plane, one-line groups at 1024),
  1, 3 and 15 coils, batches 1 and 3: relative max-norm error <= 1e-5 (the
  FP32 transform's rounding, log2 N stages per pass, is ~1e-7 of the norm);
- the adjoint gap |<A x, k> - <x, A^H k>| / (||A x|| ||k||) <= 1e-6;
- coil mixing: a 0/1 selector returns the selected coils bitwise, a complex
  mix matches to 1e-6; the FP64 coil covariance matches to 1e-9;
- Algorithm 3's coil sketch end to end (covariance, PCA, virtual maps and
  data, S_c): the sketched maps and data match the oracle's to 1e-5;
- the sketched EI loss and its image gradient (autograd over the library's
  operators and rotations) match the oracle's closed-form gradient to 1e-5
  for the full operator, the classical sketch and the coil sketch (the
  oracle running its own covariance, PCA and sketch on the same data);
- sizes that are not powers of two are refused."""
import numpy as np
import pytest
import torch

from gpu_util import dev
from oracle import mri as omri
from paper_2411_05771_amd import capi, synth

pytestmark = pytest.mark.gpu


def relerr(got, want):
    """Relative max-norm error of complex arrays: max |got - want| / max |want|
    (moduli of the complex differences, both parts compared)."""
    got = np.asarray(got, dtype=np.complex128)
    want = np.asarray(want, dtype=np.complex128)
    return float(np.max(np.abs(got - want)) / np.max(np.abs(want)))


def c64(a):
    return np.asarray(a, dtype=np.complex64).astype(np.complex128)


def cdev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).to(dev())


def chost(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def inputs(n, nc, batch, seed):
    maps = c64(synth.coil_maps(nc, n, seed))
    mask = synth.cartesian_mask(n, 4 if n >= 8 else 2, seed=seed)
    x = c64(np.stack([synth.complex_phantom(n, synth.SEED_PHANTOM + seed + i) for i in range(batch)]))
    return maps, mask, x


@pytest.fixture(scope="module")
def mri(skei):
    from paper_2411_05771_amd import mri as m
    return m


@pytest.mark.parametrize("n,nc,batch", [(4, 1, 1), (8, 3, 3), (16, 15, 1), (64, 3, 3), (128, 15, 1), (128, 15, 3),
                                        (256, 3, 1), (1024, 1, 1)])
def test_forward_adjoint_and_pinv(mri, orc, n, nc, batch):
    maps, mask, x = inputs(n, nc, batch, 7000 + n + nc)
    op = mri.MRIOperator(maps, mask, dev())
    k = op.fwd_(cdev(x))
    k_o = omri.mri_fwd(x, maps, mask)
    e_f = relerr(chost(k), k_o)
    kk = c64(omri.mri_fwd(x, maps, np.ones((n, n))) + 0.1 * synth.complex_noise((batch, nc, n, n), 5))
    xa = op.adj_(cdev(kk))
    e_a = relerr(chost(xa), omri.mri_adj(kk, maps, mask))
    xp = op.pinv_(cdev(kk))
    e_p = relerr(chost(xp), omri.mri_pinv(kk, maps, mask))
    w = omri.coil_weights(maps)
    e_w = relerr(chost(op.fwd_(cdev(x), weighted=True)), omri.mri_fwd(w[None] * x, maps, mask))
    kh, xh = chost(k), chost(xa)
    gap = abs(np.vdot(kh, kk) - np.vdot(x, xh)) / (np.linalg.norm(kh) * np.linalg.norm(kk))
    print(f"\n[mri] n={n} nc={nc} b={batch}: A {e_f:.1e} A^H {e_a:.1e} pinv {e_p:.1e} AW {e_w:.1e} gap {gap:.1e}",
          flush=True)
    assert max(e_f, e_a, e_p, e_w) <= 1e-5 and gap <= 1e-6


def test_coil_mix_and_covariance(mri, orc):
    n, nc = 32, 6
    maps, mask, x = inputs(n, nc, 2, 11)
    k = c64(omri.mri_fwd(x, maps, mask))
    kd = cdev(k)
    sel = np.zeros((3, nc))
    sel[[0, 1, 2], [4, 0, 5]] = 1.0
    assert torch.equal(mri.coil_mix_(sel, kd), kd[:, [4, 0, 5]])
    G = c64(synth.complex_noise((4, nc), 3))
    assert relerr(chost(mri.coil_mix_(G, kd)), omri.coil_mix(G, k)) <= 1e-6
    V = mri.coil_covariance_(kd[0])
    assert relerr(V, omri.coil_covariance(k[0])) <= 1e-9
    assert relerr(V.imag, omri.coil_covariance(k[0]).imag) <= 1e-8   # the imaginary parts on their own


def noisy_measurement(maps, mask, x, seed):
    k = omri.mri_fwd(x, maps, mask)
    return c64(k + 0.005 * np.abs(k).max() * synth.complex_noise(k.shape, seed) * mask)


def test_coil_sketch_pipeline(mri, orc):
    n, nc, L, R, mc = 64, 15, 12, 3, 5
    maps, mask, x = inputs(n, nc, 1, 21)
    y = noisy_measurement(maps, mask, x, 22)
    op = mri.MRIOperator(maps, mask, dev())
    op_s, y_s, info = mri.coil_sketch(op, cdev(y), L, R, mc, seed=23)
    Q, w = omri.pca_coils(omri.coil_covariance(y[0]), L)
    S_c = omri.coil_sketch_matrix(L, R, synth.rademacher_signs(mc - R, L - R, 23))
    assert np.array_equal(info["S_c"], S_c)
    assert np.max(np.abs(info["Q"] - Q)) < 1e-6 and np.max(np.abs(info["eigenvalues"] - w)) < 1e-9 * w[0]
    maps_s = omri.coil_mix(S_c, omri.coil_mix(Q.T, maps))
    y_so = omri.coil_mix(S_c, omri.coil_mix(Q.T, y))
    e_m, e_y = relerr(chost(op_s.maps), maps_s), relerr(chost(y_s), y_so)
    print(f"\n[mri] coil sketch L={L} R={R} Mc={mc}: maps {e_m:.1e} data {e_y:.1e}", flush=True)
    assert e_m <= 1e-5 and e_y <= 1e-5


@pytest.mark.parametrize("kind", ["full", "classical", "coil"])
def test_ei_loss_and_gradient(mri, orc, kind):
    n, nc = 64, 15
    maps, mask, x_true = inputs(n, nc, 1, 31)
    y = noisy_measurement(maps, mask, x_true, 32)
    op = mri.MRIOperator(maps, mask, dev())
    yd = cdev(y)
    if kind == "full":
        op_s, ys, maps_o, y_o = op, yd, maps, y
    elif kind == "classical":
        coils = [2, 7, 11, 14, 0]
        op_s, ys = mri.classical_sketch(op, yd, coils)
        maps_o, y_o = maps[coils], y[:, coils]
    else:
        op_s, ys, _ = mri.coil_sketch(op, yd, 15, 3, 5, seed=33)
        # the oracle's own coil sketch of the same measurement
        Q, _ = omri.pca_coils(omri.coil_covariance(y[0]), 15)
        S_c = omri.coil_sketch_matrix(15, 3, synth.rademacher_signs(2, 12, 33))
        maps_o = omri.coil_mix(S_c, omri.coil_mix(Q.T, maps))
        y_o = omri.coil_mix(S_c, omri.coil_mix(Q.T, y))
    x0 = c64(omri.mri_pinv(y, maps, mask))          # [1, N, N]
    phi = np.deg2rad(np.array([17.0, 212.0]))
    cs = synth.cos_sin(phi)
    xd = cdev(x0).requires_grad_(True)
    loss, _, _ = mri.mri_ei_loss(xd, ys, op_s, torch.from_numpy(cs.astype(np.float32)).to(dev()), lam=0.8)
    loss.backward()
    l_o, g_o = omri.mri_ei_loss_grad(x0, y_o, maps_o, mask, cs.astype(np.float32).astype(np.float64), lam=0.8)
    e_l = abs(float(loss) - l_o) / l_o
    e_g = relerr(chost(xd.grad), g_o)
    print(f"\n[mri] EI {kind}: loss {e_l:.1e} grad {e_g:.1e}", flush=True)
    assert e_l <= 1e-5 and e_g <= 1e-5


def test_rejects_bad_sizes(mri):
    maps = cdev(np.ones((2, 12, 12)))
    x = cdev(np.ones((1, 12, 12)))
    k = torch.empty((1, 2, 12, 12), device=dev(), dtype=torch.complex64)
    mask = torch.ones((12, 12), device=dev())
    rc = capi.lib().skei_mri_fwd(maps.data_ptr(), 2, 12, x.data_ptr(), 1, mask.data_ptr(), None, k.data_ptr(), None)
    assert rc == -1
    rc = capi.lib().skei_mri_fwd(maps.data_ptr(), 0, 16, x.data_ptr(), 1, mask.data_ptr(), None, k.data_ptr(), None)
    assert rc == -1

"""The MRI EI iteration captured in a HIP graph (mri.MRIGraphStep) against the
same iterations run eagerly: five replays with different rotations, each
followed by unrelated eager library work and a synchronisation, must leave
the image and the loss equal to the eager iterations' (the graph holds no
memset node; every reduction is the library's fixed-order one).  Also: the
library-reduced loss and its gradient equal torch's own sums to rounding,
and a reset returns the captured iteration to its start."""
import numpy as np
import pytest
import torch

from gpu_util import dev
from oracle import mri as omri
from paper_2411_05771_amd import synth

pytestmark = pytest.mark.gpu


def cdev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).to(dev())


@pytest.fixture(scope="module")
def setup(skei):
    from paper_2411_05771_amd import mri, ttt
    n, nc = 64, 8
    maps = synth.coil_maps(nc, n, 41)
    mask = synth.cartesian_mask(n, 4, seed=41)
    x_true = synth.complex_phantom(n, synth.SEED_PHANTOM + 41)[None]
    k = omri.mri_fwd(x_true, maps, mask)
    y = k + 0.005 * np.abs(k).max() * synth.complex_noise(k.shape, 42) * mask
    op = mri.MRIOperator(maps, mask, dev())
    x0 = cdev(omri.mri_pinv(y, maps, mask))
    return mri, op, cdev(y), x0, ttt.rotation_table(dev())


def test_library_sums_match_torch_sums(setup):
    mri, op, y, x0, rot = setup
    grads, losses = [], []
    for lib in (True, False):
        x = x0.clone().requires_grad_(True)
        loss, _, _ = mri.mri_ei_loss(x, y, op, rot[16:17], 0.7, library_sums=lib)
        loss.backward()
        grads.append(x.grad.detach().clone())
        losses.append(float(loss))
    e_l = abs(losses[0] - losses[1]) / losses[1]
    e_g = float(torch.max(torch.abs(grads[0] - grads[1])) / torch.max(torch.abs(grads[1])))
    print(f"\n[mri-graph] library vs torch sums: loss {e_l:.1e} grad {e_g:.1e}", flush=True)
    assert e_l <= 1e-12 and e_g <= 1e-6


def test_graph_replays_equal_eager_iterations(setup):
    mri, op, y, x0, rot = setup
    seq = [16, 211, 4, 89, 300]
    xe = x0.clone().requires_grad_(True)
    opt = torch.optim.Adam([xe], lr=5e-4, capturable=True)
    eager = []
    for i in seq:
        opt.zero_grad(set_to_none=True)
        loss, _, _ = mri.mri_ei_loss(xe, y, op, rot[i:i + 1], 1.0, library_sums=True)
        loss.backward()
        opt.step()
        eager.append((xe.detach().clone(), float(loss)))
    g = mri.MRIGraphStep(x0, y, op)
    assert torch.equal(g.x.detach(), x0)
    for rep, (i, (x_ref, l_ref)) in enumerate(zip(seq, eager)):
        loss = g.step(rot[i:i + 1])
        torch.cuda.synchronize()
        op.adj_(y)                      # the program's own eager work between replays
        torch.cuda.synchronize()
        dx = float(torch.max(torch.abs(g.x.detach() - x_ref)) / torch.max(torch.abs(x_ref)))
        dl = abs(float(loss) - l_ref) / l_ref
        print(f"[mri-graph] replay {rep}: image {dx:.1e} loss {dl:.1e}", flush=True)
        assert dx <= 1e-6 and dl <= 1e-9
    g.reset(x0)
    loss = g.step(rot[seq[0]:seq[0] + 1])
    torch.cuda.synchronize()
    assert float(torch.max(torch.abs(g.x.detach() - eager[0][0]))) <= 1e-6 * float(torch.max(torch.abs(eager[0][0])))


def test_classical_sketch_graph_equals_eager(setup):
    mri, op, y, x0, rot = setup
    subsets = [[1, 4, 6], [0, 7, 2], [5, 3, 1]]
    seq = [30, 150, 270]
    xe = x0.clone().requires_grad_(True)
    opt = torch.optim.Adam([xe], lr=5e-4, capturable=True)
    eager = []
    for i, coils in zip(seq, subsets):
        op_s, y_s = mri.classical_sketch(op, y, coils)
        opt.zero_grad(set_to_none=True)
        loss, _, _ = mri.mri_ei_loss(xe, y_s, op_s, rot[i:i + 1], 1.0, library_sums=True)
        loss.backward()
        opt.step()
        eager.append((xe.detach().clone(), float(loss)))
    g = mri.MRIGraphStep(x0, y, op, select=3)
    for rep, (i, coils, (x_ref, l_ref)) in enumerate(zip(seq, subsets, eager)):
        loss = g.step(rot[i:i + 1], coils)
        torch.cuda.synchronize()
        op.fwd_(x0)
        torch.cuda.synchronize()
        dx = float(torch.max(torch.abs(g.x.detach() - x_ref)) / torch.max(torch.abs(x_ref)))
        dl = abs(float(loss) - l_ref) / l_ref
        print(f"[mri-graph] classical replay {rep} coils {coils}: image {dx:.1e} loss {dl:.1e}", flush=True)
        assert dx <= 1e-6 and dl <= 1e-9


"""Sketched test-time EI loss and gradient (Eq. skeilossttt, Algorithm 2).

With the reconstruction network taken as the identity (the network, its
weights and its optimiser are outside this library), one iteration of
Algorithm 2 evaluates, for the current image estimate x:

    r_MC   = y[mc] - A_mc x                              (MC term)
    z_c    = T_c x,  r_c = z_c - fbp_S(A_S z_c)          (sketched EI term)
    loss   = ||r_MC||^2 + (lambda / C) sum_c ||r_c||^2
    grad   = -2 A_mc^T r_MC + (2 lambda / C) sum_c T_c^T (r_c - A_S^T fbp_S^T r_c)

``EIStep`` runs this as one fused sequence of library kernels
(``skei_ei_loss_grad``) with a reusable device workspace.  ``ei_loss_autograd``
builds the same loss from the differentiable operators of ``ops`` so that
torch.autograd differentiates it through the hand-written transposes.
"""
from __future__ import annotations

import ctypes

import torch

from . import capi, ops


class EIStep:
    """Fused EI loss/gradient for a fixed geometry, batch and copy count.

    y: full measured sinogram [B, N_theta, N_det] (device, float32).
    The sketch, MC angle list and rotations may change between calls
    (``set_sketch`` / ``set_rotations``) without reallocating.
    """

    def __init__(self, geom: ops.Geometry, y: torch.Tensor, sketch, cos_sin, lam: float = 1.0, mc=None):
        self.geom = geom
        y3 = y.unsqueeze(0) if y.dim() == 2 else y
        ops._check(y3, torch.float32, geom.device, "y")
        if tuple(y3.shape[1:]) != (geom.n_angles, geom.n_det):
            raise ValueError("y must be the full sinogram [B, N_theta, N_det]")
        self.y = y3
        self.batch = y3.shape[0]
        self.lam = float(lam)
        self.sk = ops._as_sketch(geom, sketch)
        self.mc = ops._as_sketch(geom, mc)
        self.cs = cos_sin if isinstance(cos_sin, torch.Tensor) else ops.cos_sin_tensor(cos_sin, geom.device)
        self.copies = self.cs.shape[0]
        self._alloc()
        self.loss = torch.zeros((), dtype=torch.float64, device=geom.device)

    def _alloc(self):
        nb = capi.query("skei_ei_workspace_bytes", self.geom.handle, self.batch, self.mc.m, self.sk.m, self.copies)
        self._ws_bytes = int(nb)
        self._ws = torch.empty(max(self._ws_bytes, 1), dtype=torch.uint8, device=self.geom.device)

    def set_sketch(self, sketch):
        sk = ops._as_sketch(self.geom, sketch)
        grow = sk.m > self.sk.m
        self.sk = sk
        if grow:
            self._alloc()

    def set_rotations(self, cos_sin):
        cs = cos_sin if isinstance(cos_sin, torch.Tensor) else ops.cos_sin_tensor(cos_sin, self.geom.device)
        if cs.shape[0] != self.copies:
            raise ValueError("copy count is fixed per EIStep")
        self.cs = cs

    def __call__(self, x: torch.Tensor, grad: torch.Tensor | None = None, want_grad: bool = True):
        x3 = ops._img(self.geom, x)
        if x3.shape[0] != self.batch:
            raise ValueError("batch mismatch")
        if want_grad and grad is None:
            grad = torch.empty_like(x3)
        capi.call("skei_ei_loss_grad", self.geom.handle, ops._ptr(x3), ops._ptr(self.y), self.batch,
                  ops._ptr(self.mc.dev), self.mc.m, ops._ptr(self.sk.dev), self.sk.m, self.copies,
                  ops._ptr(self.cs), ctypes.c_float(self.lam), ops._ptr(self.loss),
                  ops._ptr(grad) if want_grad else None, ops._ptr(self._ws), self._ws_bytes, ops._stream())
        if want_grad and x.dim() == 2:
            grad = grad[0]
        return self.loss, grad


def ei_loss_autograd(x, y, geom: ops.Geometry, sketch, cos_sin, lam: float = 1.0, mc=None):
    """The same loss assembled from the differentiable operators.

    x: [B,N,N] (requires_grad as needed); y: [B,N_theta,N_det].  The EI
    subtraction and the sums of squares are torch glue; every operator
    (the MC residual y[mc] - A_mc x, T, A_S, fbp_S and their transposes in
    backward) is a library call.
    """
    sk = ops._as_sketch(geom, sketch)
    mcs = ops._as_sketch(geom, mc)
    cs = cos_sin if isinstance(cos_sin, torch.Tensor) else ops.cos_sin_tensor(cos_sin, geom.device)
    x3 = x.unsqueeze(0) if x.dim() == 2 else x
    y3 = y.unsqueeze(0) if y.dim() == 2 else y
    b, n = x3.shape[0], geom.n
    c = cs.shape[0]
    r_mc = ops.radon_resid(x3, y3, geom, mcs)   # the difference is taken in double
    z = ops.rotate(x3, cs).reshape(b * c, n, n)
    w = ops.fbp(ops.radon_fwd(z, geom, sk), geom, sk)
    r = z - w
    return (r_mc.double() ** 2).sum() + (lam / c) * (r.double() ** 2).sum()


class EIProblem:
    """One problem of a batched plan: the inputs of an ``EIStep`` call.

    x: image batch [B,N,N]; y: full sinogram [B,N_theta,N_det]; both device
    float32 and kept alive (and in place) for the plan's lifetime -- the plan
    binds their addresses.  ``grad=False`` asks for the loss only; ``step``
    > 0 makes every run end with the gradient step x -= step * grad.
    """

    def __init__(self, geom: ops.Geometry, x, y, sketch, cos_sin, lam: float = 1.0, mc=None, grad: bool = True,
                 step: float = 0.0, own_workspace: bool = False):
        self.geom = geom
        self.x = ops._img(geom, x)
        y3 = y.unsqueeze(0) if y.dim() == 2 else y
        ops._check(y3, torch.float32, geom.device, "y")
        if tuple(y3.shape) != (self.x.shape[0], geom.n_angles, geom.n_det):
            raise ValueError("y must be the full sinogram [B, N_theta, N_det] of the image batch")
        self.y = y3
        self.sk = ops._as_sketch(geom, sketch)
        self.mc = ops._as_sketch(geom, mc)
        self.cs = cos_sin if isinstance(cos_sin, torch.Tensor) else ops.cos_sin_tensor(cos_sin, geom.device)
        self.lam = float(lam)
        self.want_grad = bool(grad)
        self.grad = torch.empty_like(self.x) if grad else None
        if step and not grad:
            raise ValueError("a gradient step needs the gradient")
        self.step = float(step)   # x -= step * grad after each evaluation (in place)
        self.work = None          # own scratch (kept across plans), else carved from a plan's workspace
        if own_workspace:
            # the size query reads no memory; the loss address is a placeholder
            nb = int(capi.query("skei_ei_problem_workspace_bytes", ctypes.byref(self.record(256))))
            if nb == 0:
                raise ValueError("invalid problem")
            self.work = torch.empty(nb, dtype=torch.uint8, device=geom.device)

    def record(self, loss_ptr: int) -> capi.EiProblem:
        h = self.geom.handle
        return capi.EiProblem(h.value if isinstance(h, ctypes.c_void_p) else h, self.x.shape[0],
                              self.x.data_ptr(), self.y.data_ptr(), self.mc.dev.data_ptr(), self.mc.m,
                              self.sk.dev.data_ptr(), self.sk.m, self.cs.shape[0], self.cs.data_ptr(), self.lam,
                              loss_ptr, self.grad.data_ptr() if self.grad is not None else None, self.step,
                              self.work.data_ptr() if self.work is not None else None,
                              self.work.numel() if self.work is not None else 0)


class EIPlan:
    """Batched EI step over problems of different sizes (skei_ei_plan_*).

    Every stage of the step runs as one launch for all problems; problem i's
    loss lands in ``losses[i]`` and its gradient in ``problems[i].grad``,
    bitwise equal to what ``EIStep`` gives for it alone.
    """

    def __init__(self, problems: list[EIProblem]):
        if not problems:
            raise ValueError("a plan needs at least one problem")
        dev = problems[0].geom.device
        self.problems = list(problems)
        self.losses = torch.zeros(len(problems), dtype=torch.float64, device=dev)
        base = self.losses.data_ptr()
        self._recs = (capi.EiProblem * len(problems))(*[p.record(base + 8 * i) for i, p in enumerate(problems)])
        self.workspace_bytes = int(capi.query("skei_ei_plan_workspace_bytes", self._recs, len(problems)))
        self._ws = (torch.empty(self.workspace_bytes, dtype=torch.uint8, device=dev)
                    if self.workspace_bytes else None)
        self._dev = dev
        h = ctypes.c_void_p()
        capi.call("skei_ei_plan_create", self._recs, len(problems),
                  ops._ptr(self._ws) if self._ws is not None else None, self.workspace_bytes, ctypes.byref(h))
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan is closed")
        return self._h

    def run(self):
        capi.call("skei_ei_plan_run", self.handle, ops._stream())
        return self.losses, [p.grad for p in self.problems]

    def configure(self, stage: str | int, dispatch: int, shape: int = 0):
        s = capi.STAGES.index(stage) if isinstance(stage, str) else int(stage)
        capi.call("skei_ei_plan_configure", self.handle, s, int(dispatch), int(shape))

    def config(self, stage: str | int):
        s = capi.STAGES.index(stage) if isinstance(stage, str) else int(stage)
        d, sh = ctypes.c_int(), ctypes.c_int()
        capi.call("skei_ei_plan_get_config", self.handle, s, ctypes.byref(d), ctypes.byref(sh))
        return d.value, sh.value

    def autotune(self, reps: int = 5, cache_path: str | None = None):
        """Times every stage's (dispatch, shape) candidates and keeps the best.
        The problems' images are left unchanged (no gradient step is applied)."""
        capi.call("skei_ei_plan_autotune", self.handle, ops._stream(), int(reps),
                  cache_path.encode() if cache_path else None)
        return {name: self.config(name) for name in capi.STAGES}

    def close(self):
        if self._h is not None:
            torch.cuda.synchronize(self._dev)
            capi.call("skei_ei_plan_destroy", self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

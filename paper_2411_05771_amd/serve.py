"""Continuous-batching server for test-time EI adaptation jobs.

A job is one measured sinogram y to be reconstructed by test-time EI
adaptation (Algorithm 2 with the network taken as the identity, so the
adapted quantity is the image itself): x starts at FBP(y) and takes `iters`
gradient steps x <- x - eta * grad L(x) on the sketched EI loss, a new
interleaved sketch S_k (k = iteration mod ratio, Sec. 4.2.1) and a new set
of rotations per iteration.

Scheduling.  Jobs arrive over time; a job is admitted (FIFO) as soon as it
has arrived, a slot is free and its device footprint fits in the HBM budget
beside the jobs already running.  Each server iteration runs ONE step of
every admitted job: the GPU executor batches them into one EI plan (one
launch per stage for all jobs, skei_ei_plan_run with the gradient step fused
into the last kernel), so jobs that arrive while others run join the next
iteration and their work overlaps on the device.  Finished jobs leave and
free their memory.  A job's results depend only on its own inputs and
iteration count -- the plan computes every problem bitwise as it would alone
-- so a job gives the same answer alone and in any mix.

The scheduler (``Server``) is device-agnostic: it talks to an executor
(footprint / start / step / finish) and a clock (now / sleep_until), so its
logic is tested on the CPU with fakes.
"""
from __future__ import annotations

import ctypes
import itertools
import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Job:
    spec: dict
    arrival: float
    footprint: int
    it: int = 0
    admitted: float | None = None
    finished: float | None = None
    state: object = None
    result: object = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class WallClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def sleep_until(self, t: float):
        dt = t - self.now()
        if dt > 0:
            time.sleep(dt)


@dataclass
class ServeReport:
    done: list
    rejected: list
    iterations: int
    max_active: int
    peak_bytes: int
    makespan: float
    batch_sizes: list = field(default_factory=list)

    def latencies(self) -> np.ndarray:
        return np.array([j.latency for j in self.done], dtype=np.float64)

    def percentile(self, q: float) -> float:
        lat = self.latencies()
        return float(np.percentile(lat, q)) if lat.size else math.nan


class Server:
    """FIFO admission under a device-memory budget and a slot limit;
    continuous batching: every step advances every admitted job (by one
    iteration, or by the counts the executor's step returns)."""

    def __init__(self, executor, budget_bytes: int, max_active: int = 64, clock=None):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.clock = clock or WallClock()

    def run(self, specs) -> ServeReport:
        pending = deque(Job(s, float(s["arrival"]), int(self.ex.footprint(s)))
                        for s in sorted(specs, key=lambda s: (s["arrival"], s["job"])))
        active: list[Job] = []
        done, rejected, sizes = [], [], []
        used = peak = 0
        iters = 0
        start = self.clock.now()
        while pending or active:
            now = self.clock.now()
            while pending and pending[0].arrival <= now:
                j = pending[0]
                if j.footprint > self.budget:          # can never fit
                    rejected.append(pending.popleft())
                    continue
                if len(active) >= self.max_active or used + j.footprint > self.budget:
                    break                                # head of line waits
                pending.popleft()
                j.admitted = now
                j.state = self.ex.start(j.spec)
                used += j.footprint
                peak = max(peak, used)
                active.append(j)
            if not active:
                if pending:
                    self.clock.sleep_until(pending[0].arrival)
                continue
            done_its = self.ex.step([j.state for j in active])
            iters += 1
            sizes.append(len(active))
            now = self.clock.now()
            still = []
            for k, j in enumerate(active):
                j.it += 1 if done_its is None else int(done_its[k])
                if j.it >= j.spec["iters"]:
                    j.finished = now
                    j.result = self.ex.finish(j.state)
                    j.state = None
                    used -= j.footprint
                    done.append(j)
                else:
                    still.append(j)
            active = still
        return ServeReport(done, rejected, iters, self.max_active, peak, self.clock.now() - start, sizes)


def step_size(n: int, n_angles_mc: int, lam: float) -> float:
    """A gradient step below 1/L for the EI loss: the MC term's Hessian
    2 A^T A has norm <= 2 ||A||_1 ||A||_inf <= 2 (1.5 N_theta)(sqrt(2) N)
    (Joseph columns sum to <= ~1.5 per angle, rows to <= sqrt(2) N), and the
    EI term adds at most ~20 lambda."""
    return 1.0 / (2.0 * 1.5 * math.sqrt(2.0) * n * n_angles_mc + 20.0 * lam)


def iteration_cost(spec) -> float:
    """Relative device cost of one iteration of a job: ray-lines of its
    projector work (A on the full scan, A_S on every copy, forward and
    transpose) -- every operator of the step scales alike."""
    return float((spec["n_angles"] + spec["copies"] * spec["m"]) * spec["n_det"] * spec["n"])


def executor_share(batched: bool, fair: bool | None = None, share: float | None = None) -> float:
    """The per-step share of GpuExecutor (see there): `share` if given, else
    1 / 0 for fair=True / False, else 0.25 batched and 0 per call."""
    if share is None:
        share = (0.25 if batched else 0.0) if fair is None else (1.0 if fair else 0.0)
    if not share >= 0.0:
        raise ValueError("share must be >= 0")
    return float(share)


class GpuExecutor:
    """Runs jobs on the device through the library.

    batched=True : the admitted jobs run as batched EI plans -- one launch per
                   stage for a whole class of jobs.
    batched=False: the per-call baseline -- each job has its own one-problem
                   plan and the jobs' iterations run one after another.
    share        : device time a cheap job may take per step, as a fraction of
                   one iteration of the costliest active job.  A job whose
                   iteration costs c runs max(1, floor(share * c_max / c))
                   iterations in the step (capped by what it has left), so
                   cheap jobs are not paced by expensive ones; jobs with equal
                   repetitions and image and detector sizes form one class
                   (one plan, whose launches share one shape).  share = 0 runs one
                   iteration of every job per step (round robin, one plan when
                   batched); share = 1 gives every cost class about the same
                   device time per step.  Larger shares finish cheap jobs
                   sooner (lower median latency) and slow the costliest ones
                   (higher tail latency).  Default: 0.25 batched, 0 per call.
                   `fair` is the older switch: True = share 1, False = share 0.
    Each job owns its scratch (allocated at admission and counted in its
    footprint), so rebuilding a plan allocates only its small work table.
    Inputs (the measured sinograms) are made once by ``prepare`` and kept in
    pinned host memory; ``start`` copies a job's sinogram to the device and
    forms x = FBP(y) there, as a server ingesting a request would.
    """

    def __init__(self, batched: bool = True, fair: bool | None = None, lam: float = 1.0,
                 record_loss: bool = False, share: float | None = None):
        import torch

        from . import ops
        self.torch, self.ops = torch, ops
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.batched = batched
        self.share = executor_share(batched, fair, share)
        self.lam = float(lam)
        self.record_loss = record_loss
        self.geoms = {}
        self.host_y = {}
        self._plans = {}                  # member tokens -> plan, least recently used first
        self.max_plans = 64
        self._tokens = itertools.count()
        self.plan_builds = 0

    # ---------------------------------------------------------------- inputs
    def geometry(self, spec):
        key = (spec["n"], spec["n_angles"], spec["n_det"])
        if key not in self.geoms:
            self.geoms[key] = self.ops.Geometry(*key, device=self.dev)
        return self.geoms[key]

    def prepare(self, specs):
        """Measured sinograms y = A x_true + 1 % noise of each job (device
        forward projection of its seeded phantom), kept in pinned host memory."""
        from . import synth
        torch = self.torch
        for s in specs:
            g = self.geometry(s)
            xt = torch.from_numpy(synth.ellipse_phantom(s["n"], s["phantom_seed"])[None]).to(self.dev)
            y = self.ops.radon_fwd_(g, xt, g.full())
            z = torch.from_numpy(synth.std_noise(tuple(y.shape), s["noise_seed"])).to(self.dev, torch.float32)
            y = (y + 0.01 * y.max() * z).contiguous()
            self.host_y[s["job"]] = y.cpu().pin_memory()
        torch.cuda.synchronize()

    def footprint(self, spec) -> int:
        from . import capi
        g = self.geometry(spec)
        n, na, nd, m, c = spec["n"], spec["n_angles"], spec["n_det"], spec["m"], spec["copies"]
        fake = 256   # sizes only: the query reads no memory
        rec = capi.EiProblem(g.handle.value, 1, fake, fake, fake, na, fake, m, c, fake, self.lam, fake, fake, 0.0,
                             None, 0)
        ws = int(capi.query("skei_ei_problem_workspace_bytes", ctypes.byref(rec)))
        own = 4 * (3 * n * n + na * nd + spec["ratio"] * m + spec["iters"] * c * 2 + m + 2 * c) + 8 * spec["iters"]
        return ws + own

    # ------------------------------------------------------------ lifecycle
    def start(self, spec):
        from . import ei, synth
        torch, ops = self.torch, self.ops
        g = self.geometry(spec)
        y = self.host_y[spec["job"]].to(self.dev, non_blocking=True)
        x = ops.fbp_(g, y, g.full()).contiguous()
        na, ratio, m = spec["n_angles"], spec["ratio"], spec["m"]
        subsets = np.stack([k + ratio * np.arange(m) for k in range(ratio)]).astype(np.int32)
        st = _JobState()
        st.token = next(self._tokens)   # stable identity for the plan cache (never reused)
        st.spec = spec
        st.cost = iteration_cost(spec)
        st.sk_table = torch.from_numpy(subsets).to(self.dev)
        phis = synth.rotation_angles(spec["iters"] * spec["copies"], spec["rotation_seed"])
        st.cs_table = torch.from_numpy(synth.cos_sin(phis).reshape(spec["iters"], spec["copies"], 2)).to(
            self.dev, torch.float32)
        st.sketch = g.sketch(subsets[0])
        st.cs = st.cs_table[0].clone()
        st.it = 0
        st.eta = step_size(spec["n"], na, self.lam)
        st.problem = ei.EIProblem(g, x, y, st.sketch, st.cs, self.lam, grad=True, step=st.eta, own_workspace=True)
        st.loss = torch.zeros(spec["iters"], dtype=torch.float64, device=self.dev) if self.record_loss else None
        return st

    def _inputs(self, st):
        # this iteration's sketch S_k (k = it mod ratio) and rotations
        st.sketch.dev.copy_(st.sk_table[st.it % st.spec["ratio"]])
        st.cs.copy_(st.cs_table[st.it])

    def _plan(self, members):
        """The plan of a class of jobs, cached under the members' tokens (a
        token is drawn once per job and never reused, so a cached plan is
        only ever bound to the problems of exactly these jobs)."""
        from . import ei
        key = tuple(st.token for st in members)
        plan = self._plans.pop(key, None)
        if plan is None:
            plan = ei.EIPlan([st.problem for st in members])
            self.plan_builds += 1
        self._plans[key] = plan           # most recently used last
        return key, plan

    def _run(self, members, reps):
        key, plan = self._plan(members)
        for _ in range(reps):
            for st in members:
                self._inputs(st)
            plan.run()
            for i, st in enumerate(members):
                if self.record_loss:
                    st.loss[st.it].copy_(plan.losses[i])
                st.it += 1
        return key

    def step(self, states):
        """Runs the step; returns the iterations each job advanced."""
        if self.share > 0:
            cmax = max(st.cost for st in states)
            reps = [max(1, min(int(self.share * cmax // st.cost), st.spec["iters"] - st.it)) for st in states]
        else:
            reps = [1] * len(states)
        if any(st.it + r > st.spec["iters"] for st, r in zip(states, reps)):
            raise RuntimeError("a job was stepped past its iterations")
        if self.batched:
            # a class shares every launch of a plan, and a launch takes one
            # shape for all its jobs (rays per thread from the widest detector
            # row, ...): only jobs of one geometry size share a class
            classes = {}
            for st, r in zip(states, reps):
                classes.setdefault((r, st.spec["n"], st.spec["n_det"]), []).append(st)
            for key in sorted(classes, reverse=True):
                self._run(classes[key], key[0])
        else:
            for st, r in zip(states, reps):
                self._run([st], r)
        # A class plan stays cached while all its members are active (class
        # membership changes as repetition counts shift, and recurs); plans
        # with a member that has left, and the least recently used beyond
        # the cache size, free their tables.
        active = {st.token for st in states}
        for key in [k for k in self._plans if not active.issuperset(k)]:
            self._plans.pop(key).close()
        while len(self._plans) > self.max_plans:
            self._plans.pop(next(iter(self._plans))).close()
        self.torch.cuda.synchronize()
        return reps

    def finish(self, st):
        return {"x": st.problem.x.clone(), "loss": st.loss}

    def close(self):
        for plan in self._plans.values():
            plan.close()
        self._plans.clear()


class _JobState:
    pass


def job_rays(spec) -> float:
    """Projector rays one iteration of a job evaluates: A on the full scan
    and A_S on every copy, forward and adjoint."""
    return 2.0 * (spec["n_angles"] + spec["copies"] * spec["m"]) * spec["n_det"] * spec["iters"]

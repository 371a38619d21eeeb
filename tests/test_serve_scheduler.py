"""Host logic of the continuous-batching server (paper_2411_05771_amd.serve),
with a fake clock and a fake executor: admission under the memory budget and
the slot limit, FIFO order, continuous batching (jobs join between
iterations), completion after exactly `iters` steps, rejection of jobs that
can never fit, and idle gaps."""
import pytest

from paper_2411_05771_amd import serve, synth


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep_until(self, t):
        self.t = max(self.t, t)


class FakeExecutor:
    """Step time = base + per-job cost (batching amortises `base`)."""

    def __init__(self, clock, budget, base=1.0, per_job=0.25):
        self.clock, self.budget = clock, budget
        self.base, self.per_job = base, per_job
        self.steps = []          # (time, [job ids]) per step
        self.started, self.finished = [], []
        self.active = {}

    def footprint(self, spec):
        return spec["bytes"]

    def start(self, spec):
        self.started.append((self.clock.now(), spec["job"]))
        self.active[spec["job"]] = spec
        assert sum(s["bytes"] for s in self.active.values()) <= self.budget
        return {"job": spec["job"], "it": 0}

    def step(self, states):
        self.steps.append((self.clock.now(), [s["job"] for s in states]))
        for s in states:
            s["it"] += 1
        self.clock.t += self.base + self.per_job * len(states)

    def finish(self, state):
        self.finished.append((self.clock.now(), state["job"]))
        del self.active[state["job"]]
        return state["it"]


def jobs(arrivals, sizes, iters=3):
    return [dict(job=i, arrival=a, bytes=b, iters=iters) for i, (a, b) in enumerate(zip(arrivals, sizes))]


def run(specs, budget, max_active=64, **kw):
    clock = FakeClock()
    ex = FakeExecutor(clock, budget, **kw)
    rep = serve.Server(ex, budget, max_active=max_active, clock=clock).run(specs)
    return rep, ex


def test_every_job_runs_exactly_its_iterations():
    specs = jobs([0.0, 0.1, 0.2, 5.0], [10, 10, 10, 10], iters=4)
    rep, ex = run(specs, budget=100)
    assert sorted(j.spec["job"] for j in rep.done) == [0, 1, 2, 3]
    assert all(j.result == 4 for j in rep.done)
    for j in rep.done:
        assert sum(j.spec["job"] in ids for _, ids in ex.steps) == 4
        assert j.finished > j.arrival and j.latency > 0


def test_continuous_batching_admits_between_iterations():
    # job 1 arrives while job 0's first step runs (0 .. 1.25): it joins at the next step
    specs = jobs([0.0, 0.5], [10, 10], iters=3)
    rep, ex = run(specs, budget=100)
    assert ex.steps[0][1] == [0]
    assert ex.steps[1][1] == [0, 1]
    admitted = {j.spec["job"]: j.admitted for j in rep.done}
    assert admitted[1] == pytest.approx(ex.steps[1][0])
    assert max(len(ids) for _, ids in ex.steps) == 2


def test_budget_and_fifo_head_of_line():
    # job 1 (60) does not fit beside job 0 (50) in 100: it waits, and job 2
    # (10, which would fit) waits behind it -- FIFO
    specs = jobs([0.0, 0.1, 0.2], [50, 60, 10], iters=2)
    rep, ex = run(specs, budget=100)
    order = [jid for _, jid in ex.started]
    assert order == [0, 1, 2]
    t_start = dict((jid, t) for t, jid in ex.started)
    t_fin = dict((jid, t) for t, jid in ex.finished)
    assert t_start[1] >= t_fin[0]
    assert t_start[2] >= t_start[1]
    assert rep.peak_bytes <= 100


def test_slot_limit():
    specs = jobs([0.0] * 6, [1] * 6, iters=2)
    rep, ex = run(specs, budget=100, max_active=2)
    assert max(len(ids) for _, ids in ex.steps) == 2
    assert len(rep.done) == 6


def test_job_larger_than_budget_is_rejected():
    specs = jobs([0.0, 0.0], [500, 10], iters=2)
    rep, ex = run(specs, budget=100)
    assert [j.spec["job"] for j in rep.rejected] == [0]
    assert [j.spec["job"] for j in rep.done] == [1]


def test_idle_gap_jumps_to_next_arrival():
    specs = jobs([0.0, 100.0], [10, 10], iters=1)
    rep, ex = run(specs, budget=100)
    assert ex.steps[1][0] == pytest.approx(100.0)
    lat = sorted(j.latency for j in rep.done)
    assert lat[0] == pytest.approx(1.25) and lat[1] == pytest.approx(1.25)


def test_batching_beats_one_at_a_time_under_load():
    specs = jobs([0.1 * i for i in range(8)], [10] * 8, iters=5)
    batched, _ = run(specs, budget=1000)
    serial, _ = run(specs, budget=1000, max_active=1)
    assert batched.percentile(50) < serial.percentile(50)
    assert batched.makespan < serial.makespan


def test_poisson_job_stream_is_seeded_and_shaped():
    a = synth.poisson_jobs(40, rate=2.0)
    b = synth.poisson_jobs(40, rate=2.0)
    assert a == b
    assert a[0]["arrival"] == 0.0
    assert all(a[i]["arrival"] < a[i + 1]["arrival"] for i in range(39))
    for s in a:
        assert s["n"] in (256, 512, 1024) and 180 <= s["n_angles"] <= 1440 and s["ratio"] in (2, 4, 8)
        assert s["m"] == s["n_angles"] // s["ratio"]
        assert s["ratio"] * (s["m"] - 1) + s["ratio"] - 1 < s["n_angles"]   # every interleaved subset fits
    gaps = [a[i + 1]["arrival"] - a[i]["arrival"] for i in range(39)]
    assert 0.2 < sum(gaps) / len(gaps) < 1.0     # mean gap ~ 1 / rate


def test_step_size_is_below_the_curvature_bound():
    # eta L_MC < 1 for the bound 2 ||A||_1 ||A||_inf with Joseph row/column sums
    for n, na in ((64, 60), (256, 360), (1024, 1440)):
        eta = serve.step_size(n, na, 1.0)
        assert eta * 2 * (1.5 * na) * (2 ** 0.5 * n) < 1.0


class UnevenExecutor(FakeExecutor):
    """Advances job 0 by two iterations per step (as a fair executor does for
    a job whose iterations cost half as much)."""

    def step(self, states):
        super().step(states)
        return [min(2, s["iters_left"]) if s["job"] == 0 else 1 for s in states]

    def start(self, spec):
        st = super().start(spec)
        st["iters_left"] = spec["iters"]
        return st


def test_executor_may_advance_jobs_by_several_iterations():
    clock = FakeClock()
    ex = UnevenExecutor(clock, 100)
    specs = jobs([0.0, 0.0], [10, 10], iters=4)
    rep = serve.Server(ex, 100, clock=clock).run(specs)
    steps_of = {j.spec["job"]: sum(j.spec["job"] in ids for _, ids in ex.steps) for j in rep.done}
    assert steps_of == {0: 2, 1: 4}
    assert rep.done[0].spec["job"] == 0 and rep.done[0].finished < rep.done[1].finished


# ------------------------------------------------------------------ GpuExecutor plan cache
class _FakePlan:
    """Stands in for ei.EIPlan: records which problems every run computes."""

    def __init__(self, problems):
        self.problems = list(problems)
        self.runs = []
        self.closed = False

    def run(self):
        self.runs.append(list(self.problems))

    def close(self):
        self.closed = True


def _host_executor(monkeypatch, batched=True, share=0.0):
    """A GpuExecutor whose device parts (torch sync, plans, per-iteration
    input copies) are replaced by host fakes; step() and the plan cache are
    the real ones."""
    import itertools
    import types

    from paper_2411_05771_amd import ei
    monkeypatch.setattr(ei, "EIPlan", _FakePlan)
    ex = object.__new__(serve.GpuExecutor)
    ex.batched, ex.share, ex.record_loss = batched, share, False
    ex._plans, ex._tokens, ex.plan_builds, ex.max_plans = {}, itertools.count(), 0, 64
    ex.torch = types.SimpleNamespace(cuda=types.SimpleNamespace(synchronize=lambda: None))
    ex._inputs = lambda st: None
    return ex


def _state(ex, iters=1, cost=1.0, n=64, n_det=91):
    st = serve._JobState()
    st.token = next(ex._tokens)          # as GpuExecutor.start draws it
    st.problem = object()
    st.spec = {"iters": iters, "n": n, "n_det": n_det}
    st.it = 0
    st.cost = cost
    return st


def test_plan_cache_never_serves_a_finished_jobs_plan(monkeypatch):
    """A job finishes and a new one-member class is admitted at the next step.
    CPython may give the new job's state the finished state's address; the
    cached plan must still never be the finished job's (it would compute the
    finished job's problem and leave the new job's image untouched)."""
    ex = _host_executor(monkeypatch)
    first = _state(ex)
    ex.step([first])
    old_id = id(first)
    del first                             # the server drops a finished job's state
    keep, new = [], None
    for _ in range(1000):                 # try to land a new state on the freed address
        st = _state(ex)
        if id(st) == old_id:
            new = st
            break
        keep.append(st)
    new = new if new is not None else _state(ex)
    ex.step([new])
    runs = [r for plan in ex._plans.values() for r in plan.runs]
    assert runs and runs[-1] == [new.problem], "the new job ran another job's plan"


def test_per_call_executor_honours_fair_repetitions(monkeypatch):
    """batched=False with share 1: each job runs as many iterations as the
    step reports for it."""
    ex = _host_executor(monkeypatch, batched=False, share=1.0)
    cheap, dear = _state(ex, iters=10, cost=1.0), _state(ex, iters=10, cost=4.0)
    reps = ex.step([cheap, dear])
    assert reps == [4, 1]
    assert cheap.it == 4 and dear.it == 1


@pytest.mark.parametrize("share,want", [(0.0, [1, 1, 1]), (0.25, [2, 1, 1]), (0.5, [4, 2, 1]), (1.0, [8, 4, 1])])
def test_share_sets_the_repetitions_of_cheap_jobs(monkeypatch, share, want):
    """A job of iteration cost c runs max(1, floor(share * c_max / c))
    iterations per step, capped by what it has left; equal repetitions form
    one class (one plan run per repetition)."""
    ex = _host_executor(monkeypatch, batched=True, share=share)
    sts = [_state(ex, iters=10, cost=1.0), _state(ex, iters=10, cost=2.0), _state(ex, iters=10, cost=8.0)]
    assert ex.step(sts) == want
    assert [st.it for st in sts] == want
    runs = sorted(len(plan.runs) for plan in ex._plans.values())
    assert sum(runs) == sum(sorted(set(want)))
    left = _state(ex, iters=1, cost=1.0)              # capped by what it has left
    assert ex.step([left, _state(ex, iters=10, cost=8.0)])[0] == 1


def test_executor_share_defaults():
    assert serve.executor_share(True) == 0.25
    assert serve.executor_share(False) == 0.0
    assert serve.executor_share(True, fair=True) == 1.0
    assert serve.executor_share(True, fair=False) == 0.0
    assert serve.executor_share(False, share=0.5) == 0.5
    with pytest.raises(ValueError):
        serve.executor_share(True, share=-1.0)


def test_class_plans_are_kept_while_their_members_run(monkeypatch):
    """Repetition classes regroup as jobs near their end; a class plan is kept
    while all its members are active (no rebuild when the class recurs) and
    closed once a member has left; the cache holds at most max_plans plans."""
    ex = _host_executor(monkeypatch, batched=True, share=1.0)
    a, b = _state(ex, iters=3, cost=1.0), _state(ex, iters=10, cost=2.0)
    assert ex.step([a, b]) == [2, 1]          # classes (a,) x2 and (b,) x1
    assert ex.step([a, b]) == [1, 1]          # a has one left: class (a, b)
    assert ex.plan_builds == 3
    kept = dict(ex._plans)
    assert set(kept) == {(a.token,), (b.token,), (a.token, b.token)}
    ex.step([b])                              # a has finished
    assert ex.plan_builds == 3                # (b,) served from the cache
    assert all(p.closed for k, p in kept.items() if a.token in k)
    assert list(ex._plans) == [(b.token,)]
    ex.max_plans = 1
    c = _state(ex, iters=10, cost=2.0)
    ex.step([b, c])
    assert len(ex._plans) == 1


def test_classes_hold_one_geometry_size(monkeypatch):
    """Jobs of different image or detector sizes never share a plan (its
    launches take one shape); equal sizes and repetitions do."""
    ex = _host_executor(monkeypatch, batched=True, share=0.0)
    a, b = _state(ex, iters=5, n=64, n_det=91), _state(ex, iters=5, n=64, n_det=91)
    c = _state(ex, iters=5, n=128, n_det=182)
    ex.step([a, b, c])
    assert sorted(len(k) for k in ex._plans) == [1, 2]
    assert (c.token,) in ex._plans and (a.token, b.token) in ex._plans

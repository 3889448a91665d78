"""Host-only checks of the continuous-batching scheduler with a stand-in backend."""
import dataclasses

import numpy as np

from paper_2405_13973_amd import inputs, serving


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, s):
        self.t += s


class FakeCrystal:
    def __init__(self, log, n):
        self.n, self.log, self.steps = n, log, 0
        self.alive = True

    def set_trap(self, **k):
        pass

    def set_laser(self, *a):
        pass

    def set_force(self, *a):
        pass

    def read_state(self):
        return dict(pos=np.zeros((self.n, 3)), vel=np.zeros((self.n, 3)), photons=np.zeros(self.n, np.int32),
                    step=self.steps)

    def destroy(self):
        self.alive = False


class FakeNative:
    PT_ENOMEM = -2

    class PTError(RuntimeError):
        def __init__(self, code):
            super().__init__(code)
            self.code = code

    def __init__(self, clock, sec_per_ion_step, ctx=None):
        self.clock, self.rate = clock, sec_per_ion_step
        self.calls = []
        self.ctx = ctx

    def step_batch(self, cs, n):
        if self.ctx is not None:  # the batch workspace grows to the batch, never shrinks
            need = max(self.ctx.ws, int(self.ctx.ws_per_ion * sum(c.n for c in cs)))
            live = self.ctx.memory()[0] - self.ctx.ws
            if self.ctx.hard_budget and live + need > self.ctx.hard_budget:
                raise self.PTError(self.PT_ENOMEM)  # nothing stepped, as in the library
            self.ctx.ws = need
        self.calls.append([(c.n, k) for c, k in zip(cs, n)])
        for c, k in zip(cs, n):
            c.steps += k
        # time advances with the work of the longest crystal in the batch
        self.clock.t += self.rate * sum(c.n * k for c, k in zip(cs, n))

    def rotating_diagnostics_batch(self, cs):
        self.diag_calls = getattr(self, "diag_calls", []) + [[c.n for c in cs]]
        return [dict(energy=float(c.n), steps=c.steps) for c in cs]


class FakeCtx:
    """Device memory as the library counts it: each live crystal's state plus a
    grow-only batch workspace of ws_per_ion bytes per ion of the largest batch."""

    def __init__(self, ws_per_ion=300.0, hard_budget=0):
        self.created = []
        self.ws, self.ws_per_ion = 0, ws_per_ion
        self.hard_budget = hard_budget

    def crystal(self, pos, vel, q, m, seed):
        c = FakeCrystal(None, len(pos))
        self.created.append(c)
        return c

    def synchronize(self):
        pass

    def memory(self):
        live = sum(serving.state_bytes(c.n) for c in self.created if c.alive)
        return live + self.ws, 0


def _reqs(ns, ks, arrivals):
    out = []
    for n, k, a in zip(ns, ks, arrivals):
        pos = np.zeros((n, 3))
        out.append(inputs.Request(a, inputs.Crystal(pos, pos.copy()), k))
    return out


def test_all_requests_complete_with_their_steps():
    clk = FakeClock()
    nat = FakeNative(clk, 1e-9)
    ctx = FakeCtx()
    reqs = _reqs([100, 2000, 500, 50], [120, 35, 60, 10], [0.0, 0.0, 0.01, 0.5])
    rep = serving.Server(ctx, nat, budget_bytes=1 << 40, chunk=25, clock=clk, sleep=clk.sleep).run(reqs)
    assert sorted(d.index for d in rep.done) == [0, 1, 2, 3]
    for c, r in zip(ctx.created, sorted(reqs, key=lambda r: r.arrival_s)):
        pass
    assert all(not c.alive for c in ctx.created)
    assert sum(c.steps for c in ctx.created) == 120 + 35 + 60 + 10
    assert rep.ion_steps == 100 * 120 + 2000 * 35 + 500 * 60 + 50 * 10
    for d in rep.done:
        assert d.finish_s >= d.admit_s >= d.arrival_s - 1e-12
    # every call steps each resident crystal by at most the chunk
    assert all(k <= 25 for call in nat.calls for _, k in call)
    # continuous batching: requests arriving while others run share calls
    assert any(len(call) > 1 for call in nat.calls)
    # each request's end-of-run diagnostics come from one batched call per tick,
    # taken after its last steps
    assert sorted(n for call in nat.diag_calls for n in call) == sorted(d.n_ions for d in rep.done)
    for d in rep.done:
        assert d.diagnostics["energy"] == d.n_ions and d.diagnostics["steps"] == d.steps


def test_admission_waits_for_memory():
    clk = FakeClock()
    nat = FakeNative(clk, 1e-9)
    ctx = FakeCtx()
    nat.ctx = ctx
    n = 10000
    budget = serving.footprint(n) + serving.footprint(n) // 2  # room for one crystal at a time
    reqs = _reqs([n, n, n], [30, 30, 30], [0.0, 0.0, 0.0])
    rep = serving.Server(ctx, nat, budget_bytes=budget, chunk=10, clock=clk, sleep=clk.sleep).run(reqs)
    assert rep.max_resident == 1
    assert rep.max_resident_bytes <= budget
    assert len(rep.done) == 3
    fin = sorted(d.finish_s for d in rep.done)
    assert fin[0] < fin[1] < fin[2]


def test_latency_percentiles():
    clk = FakeClock()
    nat = FakeNative(clk, 1e-9)
    reqs = _reqs([300] * 5, [40] * 5, [0.0, 0.1, 0.2, 0.3, 0.4])
    rep = serving.Server(FakeCtx(), nat, budget_bytes=1 << 40, chunk=20, clock=clk, sleep=clk.sleep).run(reqs)
    p50, p99 = rep.latency_percentiles()
    assert 0 < p50 <= p99
    assert rep.ion_steps_per_s > 0


def test_footprint_grows_with_smaller_leaves_and_higher_degree():
    """More boxes per ion (small leaves) and longer expansions (high p, FP64)
    take more workspace per ion."""
    f = serving.workspace_bytes_per_ion
    assert f(11, 32, "mixed") > f(11, 384, "mixed")
    assert f(12, 64, "mixed") > f(8, 64, "mixed")
    assert f(11, 64, "fp64") > f(11, 64, "mixed")
    assert serving.footprint(1000, 11, 32) > serving.state_bytes(1000)


def test_admission_learns_the_measured_workspace():
    """When the batch workspace per ion is larger than the estimate, the server
    raises its rate to the measured one after the first tick and still keeps the
    memory it uses within the budget."""
    clk = FakeClock()
    ctx = FakeCtx(ws_per_ion=3 * serving.workspace_bytes_per_ion(11, 32, "mixed"))
    nat = FakeNative(clk, 1e-9, ctx)
    n = 4000
    per = serving.state_bytes(n) + ctx.ws_per_ion * n
    budget = int(2.5 * per)  # two such requests fit, three do not
    reqs = _reqs([n] * 6, [20] * 6, [0.0, 0.0, 0.001, 0.001, 0.002, 0.002])
    srv = serving.Server(ctx, nat, budget_bytes=budget, chunk=5, clock=clk, sleep=clk.sleep)
    rep = srv.run(reqs)
    assert len(rep.done) == 6
    assert srv.ws_rate >= ctx.ws_per_ion * 0.999
    assert rep.max_resident_bytes <= budget


def test_out_of_memory_tick_requeues_the_newest_request():
    """The context's own budget is the hard limit: when the workspace outgrows the
    estimate so that a tick fails with PT_ENOMEM, the newest request that has not
    stepped goes back to the head of the queue and every request still completes,
    without the memory in use ever passing the budget."""
    clk = FakeClock()
    n = 4000
    true_rate = 4 * serving.workspace_bytes_per_ion(11, 32, "mixed")
    budget = int(2.5 * (serving.state_bytes(n) + true_rate * n))
    ctx = FakeCtx(ws_per_ion=true_rate, hard_budget=budget)
    nat = FakeNative(clk, 1e-9, ctx)
    reqs = _reqs([n] * 5, [20] * 5, [0.0] * 5)
    srv = serving.Server(ctx, nat, budget_bytes=budget, chunk=5, clock=clk, sleep=clk.sleep)
    rep = srv.run(reqs)
    assert sorted(d.index for d in rep.done) == list(range(5))
    assert all(d.steps == 20 for d in rep.done)
    assert srv.requeued >= 1
    assert rep.max_resident_bytes <= budget
    assert rep.ion_steps == 5 * 20 * n

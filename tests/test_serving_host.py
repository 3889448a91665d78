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
        code = 0

    def __init__(self, clock, sec_per_ion_step):
        self.clock, self.rate = clock, sec_per_ion_step
        self.calls = []

    def step_batch(self, cs, n):
        self.calls.append([(c.n, k) for c, k in zip(cs, n)])
        for c, k in zip(cs, n):
            c.steps += k
        # time advances with the work of the longest crystal in the batch
        self.clock.t += self.rate * sum(c.n * k for c, k in zip(cs, n))

    def rotating_diagnostics_batch(self, cs):
        self.diag_calls = getattr(self, "diag_calls", []) + [[c.n for c in cs]]
        return [dict(energy=float(c.n), steps=c.steps) for c in cs]


class FakeCtx:
    def __init__(self):
        self.created = []

    def crystal(self, pos, vel, q, m, seed):
        c = FakeCrystal(None, len(pos))
        self.created.append(c)
        return c

    def synchronize(self):
        pass


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

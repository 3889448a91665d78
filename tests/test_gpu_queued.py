"""Queued FMM steps (no host wait per step) against steps that measure their
tree every time, and against runs whose capacities are forced one box short
so that every queued step overflows, halts on the device and is run again
from the last completed step: all three give the same states bit for bit, in
both precisions, for a single crystal and for a batch whose crystals stop at
different steps."""
import numpy as np
import pytest

from paper_2405_13973_amd import inputs, native

pytestmark = pytest.mark.gpu


def _run(monkeypatch, env, crs, steps, precision, leaf):
    for k in ("PT_QUEUED_STEPS", "PT_CAPS_TIGHT", "PT_PARTIAL_SORT"):
        monkeypatch.delenv(k, raising=False)
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    with native.Context(0) as ctx:
        cs = []
        for cr in crs:
            c = ctx.crystal(cr.pos, cr.vel, cr.charge, cr.mass, cr.seed)
            c.set_trap(B=cr.B, omega_z=cr.omega_z, dt=cr.dt)
            c.set_laser(cr.photon_mean)
            c.set_force("fmm", 10, leaf, precision)
            cs.append(c)
        native.step_batch(cs, steps)
        ctx.synchronize()
        # a second call on the same batch: its steps are queued from the first
        native.step_batch(cs, [k // 2 for k in steps])
        out = [c.read_state() for c in cs]
        stats = ctx.step_stats()
    return out, stats


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_queued_measured_and_rerun_steps_agree(monkeypatch, precision):
    crs = inputs.ensemble(count=4, seed=71, n_lo=3000, n_hi=20000)
    steps = [9, 4, 9, 6]
    print(f"queued steps {precision}", flush=True)
    ref, s_meas = _run(monkeypatch, {"PT_QUEUED_STEPS": "0"}, crs, steps, precision, 48)
    got, s_q = _run(monkeypatch, {}, crs, steps, precision, 48)
    tight, s_t = _run(monkeypatch, {"PT_CAPS_TIGHT": "1"}, crs, steps, precision, 48)
    assert s_meas["queued"] == 0 and s_meas["reruns"] == 0
    assert s_q["queued"] > 0 and s_q["reruns"] == 0
    assert s_t["reruns"] > 0
    for a, b, c, k in zip(ref, got, tight, steps):
        assert a["step"] == b["step"] == c["step"] == k + k // 2
        for key in ("pos", "vel", "photons"):
            assert np.array_equal(a[key], b[key]), key
            assert np.array_equal(a[key], c[key]), key


def test_queued_steps_at_full_size(monkeypatch):
    """The benchmark crystal (N = 1e5, p = 11, leaf 256): 12 queued steps equal 12
    measured ones bit for bit."""
    cr = inputs.config3()
    print("queued steps N=1e5", flush=True)
    res = []
    for env in ({"PT_QUEUED_STEPS": "0"}, {}):
        for k in ("PT_QUEUED_STEPS", "PT_CAPS_TIGHT"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        with native.Context(0) as ctx:
            c = ctx.crystal(cr.pos, cr.vel, cr.charge, cr.mass, cr.seed)
            c.set_force("fmm", 11, 256, "mixed")
            c.step(12)
            res.append((c.read_state(), ctx.step_stats()))
    (a, sa), (b, sb) = res
    assert sa["queued"] == 0 and sb["queued"] == 11
    assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["vel"], b["vel"])


def test_sort_refine_overflow_reruns_with_the_full_sort(monkeypatch):
    """Queued steps sort by the top Morton levels and order each run of equal
    top digits by (key, index).  A far outlier stretches the root cube so that
    the whole cluster shares a few cells at that level: the runs are too long,
    the queued step halts and is run again, later queued steps sort by more
    digits, and the states equal those of measured steps and of the full sort
    throughout."""
    g = inputs.rng(81)
    pos = inputs.uniform_ball(3000, 1e-4, g)
    pos[0] = (5e-2, 0.0, 0.0)
    vel = inputs.thermal_velocities(3000, 10e-3, inputs.ION_MASS, g)
    cr = inputs.Crystal(pos, vel, seed=81)
    print("sort refine overflow", flush=True)
    runs = {}
    for name, env in (("measured", {"PT_QUEUED_STEPS": "0"}), ("full", {"PT_PARTIAL_SORT": "0"}), ("partial", {})):
        for k in ("PT_QUEUED_STEPS", "PT_CAPS_TIGHT", "PT_PARTIAL_SORT"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        with native.Context(0) as ctx:
            c = ctx.crystal(cr.pos, cr.vel, cr.charge, cr.mass, cr.seed)
            c.set_trap(B=cr.B, omega_z=cr.omega_z, dt=cr.dt)
            c.set_force("fmm", 8, 48, "fp64")
            c.step(6)
            runs[name] = (c.read_state(), ctx.step_stats())
    (m, sm), (f, sf), (p, sp) = runs["measured"], runs["full"], runs["partial"]
    assert sm["queued"] == 0 and sp["reruns"] > sf["reruns"]
    for key in ("pos", "vel"):
        assert np.array_equal(m[key], f[key]) and np.array_equal(m[key], p[key]), key

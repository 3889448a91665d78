"""Batched forms on the GPU: an ensemble stepped together equals each crystal
stepped alone, and a request served in a mixed stream ends in the same state as
when run alone (bit for bit)."""
import numpy as np
import pytest

from paper_2405_13973_amd import inputs, native, serving

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = native.Context(0)
    yield c
    c.close()


def _make(ctx, cr, precision, p=8, leaf=24):
    c = ctx.crystal(cr.pos, cr.vel, cr.charge, cr.mass, cr.seed)
    c.set_trap(B=cr.B, omega_z=cr.omega_z, dt=cr.dt)
    c.set_laser(cr.photon_mean)
    c.set_force("fmm", p, leaf, precision)
    return c


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_ensemble_step_equals_alone(ctx, precision):
    crs = inputs.ensemble(count=6, seed=44, n_lo=100, n_hi=3000)
    steps = [7, 3, 7, 5, 1, 7]
    alone = []
    for cr, k in zip(crs, steps):
        c = _make(ctx, cr, precision)
        c.step(k)
        alone.append(c.read_state())
        c.destroy()
    cs = [_make(ctx, cr, precision) for cr in crs]
    native.step_batch(cs, steps)
    for c, a, k in zip(cs, alone, steps):
        st = c.read_state()
        assert st["step"] == k
        assert np.array_equal(st["pos"], a["pos"]) and np.array_equal(st["vel"], a["vel"])
        assert np.array_equal(st["photons"], a["photons"])
        c.destroy()


def test_serving_alone_equals_mix(ctx):
    reqs = inputs.serving_stream(count=5, rate_hz=200.0, seed=55, n_lo=200, n_hi=3000, k_lo=10, k_hi=40)
    srv = serving.Server(ctx, native, budget_bytes=8 << 30, precision="mixed", p=8, leaf=24, chunk=9)
    rep = srv.run(reqs)
    assert len(rep.done) == len(reqs)
    for d in rep.done:
        ref = serving.run_alone(ctx, native, reqs[d.index], precision="mixed", p=8, leaf=24)
        assert np.array_equal(d.pos, ref["pos"]) and np.array_equal(d.vel, ref["vel"])
        assert np.array_equal(d.photons, ref["photons"])

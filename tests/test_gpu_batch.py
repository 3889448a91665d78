"""Batched forms on the GPU: an ensemble stepped together equals each crystal
stepped alone, and a request served in a mixed stream ends in the same state as
when run alone (bit for bit); in FP64 both also end within the config-1 bars of
the CPU oracle's run of each crystal (positions 1e-10, velocities 1e-8 of their
rms: the per-step force parity is 1e-11 and a few steps stay far inside the
crystals' divergence time)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
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
    for c, a, k, cr in zip(cs, alone, steps, crs):
        st = c.read_state()
        assert st["step"] == k
        assert np.array_equal(st["pos"], a["pos"]) and np.array_equal(st["vel"], a["vel"])
        assert np.array_equal(st["photons"], a["photons"])
        c.destroy()
        if precision == "fp64":
            _against_oracle(st, cr, k, 8, 24)


def _rms(a):
    return math.sqrt((np.linalg.norm(a, axis=1) ** 2).mean())


def _against_oracle(st, cr, steps, p, leaf):
    x, v, ph = O.run(cr.pos, cr.vel, cr.charge, cr.mass, cr.trap(), cr.dt, steps, seed=cr.seed, laser=cr.laser(),
                     method="fmm", p=p, leaf_size=leaf, return_photons=True)
    dx = np.linalg.norm(st["pos"] - x, axis=1).max() / _rms(x)
    dv = np.linalg.norm(st["vel"] - v, axis=1).max() / _rms(v)
    assert dx <= 1e-10 and dv <= 1e-8, (dx, dv)
    assert np.array_equal(st["photons"], ph)


def test_served_fp64_requests_match_oracle(ctx):
    reqs = inputs.serving_stream(count=4, rate_hz=300.0, seed=56, n_lo=200, n_hi=2000, k_lo=4, k_hi=12)
    srv = serving.Server(ctx, native, budget_bytes=8 << 30, precision="fp64", p=8, leaf=24, chunk=5)
    rep = srv.run(reqs)
    assert len(rep.done) == len(reqs)
    for d in rep.done:
        r = reqs[d.index]
        _against_oracle({"pos": d.pos, "vel": d.vel, "photons": d.photons}, r.crystal, r.steps, 8, 24)


def test_serving_alone_equals_mix(ctx):
    reqs = inputs.serving_stream(count=5, rate_hz=200.0, seed=55, n_lo=200, n_hi=3000, k_lo=10, k_hi=40)
    srv = serving.Server(ctx, native, budget_bytes=8 << 30, precision="mixed", p=8, leaf=24, chunk=9)
    rep = srv.run(reqs)
    assert len(rep.done) == len(reqs)
    for d in rep.done:
        ref = serving.run_alone(ctx, native, reqs[d.index], precision="mixed", p=8, leaf=24)
        assert np.array_equal(d.pos, ref["pos"]) and np.array_equal(d.vel, ref["vel"])
        assert np.array_equal(d.photons, ref["photons"])

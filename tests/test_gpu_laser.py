"""Beam-mode laser (eqs. scattering_rate, laser_kick) on the GPU vs the CPU oracle,
through the C ABI.

Bars:
  - photon counts: bit-exact, step by step (integers decided in FP64 on both sides
    from the same Philox draws; a count could differ only if a uniform fell within
    rounding of a CDF boundary, probability ~1e-16 per draw).
  - positions / velocities: within 1e-12 / 1e-10 of their rms after the steps, the
    one-step bars of the force tests widened for several steps.
  - batches: bit-identical to the crystal stepped alone.
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_13973_amd import inputs, native

pytestmark = pytest.mark.gpu

Q, M = inputs.ION_CHARGE, inputs.ION_MASS


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = native.Context(0)
    yield c
    c.close()


def strong_beams():
    """The cooling geometry with intensities raised so that ~2% of the ions scatter a
    photon per beam and step (saturated axial beams, a 30 um planar waist)."""
    return inputs.cooling_beams(w_y=30e-6, s_perp=2.0, s_par=0.5, offset=5e-6)


def crystal(n, seed, beams):
    g = inputs.rng(seed)
    pos = inputs.uniform_ball(n, 1e-4, g)
    vel = inputs.thermal_velocities(n, 10e-3, M, g)  # Doppler shifts of order gamma0
    return inputs.Crystal(pos, vel, beams=beams, seed=seed)


def make(ctx, cr, method="direct", p=8, leaf=32, precision="fp64"):
    c = ctx.crystal(cr.pos, cr.vel, cr.charge, cr.mass, cr.seed)
    c.set_trap(B=cr.B, omega_z=cr.omega_z, delta=cr.delta, omega_r=cr.omega_r, dt=cr.dt)
    c.set_beams(cr.beams)
    c.set_force(method, p, leaf, precision)
    return c


def test_beam_counts_and_state_match_oracle(ctx):
    say("beam mode: counts per step and the state after 4 steps")
    cr = crystal(1000, 41, strong_beams())
    c = make(ctx, cr)
    x, v = cr.pos, cr.vel
    total = 0
    for s in range(4):
        c.step(1)
        st = c.read_state()
        x, v, ph = O.run(x, v, Q, M, cr.trap(), cr.dt, 1, step0=s, seed=cr.seed, laser=cr.laser(),
                         return_photons=True)
        assert np.array_equal(st["photons"], ph), s
        total += int(ph.sum())
    c.destroy()
    say(f"   {total} photons over 4 steps")
    assert total > 100  # the test exercises the kick, not an empty laser
    assert np.abs(st["pos"] - x).max() <= 1e-12 * math.sqrt((x ** 2).sum(1).mean())
    assert np.abs(st["vel"] - v).max() <= 1e-10 * math.sqrt((v ** 2).sum(1).mean())


def test_beam_mode_with_fmm_and_batch_equals_alone(ctx):
    say("beam mode: FMM mixed, batch vs alone")
    crs = [crystal(n, 50 + n, strong_beams()) for n in (600, 1500)]
    alone = []
    for cr in crs:
        c = make(ctx, cr, "fmm", 8, 32, "mixed")
        c.step(3)
        alone.append(c.read_state())
        c.destroy()
    cs = [make(ctx, cr, "fmm", 8, 32, "mixed") for cr in crs]
    native.step_batch(cs, [3, 3])
    for c, a in zip(cs, alone):
        b = c.read_state()
        c.destroy()
        assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["vel"], b["vel"])
        assert np.array_equal(a["photons"], b["photons"])


def test_beam_kick_adds_near_partials_beside_the_far_field(monkeypatch):
    """Leaves of 128 ions: the near field runs beside the far field and the beam
    variant of the kick adds the near-field partials to the far field itself;
    the states and photon counts equal those of the schedule with the near
    field after the far field (the partials added by the far-field kernel), bit
    for bit."""
    say("beam mode: kick-side near-field partials vs the serial schedule")
    cr = crystal(3000, 61, strong_beams())
    out = {}
    for conc in ("0", "1"):
        monkeypatch.setenv("PT_NEAR_CONCURRENT", conc)
        with native.Context(0) as c2:
            k = make(c2, cr, "fmm", 8, 128, "mixed")
            k.step(3)
            out[conc] = k.read_state()
    a, b = out["0"], out["1"]
    assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["vel"], b["vel"])
    assert np.array_equal(a["photons"], b["photons"]) and int(a["photons"].sum()) > 0


def test_invalid_beam_parameters(ctx):
    say("beam mode: invalid parameters")
    cr = crystal(10, 7, strong_beams())
    c = make(ctx, cr)

    def bad(**kw):
        las = strong_beams()
        beams = [dict(b) for b in las["beams"]]
        for k, val in kw.items():
            if k in ("gamma0", "wavelength"):
                las[k] = val
            else:
                beams[2][k] = val
        las["beams"] = beams
        with pytest.raises(native.PTError) as e:
            c.set_beams(las)
        assert e.value.code == native.PT_EINVAL, kw

    bad(gamma0=0.0)
    bad(gamma0=float("nan"))
    bad(wavelength=-1.0)
    bad(khat=(0.0, 0.0, 0.0))
    bad(s0=-0.1)
    bad(waist_y=0.0)
    bad(detuning=float("inf"))
    with pytest.raises(native.PTError) as e:  # no beams
        c.set_beams(dict(wavelength=313e-9, gamma0=inputs.GAMMA0, beams=[]))
    assert e.value.code == native.PT_EINVAL
    # gamma0 dt > 4 would allow photon means above 2 per step
    with pytest.raises(native.PTError) as e:
        c.set_trap(dt=1e-7)
    assert e.value.code == native.PT_EINVAL
    p = native.LaserParams(3, 0.0, 313e-9)
    assert native.load().pt_set_laser_params(c.h, p) == native.PT_EINVAL
    # the parameters in force before the rejected calls still work
    c.step(1)
    assert c.read_state()["step"] == 1
    c.destroy()

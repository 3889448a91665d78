"""Artificial damping (the paper's proposal for crystal equilibria) on the GPU vs the
CPU oracle, through the C ABI.

Bars:
  - a damped run: positions / velocities within 1e-11 / 1e-9 of their rms after
    2,000 steps (the damping contracts the dynamics, so rounding differences do not
    grow; the one-step bars are 1e-13 / 1e-11).
  - two ions relax to the closed-form separation within 5e-5 (the oracle pin's bar:
    the damped fixed point's O(dt^2) offset at dt = 2 ns is 2.7e-5).
  - batches: bit-identical to each crystal alone.
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


def larmor_trap(beta=0.6, delta=0.05, damping=2e6):
    """Rotating frame at omega_c / 2 (no effective magnetic field there), B set for beta."""
    wz = 2 * math.pi * 1.5e6
    wc = 2 * wz * math.sqrt(beta + 0.5)
    return dict(B=wc * M / Q, omega_z=wz, delta=delta, omega_r=0.5 * wc, damping=damping)


def make(ctx, pos, trap, dt, method="direct", p=8, leaf=32, precision="fp64"):
    wr = trap["omega_r"]
    vel = wr * np.stack([pos[:, 1], -pos[:, 0], np.zeros(len(pos))], 1)
    c = ctx.crystal(pos, vel, Q, M)
    c.set_trap(B=trap["B"], omega_z=trap["omega_z"], delta=trap["delta"], omega_r=wr, dt=dt,
               damping=trap["damping"])
    c.set_force(method, p, leaf, precision)
    return c, vel


def rms(a):
    return math.sqrt((a ** 2).sum(1).mean())


def test_damped_run_matches_oracle(ctx):
    say("damped run vs oracle")
    trap = larmor_trap()
    pos = inputs.uniform_ball(30, 2e-5, inputs.rng(41))
    c, vel = make(ctx, pos, trap, 2e-9)
    c.step(2000)
    st = c.read_state()
    c.destroy()
    x, v = O.run(pos, vel, Q, M, trap, 2e-9, 2000)
    say(f"   pos {np.abs(st['pos'] - x).max() / rms(x):.1e}, vel {np.abs(st['vel'] - v).max() / rms(v):.1e}")
    assert np.abs(st["pos"] - x).max() <= 1e-11 * rms(x)
    assert np.abs(st["vel"] - v).max() <= 1e-9 * rms(v)


def test_two_ions_relax_to_the_closed_form(ctx):
    say("two ions relax")
    trap = larmor_trap()
    wz, wr = trap["omega_z"], trap["omega_r"]
    beta = wr * (Q * trap["B"] / M - wr) / wz ** 2 - 0.5
    d_ref = (2 * O.K_E * Q * Q / (M * wz ** 2 * (beta - trap["delta"] / 2))) ** (1 / 3)
    pos = np.array([[3e-6, 2e-6, 1e-6], [-4e-6, -1e-6, -0.5e-6]])
    c, _ = make(ctx, pos, trap, 2e-9)
    c.step(12000)
    xr, vr = c.read_rotating_state()
    d = c.rotating_diagnostics()
    c.destroy()
    sep = xr[0] - xr[1]
    err = abs(np.linalg.norm(sep) / d_ref - 1)
    say(f"   separation vs closed form {err:.1e}; rotating-frame KE {d['ke_axial'] + d['ke_planar']:.1e} J")
    assert err < 5e-5
    assert abs(abs(sep[1]) / np.linalg.norm(sep) - 1) < 1e-9
    assert np.abs(vr).max() < 1e-6


def test_damping_with_fmm_batch_equals_alone_and_invalid(ctx):
    say("damping: FMM batch, invalid values")
    trap = larmor_trap()
    poss = [inputs.uniform_ball(n, 4e-5, inputs.rng(80 + n)) for n in (400, 900)]
    alone = []
    for pos in poss:
        c, _ = make(ctx, pos, trap, 2e-9, "fmm", 8, 32, "mixed")
        c.step(20)
        alone.append(c.read_state())
        c.destroy()
    cs = [make(ctx, pos, trap, 2e-9, "fmm", 8, 32, "mixed")[0] for pos in poss]
    native.step_batch(cs, [20, 20])
    for c, a in zip(cs, alone):
        b = c.read_state()
        assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["vel"], b["vel"])
    c = cs[0]
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(native.PTError) as e:
            c.set_trap(damping=bad)
        assert e.value.code == native.PT_EINVAL
    for c in cs:
        c.destroy()

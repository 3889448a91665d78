"""GPU path vs the CPU oracle, through the C ABI.

Bars:
  - Morton keys, permutation, boxes, interaction lists, photon counts: bit-exact.
  - direct-sum forces: max_i |F_gpu - F_oracle| / rms_j |F_oracle| <= 1e-12.
  - FP64 FMM forces vs the oracle FMM at the same p and leaf size: <= 1e-11 (same metric).
  - one step: positions / velocities within 1e-13 / 1e-11 relative to their rms.
FP64 sums of 1e3-1e4 similar terms round at ~1e-15..1e-14 relative; the GPU and
oracle FMM differ in basis and summation order only, so 1e-11 leaves three
orders of margin while any formula error shows at the truncation level (~1e-6)
or worse.
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


def rel_max(a, b):
    """max_i |a_i - b_i| / rms_j |b_j| over 3-vectors."""
    return np.linalg.norm(a - b, axis=1).max() / math.sqrt((np.linalg.norm(b, axis=1) ** 2).mean())


def make(ctx, cr: inputs.Crystal, method="direct", p=8, leaf=32, precision="fp64"):
    c = ctx.crystal(cr.pos, cr.vel, cr.charge, cr.mass, cr.seed)
    c.set_trap(B=cr.B, omega_z=cr.omega_z, delta=cr.delta, omega_r=cr.omega_r, dt=cr.dt)
    c.set_laser(cr.photon_mean)
    c.set_force(method, p, leaf, precision)
    return c


def ball(n, seed, R=1e-4):
    g = inputs.rng(seed)
    pos = inputs.uniform_ball(n, R, g)
    vel = inputs.thermal_velocities(n, 10e-3, M, g)
    return inputs.Crystal(pos, vel, seed=seed)


# ---------------------------------------------------------------- direct
# sizes across the direct sum's work split: one source chunk (n < 1024), two
# (1025), eight with a ragged last tile and piece (4100), sixteen (9001)
@pytest.mark.parametrize("n", [1, 2, 3, 511, 1000, 1025, 4100, 9001])
def test_direct_forces_match_oracle(ctx, n):
    say(f"direct forces n={n}")
    cr = ball(n, 100 + n)
    c = make(ctx, cr)
    F = c.compute_forces()
    ref = O.coulomb_direct(cr.pos, Q)
    c.destroy()
    if n == 1:
        assert np.all(F == 0)
    else:
        assert rel_max(F, ref) <= 1e-12


def test_direct_batch_equals_alone(ctx):
    """Crystals with different chunk counts in one batch: each crystal's sums
    keep their order, so the batch result equals the single-crystal one bit for bit."""
    say("direct batch invariance")
    crs = [ball(n, 900 + n) for n in (1025, 3, 9001, 600)]
    alone = []
    for cr in crs:
        c = make(ctx, cr)
        alone.append(c.compute_forces())
        c.destroy()
    cs = [make(ctx, cr) for cr in crs]
    together = native.compute_forces_batch(cs)
    for c in cs:
        c.destroy()
    for a, b in zip(alone, together):
        assert np.array_equal(a, b)


def test_direct_coincident_pair_contributes_nothing(ctx):
    say("direct coincident")
    pos = np.array([[0.0, 0.0, 0.0], [1e-5, 0, 0], [1e-5, 0, 0], [0, 2e-5, 0]])
    c = ctx.crystal(pos, np.zeros_like(pos), Q, M)
    F = c.compute_forces()
    c.destroy()
    ref = O.coulomb_direct(pos, Q)
    assert np.isfinite(F).all()
    assert rel_max(F, ref) <= 1e-12


def test_one_step_direct_matches_oracle(ctx):
    say("one step direct")
    cr = ball(700, 7)
    cr.photon_mean = 0.05
    c = make(ctx, cr)
    c.step(1)
    st = c.read_state()
    c.destroy()
    x, v, ph = O.run(cr.pos, cr.vel, Q, M, cr.trap(), cr.dt, 1, seed=cr.seed, laser=cr.laser(), return_photons=True)
    assert np.array_equal(st["photons"], ph)
    assert st["step"] == 1
    assert np.abs(st["pos"] - x).max() <= 1e-13 * math.sqrt((x ** 2).sum(1).mean())
    assert np.abs(st["vel"] - v).max() <= 1e-11 * math.sqrt((v ** 2).sum(1).mean())


def test_photon_counts_bit_exact_over_steps(ctx):
    say("photon counts")
    n = 4000
    pos = np.zeros((n, 3))
    pos[:, 0] = np.arange(n) * 1e-3  # far apart: Coulomb negligible, state irrelevant for counts
    cr = inputs.Crystal(pos, np.zeros((n, 3)), photon_mean=0.05, seed=0xDEADBEEF12345)
    c = make(ctx, cr)
    for s in range(3):
        c.step(1)
        got = c.read_state()["photons"]
        assert np.array_equal(got, O.photon_counts(n, cr.seed, s, 0.05))
    c.destroy()


def test_wall_and_trap_one_step(ctx):
    say("wall one step")
    cr = ball(300, 9)
    cr.delta, cr.omega_r = 0.01, 2 * math.pi * 180e3
    c = make(ctx, cr)
    c.step(3)
    st = c.read_state()
    c.destroy()
    x, v = O.run(cr.pos, cr.vel, Q, M, cr.trap(), cr.dt, 3, seed=cr.seed)
    assert np.abs(st["pos"] - x).max() <= 1e-12 * math.sqrt((x ** 2).sum(1).mean())
    assert np.abs(st["vel"] - v).max() <= 1e-10 * math.sqrt((v ** 2).sum(1).mean())


# ---------------------------------------------------------------- tree
@pytest.mark.parametrize("n,s", [(1, 4), (5, 4), (1000, 32), (3000, 16)])
def test_tree_bit_exact(ctx, n, s):
    say(f"tree n={n} s={s}")
    cr = ball(n, 200 + n)
    c = make(ctx, cr, "fmm", 4, s)
    c.compute_forces()
    T = c.export_tree()
    c.destroy()
    R = O.tree(cr.pos, s)
    assert np.array_equal(T["root"], R["root"])
    assert np.array_equal(T["key"], R["key"])
    assert np.array_equal(T["perm"], R["perm"])
    for k in ("level", "parent", "ion_begin", "ion_end", "coords", "is_leaf", "v_off", "v_src", "near_off",
              "near_src"):
        assert np.array_equal(T[k], R[k]), k


def test_large_batch_sort_bit_exact_and_ordered_after_queued_steps(ctx):
    """450,000 ions, above the size from which the radix passes take tiles of 8
    keys per thread: the measured evaluation's tree equals the oracle's bit for
    bit; after queued steps (the top-digit sort and its refinement) the
    permutation is one and orders the ions' keys by (key, ion)."""
    n = 450000
    say(f"large-batch sort n={n}")
    cr = ball(n, 901, R=1e-3)
    c = make(ctx, cr, "fmm", 4, 64, "mixed")
    c.compute_forces()
    T = c.export_tree()
    R = O.tree(cr.pos, 64)
    assert np.array_equal(T["key"], R["key"]) and np.array_equal(T["perm"], R["perm"])
    assert np.array_equal(T["ion_begin"], R["ion_begin"]) and np.array_equal(T["level"], R["level"])
    c.step(3)
    T = c.export_tree()
    c.destroy()
    perm = T["perm"].astype(np.int64)  # ion at each sorted slot; keys are per ion
    assert np.array_equal(np.sort(perm), np.arange(n))
    ks = T["key"][perm]
    up = ks[1:] > ks[:-1]
    tie = ks[1:] == ks[:-1]
    assert np.all(up | (tie & (perm[1:] > perm[:-1])))


def test_tree_bit_exact_clumps(ctx):
    say("tree clumps")
    g = inputs.rng(31)
    pos = np.concatenate([inputs.uniform_ball(700, 1e-4, g), 3e-4 + inputs.uniform_ball(700, 3e-6, g),
                          -2e-4 + inputs.uniform_ball(600, 2e-5, g)])
    c = ctx.crystal(pos, np.zeros_like(pos), Q, M)
    c.set_force("fmm", 4, 8)
    c.compute_forces()
    T = c.export_tree()
    wc = ctx.work_counts()
    c.destroy()
    R = O.tree(pos, 8)
    for k in ("key", "perm", "level", "parent", "ion_begin", "ion_end", "coords", "is_leaf", "v_off", "v_src",
              "near_off", "near_src"):
        assert np.array_equal(T[k], R[k]), k
    # work counts: boxes, leaves, V pairs, near-field ion pairs (self excluded)
    size = R["ion_end"] - R["ion_begin"]
    near_pairs = 0
    for b in np.flatnonzero(R["is_leaf"]):
        src = size[R["near_src"][R["near_off"][b]:R["near_off"][b + 1]]].sum()
        near_pairs += int(size[b]) * int(src) - int(size[b])
    assert list(wc[:4]) == [len(R["level"]), int(R["is_leaf"].sum()), len(R["v_src"]), near_pairs]


def test_tree_depth_limit_with_coincident_ions(ctx):
    """Two stacks of 20 identical positions inside a ball: the tree cannot separate them, so
    it runs to its depth limit (level 16) and keeps leaves above the leaf size there; the
    zero-separation pairs contribute nothing (the oracle's pin of the same case)."""
    say("tree depth limit, coincident ions")
    pos = np.concatenate([np.full((20, 3), 1e-5), np.zeros((20, 3)), inputs.uniform_ball(200, 5e-5, inputs.rng(17))])
    c = ctx.crystal(pos, np.zeros_like(pos), Q, M)
    c.set_force("fmm", 6, 4, "fp64")
    F = c.compute_forces()
    T = c.export_tree()
    c.set_force("fmm", 6, 4, "mixed")
    Fm = c.compute_forces()
    c.destroy()
    R = O.tree(pos, 4)
    assert R["level"].max() == 16
    for k in ("key", "perm", "level", "parent", "ion_begin", "ion_end", "coords", "is_leaf", "v_off", "v_src",
              "near_off", "near_src"):
        assert np.array_equal(T[k], R[k]), k
    ref = O.fmm_coulomb(pos, Q, 6, 4)
    err = rel_max(F, ref)
    say(f"   fp64 max err / rms = {err:.3e}")
    assert err <= 1e-11
    assert np.isfinite(Fm).all()
    # against the oracle FMM of the same p and leaf, so only the FP32 rounding remains
    rms = math.sqrt(((Fm - ref) ** 2).sum() / (ref ** 2).sum())
    say(f"   mixed rms rel err vs oracle FMM = {rms:.3e}")
    assert rms < 1e-5


# ---------------------------------------------------------------- FMM
@pytest.mark.parametrize("n,p,s", [(1000, 8, 32), (2000, 4, 16), (1500, 12, 64), (300, 6, 300)])
def test_fmm_fp64_matches_oracle_fmm(ctx, n, p, s):
    say(f"fmm fp64 n={n} p={p} s={s}")
    cr = ball(n, 300 + n)
    c = make(ctx, cr, "fmm", p, s)
    F = c.compute_forces()
    c.destroy()
    ref = O.fmm_coulomb(cr.pos, Q, p, s)
    err = rel_max(F, ref)
    say(f"   max err / rms = {err:.3e}")
    assert err <= 1e-11


def test_fmm_mixed_error_vs_fp64(ctx):
    say("fmm mixed")
    cr = ball(3000, 41)
    c = make(ctx, cr, "fmm", 10, 32, "mixed")
    F = c.compute_forces()
    c.destroy()
    ref = O.coulomb_direct(cr.pos, Q)
    rms = math.sqrt(((F - ref) ** 2).sum() / (ref ** 2).sum())
    say(f"   mixed p=10 rms rel err vs direct = {rms:.3e}")
    assert rms < 5e-6


def test_batch_equals_alone(ctx):
    say("batch invariance")
    crs = [ball(n, 500 + n) for n in (100, 1700, 650)]
    alone = []
    for cr in crs:
        c = make(ctx, cr, "fmm", 6, 24)
        alone.append(c.compute_forces())
        c.destroy()
    cs = [make(ctx, cr, "fmm", 6, 24) for cr in crs]
    together = native.compute_forces_batch(cs)
    for c in cs:
        c.destroy()
    for a, b in zip(alone, together):
        assert np.array_equal(a, b)

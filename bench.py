#!/usr/bin/env python3
"""Benchmark: ion-steps/s of FMM-force Penning-trap steps on one MI355X.

Workload: 100,000 ions on a 5%-jittered simple cubic lattice in a prolate
ellipsoid with semi-axes (400, 400, 800) um, 10 mK velocities, B = 4.5 T,
omega_z = 2 pi 1.5 MHz, dt = 1 ns, no laser.  The expansion degree p is the
smallest one whose RMS relative Coulomb-force error against the FP64 direct
sum is <= 1e-6, chosen at start-up (not timed); with the default --leaf 0
the leaf size is tuned too: for each candidate leaf size the smallest such
p, then the fastest pair.

Prints one JSON line: value = ion-steps/s of the mixed-precision form (or
--precision fp64) over the timed steps as the library runs them (no
instrumentation), roofline of the dominant kernel (M2L on the matrix cores,
or the P2P kernel on the vector ALUs) from HIP events over a second timed
run of the same steps from the same state that records the phase events,
and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2405_13973_amd import inputs, native  # noqa: E402

METRIC = "ion-steps/s at N=1e5, RMS rel force error≤1e-6 vs FP64; p99 latency mixed stream"
PEAK = {"mfma_fp32": 157.3, "mfma_fp64": 78.6, "valu_fp32": 157.3, "valu_fp64": 78.6}
# Algorithmic flops of one near-field pair by the measurement convention of
# the method's cost model: 3 sub (separation), 3 FMA for r^2 (6 flops), 1
# rsqrt, 3 mul for r^-3 q... counted as 20 in all.  The mixed kernel itself
# issues 14 floating-point operations per pair (3 FMA for r^2, 1 rsqrt, 2 mul,
# 3 FMA), after 3 integer subtractions and 3 conversions that make the
# separation; both figures are reported.
P2P_FLOPS_PER_PAIR = 20
P2P_ISSUED_FLOPS_PER_PAIR = 14
# with the potential: one add more (the 1/r sum)
P2P_POT_FLOPS_PER_PAIR = 21
# phase 0 includes P2M, which runs on a second stream beside the list builders
PHASES = ["tree_lists_p2m", "m2m", "m2l_kernel", "m2l_reduce_l2l", "p2p_kernel", "l2p_partials", "total"]
# leaf sizes the tuner tries (for each the smallest p meeting the error bound,
# then the fastest): step time depends on where a crystal's boxes are split,
# not monotonically on the leaf size
LEAF_CANDIDATES = (32, 64, 128, 192, 224, 256, 320, 384)
# (near-field workgroups per CU, fork direction) pairs the schedule tuner tries:
# share 0 = the library default, fork -1 = by the measured balance, 0 = the
# near field forks to the second stream (schedule parameters: no effect on the
# results)
SCHEDULE_CANDIDATES = ((0, -1), (4, -1), (5, -1), (4, 0), (5, 0))
# the timed steps record the phase events of every TIMING_EVERY-th evaluation
# (each recorded event is a packet in the stream; recording all of them slowed
# the step by 12-35%)
TIMING_EVERY = 4  # 0: the library's default (3 beside the upward pass, 4 after it)


def measured_traffic(kernel, p, leaf, precision, n):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    runs (one record per profiled workload), or None when no record matches
    the workload or the kernel source has changed since it was taken."""
    import hashlib

    try:
        recs = json.load(open(os.path.join(ROOT, "profiles", f"{kernel}_traffic.json")))["records"]
    except (OSError, ValueError, KeyError):
        return None
    for rec in recs:
        w = rec.get("workload", {})
        if (w.get("p"), w.get("leaf_size"), w.get("precision"), w.get("n_ions")) != (p, leaf, precision, n):
            continue
        try:
            src = open(os.path.join(ROOT, rec["source"]), "rb").read()
        except (OSError, KeyError):
            return None
        return rec["hbm_bytes_per_launch"] if hashlib.sha256(src).hexdigest() == rec.get("sha256") else None
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rms_rel(F, ref):
    """Relative RMS error: of the forces, and of the potential (eq. rms_pot)."""
    return math.sqrt(((F - ref) ** 2).sum() / (ref ** 2).sum())


def choose_p(c, F_dir, precision, leaf, p0, target=1e-6, pmax=16):
    errs = {}
    for p in range(p0, pmax + 1):
        c.set_force("fmm", p, leaf, precision)
        err = rms_rel(c.compute_forces(), F_dir)
        errs[p] = err
        log(f"  {precision} p={p} leaf={leaf}: rms rel force err vs direct = {err:.3e}")
        if err <= target:
            return p, err, errs
    raise SystemExit(f"no p <= {pmax} reaches rms error {target} in {precision}")


def timed_steps(ctx, c, steps, warmup, sync, phases_too=True):
    """Wall time of `steps` steps after `warmup`.  With phases_too the timed
    region itself carries the HIP-event phase timing of every TIMING_EVERY-th
    evaluation (the library keeps the event sets of up to 64 evaluations in
    flight, so the timing adds no host wait), and the same steps are run again
    from the same state without events for comparison.  Returns (seconds, phases, count, work counts, seconds of
    the uninstrumented run)."""
    c.step(warmup)
    st = c.read_state()
    sync()
    if phases_too:
        ctx.set_timing(True, every=TIMING_EVERY)
    t0 = time.perf_counter()
    c.step(steps)
    ctx.synchronize()  # also reads back the queued steps' outcome (and re-runs any that overflowed)
    sync()
    t1 = time.perf_counter()
    phases, count, wc, plain = None, 0, None, None
    if phases_too:
        phases, count = ctx.phase_times(with_count=True)
        wc = ctx.work_counts()
        ctx.set_timing(False)
        end = c.read_state()
        c.set_state(st["pos"], st["vel"], st["step"])
        sync()
        t2 = time.perf_counter()
        c.step(steps)
        ctx.synchronize()
        sync()
        plain = time.perf_counter() - t2
        c.set_state(end["pos"], end["vel"], end["step"])
    return t1 - t0, phases, count, wc, plain


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def omp_threads(k):
    """Sets the OpenMP thread count of this process (the oracle's runtime)."""
    import ctypes

    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(k))
        return True
    except OSError:
        return False


def cpu_baseline(cr, p, leaf, F_dir_gpu):
    """The FP64 CPU oracle, as it stands, on the host cores: full FMM steps of
    the same crystal (same p and leaf size) on every thread, and one step on one
    core.  Also ties the GPU direct sum used as the accuracy reference to the
    oracle on sampled ions."""
    from oracle import oracle as O

    idx = np.linspace(0, cr.n - 1, 48).astype(np.int32)
    ref = O.coulomb_direct_sampled(cr.pos, cr.charge, idx)
    dev = np.abs(F_dir_gpu[idx] - ref).max() / np.sqrt((ref ** 2).sum(1).mean())
    log(f"  GPU direct vs oracle direct on {len(idx)} sampled ions: max err / rms = {dev:.2e}")
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # one step, then more from the same state until about 10 s of work in all
    t0 = time.perf_counter()
    O.run(cr.pos, cr.vel, cr.charge, cr.mass, cr.trap(), cr.dt, 1, method="fmm", p=p, leaf_size=leaf)
    first = time.perf_counter() - t0
    steps = 1
    if first < 10.0:
        more = min(50, math.ceil((10.0 - first) / first))
        O.run(cr.pos, cr.vel, cr.charge, cr.mass, cr.trap(), cr.dt, more, method="fmm", p=p, leaf_size=leaf)
        steps += more
    el = time.perf_counter() - t0
    log(f"  oracle: {steps} FMM steps of {cr.n} ions (p={p}, leaf={leaf}) in {el:.1f} s on {cores} threads")
    # the oracle's FMM potential of all ions once (the potential measurement's baseline)
    t0 = time.perf_counter()
    O.fmm_potential(cr.pos, cr.charge, p, leaf)
    pel = time.perf_counter() - t0
    log(f"  oracle potential: {pel:.1f} s for {cr.n} ions")
    one = None
    if omp_threads(1):
        t0 = time.perf_counter()
        O.run(cr.pos, cr.vel, cr.charge, cr.mass, cr.trap(), cr.dt, 1, method="fmm", p=p, leaf_size=leaf)
        one = time.perf_counter() - t0
        omp_threads(cores)
        log(f"  oracle: 1 FMM step on 1 core in {one:.1f} s")
    return {"value": cr.n * steps / el, "unit": "ion-steps/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
            "sample": f"{steps} full FP64 FMM steps (p={p}, leaf {leaf}) of the same {cr.n}-ion crystal, "
                      f"{el:.1f} s wall on {cores} threads; direct sum checked on 48 sampled ions "
                      f"(max err/rms {dev:.1e})",
            "one_core_ion_steps_per_s": cr.n / one if one else None,
            "one_core_sample": f"1 full FP64 FMM step on 1 core, {one:.1f} s wall" if one else None,
            "potential_ion_evals_per_s": cr.n / pel,
            "potential_sample": f"one FP64 FMM potential evaluation of all {cr.n} ions, {pel:.1f} s wall"}


def bench_potential(ctx, c, cr, p, leaf, prec, evals=10):
    """Coulomb potential at every ion (the quantity of eq. rms_pot) with the
    benchmark's force parameters: device time per evaluation (HIP events),
    the near-field kernel's rate, Error_pot against the FP64 direct potential
    and the energy."""
    c.set_state(cr.pos, cr.vel, 0)
    c.set_force("direct")
    phi_dir = c.compute_potential()
    c.set_force("fmm", p, leaf, prec)
    for _ in range(2):
        c.compute_forces()
    ctx.set_timing(True)
    for _ in range(evals):
        c.compute_forces()
    f_ph = ctx.phase_times()
    ctx.set_timing(False)
    phi = c.compute_potential()
    ctx.set_timing(True)
    for _ in range(evals):
        c.compute_potential()
    ph = ctx.phase_times()
    wc = ctx.work_counts()
    ctx.set_timing(False)
    U = c.coulomb_energy()
    err = rms_rel(phi, phi_dir)
    tfl = P2P_POT_FLOPS_PER_PAIR * wc[3] / (ph[4] * 1e-3) / 1e12
    peak = PEAK["valu_fp32" if prec == "mixed" else "valu_fp64"]
    out = {
        "ms_per_eval": float(ph[6]), "ion_evals_per_s": cr.n / (ph[6] * 1e-3),
        "force_eval_ms": float(f_ph[6]), "potential_over_force_time": float(ph[6] / f_ph[6]),
        "error_pot": err, "coulomb_energy_J": U, "p": p, "leaf_size": leaf, "precision": prec,
        "p2p_kernel_ms": float(ph[4]),
        "phase_ms": {k: float(v) for k, v in zip(PHASES, ph)},
        "force_phase_ms": {k: float(v) for k, v in zip(PHASES, f_ph)},
        "p2p_roofline": {"bound": "alu", "achieved": tfl, "peak": peak, "unit": "TFLOP/s", "frac": tfl / peak,
                         "traffic": measured_traffic("p2p_pot", p, leaf, prec, cr.n),
                         "algorithmic": f"{P2P_POT_FLOPS_PER_PAIR} flops per near-field pair, {int(wc[3])} "
                                        f"ordered pairs per launch"},
    }
    log(f"  potential: {ph[6]:.3f} ms per evaluation (forces {f_ph[6]:.3f}), Error_pot {err:.2e}, U = {U:.6e} J")
    return out


# HBM bytes per ion of the kick + half-drift kernel: state read and written
# (6 FP64 each), the field read (3 FP64), the photon count written (int32)
KICK_BYTES_PER_ION = 48 + 48 + 24 + 4


def bench_diagnostics(ctx, c, cr, p, leaf, prec, sync, calls=10):
    """Rotating-frame diagnostics (eqs. rotation, pe_rot, temp_ax, temp_pl) of the
    benchmark crystal with its force parameters: wall time per call (one FMM
    Coulomb-energy evaluation, the per-crystal sums on the device, a few doubles
    back to the host)."""
    c.set_state(cr.pos, cr.vel, 0)
    c.set_force("fmm", p, leaf, prec)
    c.set_trap(B=cr.B, omega_z=cr.omega_z, dt=cr.dt, omega_r=2 * math.pi * 180e3)
    d = c.rotating_diagnostics()
    sync()
    t0 = time.perf_counter()
    for _ in range(calls):
        d = c.rotating_diagnostics()
    el = (time.perf_counter() - t0) / calls
    c.set_trap(B=cr.B, omega_z=cr.omega_z, dt=cr.dt)
    log(f"  rotating-frame diagnostics: {el * 1e3:.3f} ms per call; E_r = {d['energy']:.6e} J")
    return {"ms_per_call": el * 1e3, "omega_r": 2 * math.pi * 180e3, "values": d}


def bench_relaxation(ctx, prec, sync, n=10000, steps=5000, dt=2e-9, damping=2e6):
    """Artificial damping towards a crystal equilibrium (the paper's proposal in place
    of a BFGS minimisation for large N): n ions uniform in a ball at the density of
    the 1,000-ion configuration, at rest in a frame turning at omega_c / 2 (where
    velocity damping reaches every mode; B set for beta = 0.6, delta = 0.05), FMM
    forces (p = 8, leaf 64); rotating-frame temperatures and energy before and after
    `steps` damped steps, and the wall time."""
    wz = 2 * math.pi * 1.5e6
    wc = 2 * wz * math.sqrt(1.1)
    B, wr = wc * inputs.ION_MASS / inputs.ION_CHARGE, 0.5 * wc
    pos = inputs.uniform_ball(n, 100e-6 * (n / 1000) ** (1 / 3), inputs.rng(7))
    vel = wr * np.stack([pos[:, 1], -pos[:, 0], np.zeros(n)], 1)
    c = ctx.crystal(pos, vel, inputs.ION_CHARGE, inputs.ION_MASS, 7)
    c.set_trap(B=B, omega_z=wz, delta=0.05, omega_r=wr, dt=dt, damping=damping)
    c.set_force("fmm", 8, 64, prec)
    d0 = c.rotating_diagnostics()
    c.step(200)  # the first, fastest part of the relaxation; also the warm-up
    d1 = c.rotating_diagnostics()
    sync()
    t0 = time.perf_counter()
    c.step(steps)
    sync()
    el = time.perf_counter() - t0
    d2 = c.rotating_diagnostics()
    c.destroy()
    log(f"  relaxation: {n} ions, {steps} damped steps in {el:.2f} s; T_ax {d1['temp_axial']:.3g} -> "
        f"{d2['temp_axial']:.3g} K, T_perp {d1['temp_planar']:.3g} -> {d2['temp_planar']:.3g} K")
    return {"n_ions": n, "steps": steps, "dt_s": dt, "damping_per_s": damping, "ms_per_step": el * 1e3 / steps,
            "ion_steps_per_s": n * steps / el, "simulated_s_per_wall_s": steps * dt / el,
            "temp_axial_K": [d0["temp_axial"], d1["temp_axial"], d2["temp_axial"]],
            "temp_planar_K": [d0["temp_planar"], d1["temp_planar"], d2["temp_planar"]],
            "energy_J": [d0["energy"], d1["energy"], d2["energy"]],
            "note": "temperatures and rotating-frame energy at the start, after 200 steps, and at the end"}


def bench_beams(ctx, c, cr, p, leaf, prec, steps, warmup, sync, ref_seconds):
    """The same steps with the beam-mode laser of eq. (scattering_rate) on (the
    cooling set-up of the paper's Sec. 5: two uniform axial beams and the offset
    planar Gaussian beam), timed like the main steps."""
    c.set_state(cr.pos, cr.vel, 0)
    c.set_force("fmm", p, leaf, prec)
    c.set_beams(inputs.cooling_beams())
    # photons of the first step: the benchmark crystal starts far from equilibrium,
    # and within a few steps the trap accelerates its outer ions to speeds whose
    # Doppler shift detunes every beam
    c.step(1)
    photons = int(c.read_state()["photons"].sum())
    el = timed_steps(ctx, c, steps, warmup, sync, phases_too=False)[0]
    c.set_laser(0.0)
    log(f"  beams: {steps} steps in {el * 1e3:.2f} ms ({photons} photons in the first step)")
    return {"ms_per_step": el * 1e3 / steps, "ion_steps_per_s": cr.n * steps / el,
            "time_vs_no_laser": el / ref_seconds, "photons_first_step": photons,
            "kick_bytes_per_ion": KICK_BYTES_PER_ION,
            "setup": "two uniform axial beams (Delta=-gamma0/2, S0=5e-3) and a planar Gaussian beam along +x "
                     "(d=5 um, w_y=2.48 um, w_z=1 mm, S0=0.5, Delta=2 pi 13.6 MHz), gamma0=2 pi 18 MHz"}


BATCH_LEAVES = (64, 128, 256, 384, 512)
# steps per crystal of the ensemble configuration (config 4)
ENSEMBLE_STEPS = 500
# serving cannot tune while requests arrive: the leaf size the ensemble tuner
# picks for the same range of crystal sizes (384 and 512 within 1% there)
SERVING_LEAF = 384


def tune_batch(ctx, cs, leaves, p_fixed, p0, precision, sync, time_it=True, target=1e-6, pmax=16):
    """For each leaf size the smallest p whose RMS force error on the three
    largest crystals is <= target (or p_fixed), then the fastest batch step.
    Crystals are restored to their initial state afterwards by the caller."""
    big = sorted(cs, key=lambda c: -c.n)[:3]
    init = [c.read_state() for c in cs]
    refs = []
    for c in big:
        c.set_force("direct")
        refs.append(c.compute_forces())
    best = None
    for leaf in leaves:
        for p in ([p_fixed] if p_fixed else range(p0, pmax + 1)):
            errs = []
            for c, R in zip(big, refs):
                c.set_force("fmm", p, leaf, precision)
                errs.append(rms_rel(c.compute_forces(), R))
            log(f"  leaf {leaf} p={p}: max rms rel force err on the largest crystals {max(errs):.3e}")
            if max(errs) <= target or p_fixed:
                break
        el = 0.0
        if time_it:
            for c in cs:
                c.set_force("fmm", p, leaf, precision)
            native.step_batch(cs, [2] * len(cs))
            sync()
            t0 = time.perf_counter()
            native.step_batch(cs, [5] * len(cs))
            sync()
            el = time.perf_counter() - t0
            for c, st in zip(cs, init):
                c.set_state(st["pos"], st["vel"], st["step"])
            log(f"  leaf {leaf} p={p}: {5 * sum(c.n for c in cs) / el:.4g} ion-steps/s")
        if best is None or el < best[3]:
            best = (leaf, p, errs, el)
    return best[0], best[1], best[2]


def tune_schedule(ctx, a, run, work, what):
    """The fastest (near share, fork direction) of SCHEDULE_CANDIDATES, set on
    the context (an earlier candidate is kept unless a later one is more than
    0.5% faster); run(share, fork) returns the seconds of `work` ion-steps.
    Given shares or fork directions are kept (a fork of -2 means tuned, or -1
    when the share is given)."""
    if a.near_share >= 0:
        cands = [(a.near_share, a.fork if a.fork >= -1 else -1)]
    elif a.fork >= -1:
        cands = [(s, a.fork) for s in sorted({s for s, _ in SCHEDULE_CANDIDATES})]
    else:
        cands = list(SCHEDULE_CANDIDATES)
    best = None
    for share, fork in cands:
        ctx.set_near_share(share)
        ctx.set_fork(fork)
        if len(cands) == 1:
            return share, fork
        el = run(share, fork)
        log(f"  {what} near share {share} fork {fork}: {work / el:.4g} ion-steps/s")
        # a later candidate must be faster by more than the runs' noise (0.5%)
        if best is None or el < best[2] * 0.995:
            best = (share, fork, el)
    ctx.set_near_share(best[0])
    ctx.set_fork(best[1])
    return best[0], best[1]


def bench_ensemble(a, ctx, sync):
    """Batched ensemble: independent crystals stepped together, one launch per
    phase per step for all of them."""
    crs = inputs.ensemble(count=a.crystals, seed=4)
    ntot = sum(c.n for c in crs)
    log(f"ensemble: {len(crs)} crystals, {ntot} ions (N {min(c.n for c in crs)}..{max(c.n for c in crs)})")
    cs = []
    for cr in crs:
        c = ctx.crystal(cr.pos, cr.vel, cr.charge, cr.mass, cr.seed)
        c.set_trap(B=cr.B, omega_z=cr.omega_z, dt=cr.dt)
        c.set_laser(cr.photon_mean)
        cs.append(c)
    # the error bound is checked on the largest crystals against the FP64 direct
    # sum; leaf size and p are tuned like config 3 unless given
    leaves = (a.leaf,) if a.leaf else BATCH_LEAVES
    a.leaf, a.p, errs = tune_batch(ctx, cs, leaves, a.p, a.p0, a.precision, sync, time_it=len(leaves) > 1)
    for c, cr in zip(cs, crs):
        c.set_force("fmm", a.p, a.leaf, a.precision)

    # the schedule is timed over long runs (200 steps): shorter ones, from the
    # initial state or from later ones, misjudged which fork direction is
    # faster over the timed steps
    def run(share, fork):
        for c, cr in zip(cs, crs):
            c.set_state(cr.pos, cr.vel, 0)
        native.step_batch(cs, [2] * len(cs))
        ctx.synchronize()
        sync()
        t0 = time.perf_counter()
        native.step_batch(cs, [200] * len(cs))
        ctx.synchronize()  # also re-runs any step that outgrew the capacities
        sync()
        return time.perf_counter() - t0

    share, fork = tune_schedule(ctx, a, run, 200 * ntot, "ensemble")
    for c, cr in zip(cs, crs):
        c.set_state(cr.pos, cr.vel, 0)
    native.step_batch(cs, [a.warmup] * len(cs))
    ctx.synchronize()
    sync()
    t0 = time.perf_counter()
    native.step_batch(cs, [a.steps] * len(cs))
    ctx.synchronize()
    sync()
    el = time.perf_counter() - t0
    # per-phase times from a few more, instrumented steps (the events of every
    # TIMING_EVERY-th evaluation, as for config 3), outside the timed region
    ctx.set_timing(True, every=TIMING_EVERY)
    native.step_batch(cs, [2 * TIMING_EVERY] * len(cs))
    sync()
    phases = ctx.phase_times()
    ctx.set_timing(False)
    value = ntot * a.steps / el
    stats = ctx.step_stats()
    log(f"  {a.steps} batched steps in {el * 1e3:.1f} ms -> {value:.4g} ion-steps/s; max rms err {max(errs):.2e}; "
        f"step evaluations so far {stats}")
    return {
        "metric": "ensemble ion-steps/s (256 crystals, N log-uniform 100..20000, one launch per phase per step)",
        "value": value, "unit": "ion-steps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": el * 1e3 / a.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if a.precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": f"{len(crs)} crystals, {ntot} ions, spheres at 1000 ions/(100 um)^3, B~U[2,5] T, "
                               f"f_z~U[1,2] MHz, photon mean~U[0,0.05], FMM p={a.p} leaf {a.leaf} ({a.precision})",
                   "crystals": len(crs), "ions": ntot, "p": a.p, "leaf_size": a.leaf, "near_share": share,
                   "fork": fork,
                   "max_rms_rel_force_err_largest3": max(errs)},
        "details": {"phase_ms": {k: float(v) for k, v in zip(PHASES, phases)}, "step_evaluations": stats},
    }


def bench_scaling(a, ctx, sync):
    """Step time against N (the paper's scaling study, Sec. 3: ions uniform in a
    sphere at one density for every N, initial velocities zero): FMM steps
    (mixed, p and leaf as given, default 11 and 256) and direct-sum steps, with
    the FMM's RMS force error against the FP64 direct sum."""
    p, leaf = a.p or 11, a.leaf or 256
    points = []
    for k, n in enumerate((1000, 10000, 100000, 1000000)):
        pos = inputs.uniform_ball(n, inputs.density_radius(n), inputs.rng(20 + k))
        vel = np.zeros_like(pos)
        c = ctx.crystal(pos, vel, inputs.ION_CHARGE, inputs.ION_MASS, 20 + k)
        c.set_force("direct")
        t0 = time.perf_counter()
        F_dir = c.compute_forces()
        dir_eval = time.perf_counter() - t0
        dir_steps = 3 if n <= 100000 else 0
        dir_ms = None
        if dir_steps:
            c.step(1)
            sync()
            t0 = time.perf_counter()
            c.step(dir_steps)
            sync()
            dir_ms = (time.perf_counter() - t0) * 1e3 / dir_steps
        c.set_state(pos, vel, 0)
        c.set_force("fmm", p, leaf, a.precision)
        err = rms_rel(c.compute_forces(), F_dir)
        el = timed_steps(ctx, c, a.steps, a.warmup, sync, phases_too=False)[0]
        c.destroy()
        fmm_ms = el * 1e3 / a.steps
        log(f"  N={n}: FMM {fmm_ms:.3f} ms/step (rms err {err:.2e}), direct "
            f"{'%.3f ms/step' % dir_ms if dir_ms else '-'} (one direct force evaluation {dir_eval * 1e3:.1f} ms wall)")
        points.append({"n_ions": n, "fmm_ms_per_step": fmm_ms, "fmm_ion_steps_per_s": n / (fmm_ms * 1e-3),
                       "rms_rel_force_err": err, "direct_ms_per_step": dir_ms,
                       "direct_eval_ms_wall": dir_eval * 1e3})
    # growth over the top decade (1e5 -> 1e6); below ~1e5 ions neither path fills
    # the GPU (the direct sum has N/512 workgroups; the FMM step's fixed launch
    # and read-back costs, ~0.25 ms, dominate below 1e4), so smaller N understate it
    hi, lo = points[-1], points[-2]
    dec = math.log(hi["n_ions"] / lo["n_ions"])
    slope = math.log(hi["fmm_ms_per_step"] / lo["fmm_ms_per_step"]) / dec
    dslope = math.log(hi["direct_eval_ms_wall"] / lo["direct_eval_ms_wall"]) / dec
    log(f"  growth exponent of the step time, 1e5 -> 1e6 ions: FMM {slope:.2f}, direct force evaluation {dslope:.2f}")
    return {"metric": "scaling: step time vs N at fixed density (uniform sphere, zero initial velocity)",
            "value": points[-1]["fmm_ion_steps_per_s"], "unit": "ion-steps/s", "n_gpus": 1, "steps": a.steps,
            "warmup": a.warmup, "ms_per_step": points[-1]["fmm_ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64" if a.precision == "mixed" else "f64",
            "data": "synthetic",
            "config": {"workload": f"uniform spheres at 1000 ions per (100 um)^3, N = 1e3..1e6, FMM p={p} leaf {leaf} "
                                   f"({a.precision}), B=4.5 T, f_z=1.5 MHz, dt=1 ns", "p": p, "leaf_size": leaf},
            "points": points, "fmm_exponent_1e5_1e6": slope, "direct_exponent_1e5_1e6": dslope,
            "note": "exponents over the top decade; below ~1e5 ions neither path fills the GPU"}


def bench_serving(a, ctx, sync):
    """Serving stream: Poisson arrivals, continuous batching, admission by HBM footprint."""
    from paper_2405_13973_amd import serving

    reqs = inputs.serving_stream(count=a.requests, rate_hz=50.0, seed=5)
    offered = sum(r.crystal.n * r.steps for r in reqs) / max(r.arrival_s for r in reqs)
    log(f"serving: {len(reqs)} requests over {max(r.arrival_s for r in reqs):.1f} s, offered "
        f"{offered:.3g} ion-steps/s")
    # p from the error bound on the three largest requests (leaf 256 unless given)
    big = sorted(reqs, key=lambda r: -r.crystal.n)[:3]
    probe = [ctx.crystal(r.crystal.pos, r.crystal.vel, r.crystal.charge, r.crystal.mass, r.crystal.seed) for r in big]
    a.leaf, a.p, errs = tune_batch(ctx, probe, (a.leaf or SERVING_LEAF,), a.p, a.p0, a.precision, sync, time_it=False)
    for c in probe:
        c.destroy()
    srv = serving.Server(ctx, native, budget_bytes=a.budget_gb << 30, precision=a.precision, p=a.p, leaf=a.leaf,
                         chunk=a.chunk)
    rep = srv.run(reqs)
    p50, p99 = rep.latency_percentiles()
    log(f"  done in {rep.wall_s:.1f} s: {rep.ion_steps_per_s:.4g} ion-steps/s, latency p50 {p50:.2f} s "
        f"p99 {p99:.2f} s, max resident {rep.max_resident}")
    return {
        "metric": "serving: aggregate ion-steps/s with p50/p99 request latency (Poisson 50/s, N 200..50000, "
                  "K 100..2000)",
        "value": rep.ion_steps_per_s, "unit": "ion-steps/s", "n_gpus": 1, "steps": None, "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if a.precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": f"{len(reqs)} requests, Poisson arrivals 50/s, N log-uniform [200, 50000], "
                               f"K ~ U{{100..2000}}, photon mean 0.01, FMM p={a.p} leaf {a.leaf} ({a.precision}), "
                               f"tick {a.chunk} steps, budget {a.budget_gb} GiB",
                   "requests": len(reqs), "p": a.p, "leaf_size": a.leaf,
                   "max_rms_rel_force_err_largest3": max(errs)},
        "latency_s": {"p50": p50, "p99": p99},
        "details": {"offered_ion_steps_per_s": offered, "achieved_ion_steps_per_s": rep.ion_steps_per_s,
                    "wall_s": rep.wall_s, "max_resident": rep.max_resident,
                    "max_resident_bytes": rep.max_resident_bytes,
                    "note": "offered load above achieved: p99 is queue-dominated"
                    if offered > rep.ion_steps_per_s else "offered load below achieved",
                    # rotating-frame temperatures of the finished crystals (eqs. temp_ax, temp_pl,
                    # instantaneous), from the server's batched end-of-request diagnostics
                    "final_temp_axial_K_median": float(np.median([d.diagnostics["temp_axial"] for d in rep.done])),
                    "final_temp_planar_K_median": float(np.median([d.diagnostics["temp_planar"] for d in rep.done]))},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--leaf", type=int, default=0,
                    help="leaf size (0: tuned; serving: 256)")
    ap.add_argument("--p0", type=int, default=10, help="first p tried when choosing p")
    ap.add_argument("--near-share", type=int, default=-1,
                    help="near-field workgroups per compute unit beside the far field (-1: tuned; 0: default)")
    ap.add_argument("--fork", type=int, default=-2,
                    help="branch that keeps the stream at an early fork (1 near field, 0 far field, -1 by the "
                         "measured balance; -2: tuned with the share, or -1 when --near-share is given)")
    ap.add_argument("--n", type=int, default=100000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-potential", action="store_true", help="skip the Coulomb-potential measurement")
    ap.add_argument("--no-beams", action="store_true", help="skip the beam-mode laser measurement")
    ap.add_argument("--no-diagnostics", action="store_true", help="skip the rotating-frame diagnostics measurement")
    ap.add_argument("--no-relaxation", action="store_true", help="skip the artificial-damping relaxation")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the 256-crystal ensemble leg (config 4)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-stream leg (config 5)")
    ap.add_argument("--serving-requests", type=int, default=120,
                    help="requests of the serving leg of the default run (the first ones of the config-5 stream)")
    ap.add_argument("--workload", choices=["config3", "ensemble", "serving", "scaling"], default="config3",
                    help="config3: 1e5-ion crystal (default); ensemble: 256 crystals batched; serving: request stream; "
                         "scaling: step time against N")
    ap.add_argument("--p", type=int, default=0,
                    help="expansion degree for the ensemble / serving workloads (0: smallest meeting the bound)")
    ap.add_argument("--crystals", type=int, default=256)
    ap.add_argument("--requests", type=int, default=500)
    ap.add_argument("--chunk", type=int, default=50, help="serving: steps per tick")
    ap.add_argument("--budget-gb", type=int, default=64, help="serving: HBM budget for resident crystals")
    ap.add_argument("--roofline", choices=["auto", "m2l", "p2p"], default="auto",
                    help="kernel of the roofline entry (auto: the longer of the two in the timed region)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run one plain device copy of MIB MiB first (reference kernel for HBM byte counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the multi-GPU sharding is a "
              f"design note, not a measured path.", file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "no HIP device visible"
    stream = torch.cuda.current_stream()
    sync = torch.cuda.synchronize

    if a.copy_calibration:
        src = torch.empty(a.copy_calibration * (1 << 20) // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        sync()
        dst.copy_(src)
        sync()
        log(f"  copy calibration: {a.copy_calibration} MiB read + {a.copy_calibration} MiB written")
        del src, dst

    if a.workload != "config3":
        ctx = native.Context(0, hbm_budget=(a.budget_gb << 30) + (4 << 30), stream=stream.cuda_stream)
        out = {"ensemble": bench_ensemble, "serving": bench_serving, "scaling": bench_scaling}[a.workload](a, ctx, sync)
        ctx.close()
        print(json.dumps(out), flush=True)
        return

    cr = inputs.config3(n=a.n)
    log(f"workload: {cr.n} ions, jittered lattice in ellipsoid (400,400,800) um")
    ctx = native.Context(0, stream=stream.cuda_stream)
    c = ctx.crystal(cr.pos, cr.vel, cr.charge, cr.mass, cr.seed)
    c.set_trap(B=cr.B, omega_z=cr.omega_z, dt=cr.dt)
    c.set_force("direct")
    F_dir = c.compute_forces()

    def tune(prec, leaves):
        """Smallest p meeting the error bound per leaf size, then the fastest."""
        best = None
        for leaf in leaves:
            c.set_state(cr.pos, cr.vel, 0)  # F_dir belongs to the initial positions
            p, err, _ = choose_p(c, F_dir, prec, leaf, a.p0)
            el = 0.0
            if len(leaves) > 1:
                c.set_force("fmm", p, leaf, prec)
                el = timed_steps(ctx, c, 10, 2, sync, phases_too=False)[0]
                log(f"  {prec} leaf {leaf}: p={p} {10 * cr.n / el:.4g} ion-steps/s")
            if best is None or el < best[3]:
                best = (leaf, p, err, el)
        return best[:3]

    def tune_share(prec, leaf, p):
        """Near-field workgroups per compute unit beside the far field and the
        fork direction (schedule parameters, no effect on the results): the
        fastest of the candidates over three runs of 20 steps each, unless
        given."""
        def run(share, fork):
            c.set_state(cr.pos, cr.vel, 0)
            c.set_force("fmm", p, leaf, prec)
            return min(timed_steps(ctx, c, 20, 2, sync, phases_too=False)[0] for _ in range(3))

        share, fork = tune_schedule(ctx, a, run, 20 * cr.n, f"{prec} leaf {leaf}")
        return share, fork

    results = {}
    forms = [a.precision] + ([] if a.no_fp64_compare or a.precision == "fp64" else ["fp64"])
    for prec in forms:
        # each form at its own best leaf size (the same candidates, the same bound)
        leaves = (a.leaf,) if a.leaf else LEAF_CANDIDATES
        leaf, p, err = tune(prec, leaves)
        share, fork = tune_share(prec, leaf, p)
        c.set_state(cr.pos, cr.vel, 0)
        c.set_force("fmm", p, leaf, prec)
        sync()
        el, phases, count, wc, plain = timed_steps(ctx, c, a.steps, a.warmup, sync)
        # the accuracy bound on the state the timed steps ended on (the crystal
        # expands from its initial lattice, so its tree changes while timed)
        c.set_force("direct")
        F_end = c.compute_forces()
        c.set_force("fmm", p, leaf, prec)
        err_end = rms_rel(c.compute_forces(), F_end)
        results[prec] = dict(p=p, leaf=leaf, share=share, fork=fork, err=err, err_end=err_end, seconds=el, phases=phases,
                             count=count, wc=wc, plain=plain)
        log(f"  {prec}: p={p} leaf={leaf} {a.steps} steps in {plain * 1e3:.2f} ms -> {cr.n * a.steps / plain:.4g} "
            f"ion-steps/s (with phase events {el * 1e3:.2f} ms); rms err start {err:.2e} end {err_end:.2e}; "
            f"phases(ms) " + " ".join(f"{k} {v:.3f}" for k, v in zip(PHASES, phases)) + f" over {count} evals")

    # direct-sum rate on the same crystal, for the FMM/direct comparison and
    # the direct kernel's own roofline (mean of three evaluations)
    c.set_force("direct")
    ctx.set_timing(True)
    dir_runs = []
    for _ in range(3):
        c.compute_forces()
        dir_runs.append(ctx.phase_times()[6])
    dir_ms = float(np.mean(dir_runs))
    ctx.set_timing(False)

    main_r = results[a.precision]
    p, leaf = main_r["p"], main_r["leaf"]
    ctx.set_near_share(main_r["share"])  # the legs on the same crystal below
    ctx.set_fork(main_r["fork"])
    K = (p + 1) ** 2
    ph = main_r["phases"]
    fp32 = a.precision == "mixed"
    m2l_tflops = 2.0 * K * K * main_r["wc"][2] / (ph[2] * 1e-3) / 1e12
    p2p_tflops = P2P_FLOPS_PER_PAIR * main_r["wc"][3] / (ph[4] * 1e-3) / 1e12
    rooflines = {
        "m2l": {"bound": "mfma", "kernel": "m2l", "kernel_ms": float(ph[2]), "achieved": m2l_tflops,
                "peak": PEAK["mfma_fp32" if fp32 else "mfma_fp64"], "unit": "TFLOP/s",
                "traffic": measured_traffic("m2l", p, leaf, a.precision, cr.n),
                "algorithmic": f"2 K^2 flops per M2L pair, K=(p+1)^2={K}, {int(main_r['wc'][2])} pairs per launch"},
        "p2p": {"bound": "alu", "kernel": "p2p", "kernel_ms": float(ph[4]), "achieved": p2p_tflops,
                "peak": PEAK["valu_fp32" if fp32 else "valu_fp64"], "unit": "TFLOP/s",
                "traffic": measured_traffic("p2p", p, leaf, a.precision, cr.n),
                "algorithmic": f"{P2P_FLOPS_PER_PAIR} flops per near-field pair (the kernel issues "
                               f"{P2P_ISSUED_FLOPS_PER_PAIR}), {int(main_r['wc'][3])} ordered pairs (i != j) per launch",
                "issued_achieved": P2P_ISSUED_FLOPS_PER_PAIR * main_r["wc"][3] / (ph[4] * 1e-3) / 1e12},
    }
    for r in rooflines.values():
        r["frac"] = r["achieved"] / r["peak"]
    # the dominant kernel: the longer of the two, by its measured time in the
    # timed region (or the one asked for)
    kernel = a.roofline if a.roofline != "auto" else max(rooflines, key=lambda k: rooflines[k]["kernel_ms"])
    # the exact direct sum (not part of the FMM step): both of its kernels
    dir_pairs = float(cr.n) * (cr.n - 1)
    rooflines["direct"] = {
        "bound": "alu", "kernel": "direct", "kernel_ms": dir_ms,
        "achieved": P2P_FLOPS_PER_PAIR * dir_pairs / (dir_ms * 1e-3) / 1e12, "peak": PEAK["valu_fp64"],
        "unit": "TFLOP/s", "traffic": measured_traffic("direct", p, leaf, a.precision, cr.n),
        "algorithmic": f"{P2P_FLOPS_PER_PAIR} flops per ordered pair (i != j), {int(dir_pairs)} pairs per evaluation "
                       f"(FP64, the chunk sums and their reduction)"}
    rooflines["direct"]["frac"] = rooflines["direct"]["achieved"] / rooflines["direct"]["peak"]
    log(f"  direct sum: {dir_ms:.3f} ms per evaluation, {rooflines['direct']['achieved']:.1f} TFLOP/s "
        f"({100 * rooflines['direct']['frac']:.1f}% of the FP64 vector peak)")
    # the library's throughput: the timed steps without phase events (the
    # instrumented run of the same steps gives the phases and the rooflines)
    value = cr.n * a.steps / main_r["plain"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "ion-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": main_r["plain"] * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if fp32 else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{cr.n} ions, 5%-jittered cubic lattice in a (400,400,800) um prolate ellipsoid, "
                        f"B=4.5 T, f_z=1.5 MHz, dt=1 ns, FMM p={p} leaf {leaf} ({a.precision})",
            "n_ions": cr.n, "p": p, "leaf_size": leaf, "precision": a.precision, "near_share": main_r["share"],
            "fork": main_r["fork"],
            "rms_rel_force_err": main_r["err"], "rms_rel_force_err_after_timed_steps": main_r["err_end"],
        },
        "roofline": rooflines[kernel],
        "details": {
            "force_evals_per_s": 1e3 / ph[6],
            "phase_ms": {k: float(v) for k, v in zip(PHASES, ph)},
            "rooflines": rooflines,
            "ms_per_step_with_phase_events": main_r["seconds"] * 1e3 / a.steps,
            "direct_sum_ms": float(dir_ms),
            "boxes": int(main_r["wc"][0]), "leaves": int(main_r["wc"][1]), "m2l_pairs": int(main_r["wc"][2]),
            "p2p_pairs": int(main_r["wc"][3]),
            "m2l_tflops": m2l_tflops,
            "p2p_pairs_per_s": main_r["wc"][3] / (ph[4] * 1e-3),
        },
    }
    if "fp64" in results and a.precision == "mixed":
        f = results["fp64"]
        out["details"]["fp64_ion_steps_per_s"] = cr.n * a.steps / f["plain"]
        out["details"]["fp64_p"] = f["p"]
        out["details"]["fp64_leaf_size"] = f["leaf"]
        out["details"]["fp64_near_share"] = f["share"]
        out["details"]["fp64_fork"] = f["fork"]
        out["details"]["fp64_rms_rel_force_err"] = f["err"]
        out["details"]["fp64_rms_rel_force_err_after_timed_steps"] = f["err_end"]
        out["details"]["mixed_speedup_vs_fp64"] = f["plain"] / main_r["plain"]
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cr, p, leaf, F_dir)
        out["details"]["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
    if not a.no_beams:
        out["beams"] = bench_beams(ctx, c, cr, p, leaf, a.precision, a.steps, a.warmup, sync, main_r["plain"])
    if not a.no_potential:
        out["potential"] = bench_potential(ctx, c, cr, p, leaf, a.precision)
    if not a.no_diagnostics:
        out["diagnostics"] = bench_diagnostics(ctx, c, cr, p, leaf, a.precision, sync)
    if not a.no_relaxation:
        out["relaxation"] = bench_relaxation(ctx, a.precision, sync)
    if "cpu_baseline" in out and "potential" in out:
        out["potential"]["gpu_over_cpu"] = (out["potential"]["ion_evals_per_s"] /
                                            out["cpu_baseline"]["potential_ion_evals_per_s"])
    c.destroy()
    # the batched workloads run in a context of their own (as with --workload);
    # serving keeps the schedule the ensemble tuner set on it
    ctx.close()
    ctx = native.Context(0, hbm_budget=(a.budget_gb << 30) + (4 << 30), stream=stream.cuda_stream)
    if not a.no_ensemble:
        e = argparse.Namespace(**vars(a))
        e.steps, e.warmup, e.leaf, e.p = ENSEMBLE_STEPS, 3, SERVING_LEAF, 0
        out["ensemble"] = bench_ensemble(e, ctx, sync)
    if not a.no_serving:
        s_ = argparse.Namespace(**vars(a))
        s_.requests, s_.leaf, s_.p = a.serving_requests, SERVING_LEAF, 0
        out["serving"] = bench_serving(s_, ctx, sync)
        out["latency_s"] = out["serving"]["latency_s"]
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

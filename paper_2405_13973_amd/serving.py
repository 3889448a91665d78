"""Continuous-batching server for crystal-simulation requests.

Requests (a crystal and a number of steps) arrive over time.  Each tick the
server admits waiting requests while the device memory they would take fits the
budget -- their own state plus the growth of the shared batch workspace, from
the context's measured memory and a per-ion workspace rate that starts from an
estimate for the expansion degree and leaf size and follows the measured
high-water mark.  The estimate can fall short; the context's own HBM budget is
the hard limit: a tick that runs out of it (PT_ENOMEM, which leaves every
crystal at its last completed step) sends the newest request that has not
stepped yet back to the head of the queue, raises the rate and runs again.
Then it advances every resident crystal by up to `chunk` steps in one
pt_step_batch call -- every phase of a step is one launch for all resident
crystals, whatever their sizes -- and retires the finished ones.  A request's
state stays in HBM from admission to completion.  Results do not depend on
which other requests share a tick (every kernel is batch invariant), so a
request run alone or in the mix ends in the same state, bit for bit.

The stepping backend is the C ABI binding (`native`); a stand-in with the
same methods can be passed for host-only tests of the scheduling logic.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

# Device bytes a resident crystal owns: FP64 positions and velocities (48 per
# ion), the photon counts (4 per ion) and a status word.
STATE_BYTES_PER_ION = 52
STATE_BYTES_FIXED = 16


def state_bytes(n_ions: int) -> int:
    return STATE_BYTES_FIXED + STATE_BYTES_PER_ION * int(n_ions)


def workspace_bytes_per_ion(p: int, leaf: int, precision: str) -> float:
    """Estimate of the batch workspace per ion of the FMM step: per ion the sort
    keys and values, tree scratch, sorted positions, field and working state
    (about 200 B); per box (about 3.5 boxes per leaf-size ions) the box table,
    colleague, window and near lists (about 2.4 kB), 10 expansion rows of
    (p+1)^2 coefficients padded to 16 (M, L and the translation partial sums)
    and one row per M2L pair (about 150 pairs per box); 25 % on top for the
    workspace's growth rule."""
    kp = ((p + 1) ** 2 + 15) // 16 * 16
    esz = 4 if precision == "mixed" else 8
    per_box = 2400 + (10 + 150) * kp * esz
    return 1.25 * (200 + 3.5 / max(1, leaf) * per_box)


def footprint(n_ions: int, p: int = 11, leaf: int = 32, precision: str = "mixed") -> int:
    """Estimated device bytes a request of n_ions adds while resident: its state
    plus its share of the batch workspace."""
    return state_bytes(n_ions) + int(workspace_bytes_per_ion(p, leaf, precision) * n_ions)


@dataclasses.dataclass
class Done:
    index: int
    n_ions: int
    steps: int
    arrival_s: float
    admit_s: float
    finish_s: float
    pos: np.ndarray
    vel: np.ndarray
    photons: np.ndarray
    diagnostics: dict | None = None  # rotating-frame energies and temperatures at the end

    @property
    def latency_s(self) -> float:
        return self.finish_s - self.arrival_s


@dataclasses.dataclass
class Report:
    done: list
    wall_s: float
    ion_steps: int
    max_resident: int
    max_resident_bytes: int

    def latency_percentiles(self):
        lat = np.array([d.latency_s for d in self.done])
        return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))

    @property
    def ion_steps_per_s(self) -> float:
        return self.ion_steps / self.wall_s if self.wall_s > 0 else 0.0


class Server:
    def __init__(self, ctx, native_mod, budget_bytes: int, precision: str = "mixed", p: int = 11, leaf: int = 32,
                 chunk: int = 50, clock=time.perf_counter, sleep=time.sleep):
        self.ctx, self.native = ctx, native_mod
        self.budget = int(budget_bytes)
        self.force = ("fmm", p, leaf, precision)
        self.chunk = int(chunk)
        self.clock, self.sleep = clock, sleep
        # workspace bytes per resident ion: the estimate, raised to the measured
        # high-water mark after every tick
        self.ws_rate = workspace_bytes_per_ion(p, leaf, precision)
        self.requeued = 0  # admissions undone after the context ran out of memory

    def _projected(self, base, resident_ions, resident_state, n_new):
        """Device bytes in use if a request of n_new ions joined the residents:
        memory in use now, its state, and the workspace growth the larger batch
        would need beyond the workspace already held."""
        used = self.ctx.memory()[0]
        ws_now = max(0, used - base - resident_state)
        ws_need = self.ws_rate * (resident_ions + n_new)
        return used + state_bytes(n_new) + max(0.0, ws_need - ws_now)

    def _admit(self, req):
        cr = req.crystal
        c = self.ctx.crystal(cr.pos, cr.vel, cr.charge, cr.mass, cr.seed)
        c.set_trap(B=cr.B, omega_z=cr.omega_z, delta=cr.delta, omega_r=cr.omega_r, dt=cr.dt)
        c.set_laser(cr.photon_mean)
        c.set_force(*self.force)
        return c

    def run(self, requests, time_scale: float = 1.0) -> Report:
        """Serve `requests` (objects with arrival_s, crystal, steps) in real time;
        arrival times are multiplied by time_scale."""
        order = sorted(range(len(requests)), key=lambda i: requests[i].arrival_s)
        pending = collections.deque(order)
        waiting = collections.deque()
        active = []  # [index, crystal, remaining, admit_s, step at admission]
        done = []
        ion_steps = 0
        max_res = max_bytes = 0
        base = self.ctx.memory()[0]  # held before the first admission (tables of earlier use, flags)
        t0 = self.clock()
        while pending or waiting or active:
            now = self.clock() - t0
            while pending and requests[pending[0]].arrival_s * time_scale <= now:
                waiting.append(pending.popleft())
            while waiting:
                i = waiting[0]
                n_new = requests[i].crystal.n
                res_ions = sum(a[1].n for a in active)
                res_state = sum(state_bytes(a[1].n) for a in active)
                if active and self._projected(base, res_ions, res_state, n_new) > self.budget:
                    break  # wait for memory to free up
                try:
                    c = self._admit(requests[i])
                except self.native.PTError as e:
                    if e.code == self.native.PT_ENOMEM and active:
                        break
                    raise
                waiting.popleft()
                active.append([i, c, requests[i].steps, now, 0])  # index, crystal, remaining, admit time, step0
            max_res = max(max_res, len(active))
            if not active:
                if pending:
                    wait = requests[pending[0]].arrival_s * time_scale - (self.clock() - t0)
                    if wait > 0:
                        self.sleep(min(wait, 0.05))
                continue
            n = [min(a[2], self.chunk) for a in active]
            try:
                self.native.step_batch([a[1] for a in active], n)
            except self.native.PTError as e:
                if e.code != self.native.PT_ENOMEM:
                    raise
                # every crystal stands at its last completed step: count them
                for a in active:
                    done_now = a[1].read_state()["step"] - a[4]
                    ion_steps += (done_now - (requests[a[0]].steps - a[2])) * a[1].n
                    a[2] = requests[a[0]].steps - done_now
                fresh = [a for a in active if a[2] == requests[a[0]].steps]
                if len(active) == 1 or not fresh:
                    raise
                back = fresh[-1]
                active.remove(back)
                back[1].destroy()
                waiting.appendleft(back[0])
                self.ws_rate *= 1.25
                self.requeued += 1
                continue
            self.ctx.synchronize()
            used = self.ctx.memory()[0]
            max_bytes = max(max_bytes, used)
            res_ions = sum(a[1].n for a in active)
            ws = used - base - sum(state_bytes(a[1].n) for a in active)
            if res_ions:
                self.ws_rate = max(self.ws_rate, ws / res_ions)
            for a, k in zip(active, n):
                a[2] -= k
                ion_steps += k * a[1].n
            still = []
            finished = [a for a in active if a[2] <= 0]
            # rotating-frame energies and temperatures of the finished crystals,
            # one batched evaluation (sums on the device; eqs. pe_rot, temp_ax, temp_pl)
            diags = self.native.rotating_diagnostics_batch([a[1] for a in finished]) if finished else []
            diag_of = {id(a): d for a, d in zip(finished, diags)}
            max_bytes = max(max_bytes, self.ctx.memory()[0])
            for a in active:
                if a[2] > 0:
                    still.append(a)
                    continue
                st = a[1].read_state()
                fin = self.clock() - t0
                req = requests[a[0]]
                done.append(Done(a[0], a[1].n, req.steps, req.arrival_s * time_scale, a[3], fin, st["pos"], st["vel"],
                                 st["photons"], diag_of[id(a)]))
                a[1].destroy()
            active = still
        return Report(done, self.clock() - t0, ion_steps, max_res, max_bytes)


def run_alone(ctx, native_mod, req, precision="mixed", p=11, leaf=32):
    """The same request stepped on its own (reference for the alone-vs-mix check)."""
    cr = req.crystal
    c = ctx.crystal(cr.pos, cr.vel, cr.charge, cr.mass, cr.seed)
    c.set_trap(B=cr.B, omega_z=cr.omega_z, delta=cr.delta, omega_r=cr.omega_r, dt=cr.dt)
    c.set_laser(cr.photon_mean)
    c.set_force("fmm", p, leaf, precision)
    c.step(req.steps)
    st = c.read_state()
    c.destroy()
    return st

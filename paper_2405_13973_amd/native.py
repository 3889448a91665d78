"""ctypes binding of libpenning's C ABI (include/penning.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  ``load()`` raises if the library has not been built; nothing here
falls back to a CPU implementation.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpenning.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "penning.h")

PT_OK, PT_EINVAL, PT_ENOMEM, PT_EDEVICE, PT_ENUMERIC, PT_EBUSY = 0, -1, -2, -3, -4, -5
_NAMES = {0: "PT_OK", -1: "PT_EINVAL", -2: "PT_ENOMEM", -3: "PT_EDEVICE", -4: "PT_ENUMERIC", -5: "PT_EBUSY"}


class PTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class TrapParams(C.Structure):
    _fields_ = [("B_T", C.c_double), ("omega_z", C.c_double), ("delta", C.c_double), ("omega_r", C.c_double),
                ("dt_s", C.c_double), ("t0_s", C.c_double), ("damping_per_s", C.c_double)]


class Beam(C.Structure):
    _fields_ = [("khat", C.c_double * 3), ("detuning", C.c_double), ("s0", C.c_double), ("waist_y", C.c_double),
                ("waist_z", C.c_double), ("offset_y", C.c_double), ("uniform", C.c_int)]


MAX_BEAMS = 4


class LaserParams(C.Structure):
    _fields_ = [("mode", C.c_int), ("mean_per_step", C.c_double), ("wavelength_m", C.c_double),
                ("gamma0", C.c_double), ("n_beams", C.c_int), ("beam", Beam * MAX_BEAMS)]


class Diagnostics(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("t", "ke_axial", "ke_planar", "pe_external", "pe_coulomb", "energy",
                                          "temp_axial", "temp_planar")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ForceParams(C.Structure):
    _fields_ = [("method", C.c_int), ("p", C.c_int), ("leaf_size", C.c_int), ("precision", C.c_int)]


_lib = None
_vp = C.c_void_p
_dp = C.POINTER(C.c_double)


def header_functions():
    """Names of the functions declared in include/penning.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(pt_[a-z_0-9]+)\s*\(", txt)))


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2405_13973_amd.build`")
    L = C.CDLL(LIB_PATH)
    sig = {
        "pt_ctx_create": [C.c_int, C.c_uint64, _vp, C.POINTER(_vp)],
        "pt_ctx_destroy": [_vp],
        "pt_ctx_memory": [_vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)],
        "pt_create_crystal": [_vp, C.c_int64, _dp, _dp, C.c_double, C.c_double, C.c_uint64, C.POINTER(_vp)],
        "pt_create_crystal_device": [_vp, C.c_int64, _vp, _vp, C.c_double, C.c_double, C.c_uint64, C.POINTER(_vp)],
        "pt_destroy_crystal": [_vp],
        "pt_set_trap_params": [_vp, C.POINTER(TrapParams)],
        "pt_set_laser_params": [_vp, C.POINTER(LaserParams)],
        "pt_set_force_params": [_vp, C.POINTER(ForceParams)],
        "pt_set_state": [_vp, _dp, _dp, C.c_int64],
        "pt_compute_forces": [_vp, _dp],
        "pt_compute_forces_batch": [C.POINTER(_vp), C.c_int, C.POINTER(_dp)],
        "pt_compute_forces_noalloc": [_vp, _vp],
        "pt_compute_potential": [_vp, _dp],
        "pt_compute_potential_batch": [C.POINTER(_vp), C.c_int, C.POINTER(_dp)],
        "pt_coulomb_energy": [_vp, _dp],
        "pt_coulomb_energy_batch": [C.POINTER(_vp), C.c_int, _dp],
        "pt_rotating_diagnostics": [_vp, C.POINTER(Diagnostics)],
        "pt_rotating_diagnostics_batch": [C.POINTER(_vp), C.c_int, C.POINTER(Diagnostics)],
        "pt_read_rotating_state": [_vp, _dp, _dp],
        "pt_step": [_vp, C.c_int64],
        "pt_step_batch": [C.POINTER(_vp), C.c_int, C.POINTER(C.c_int64)],
        "pt_synchronize": [_vp],
        "pt_read_state": [_vp, _dp, _dp, C.POINTER(C.c_int64), _dp, C.POINTER(C.c_int32)],
        "pt_debug_export_tree": [_vp, C.POINTER(C.c_int64)] + [_vp] * 13,
        "pt_ctx_set_timing": [_vp, C.c_int],
        "pt_ctx_set_near_share": [_vp, C.c_int],
        "pt_ctx_set_fork": [_vp, C.c_int],
        "pt_ctx_phase_times": [_vp, _dp, C.POINTER(C.c_int64)],
        "pt_ctx_work_counts": [_vp, C.POINTER(C.c_int64)],
        "pt_ctx_step_stats": [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.pt_last_error.argtypes = []
    L.pt_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(rc):
    if rc != PT_OK:
        raise PTError(rc, load().pt_last_error().decode())


def _ptr(a, ctype=C.c_double):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


def _xyz(a, n):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(n, 3))
    return a


class Context:
    """One HIP device + stream (pass a hipStream_t handle, e.g.
    torch.cuda.current_stream().cuda_stream, or None for the library's own)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, stream: int | None = None):
        L = load()
        h = _vp()
        _check(L.pt_ctx_create(int(device), int(hbm_budget), _vp(stream) if stream else None, C.byref(h)))
        self.h = h
        self.crystals = []

    def crystal(self, pos, vel, charge, mass, seed=0) -> "Crystal":
        pos = np.asarray(pos, dtype=np.float64)
        n = len(pos)
        p, v = _xyz(pos, n), _xyz(vel, n)
        h = _vp()
        _check(load().pt_create_crystal(self.h, n, _ptr(p), _ptr(v), float(charge), float(mass), int(seed),
                                        C.byref(h)))
        c = Crystal(self, h, n)
        self.crystals.append(c)
        return c

    def crystal_from_device(self, pos_ptr: int, vel_ptr: int, n: int, charge, mass, seed=0) -> "Crystal":
        h = _vp()
        _check(load().pt_create_crystal_device(self.h, int(n), _vp(pos_ptr), _vp(vel_ptr), float(charge),
                                               float(mass), int(seed), C.byref(h)))
        c = Crystal(self, h, n)
        self.crystals.append(c)
        return c

    def memory(self):
        used, budget = C.c_uint64(), C.c_uint64()
        _check(load().pt_ctx_memory(self.h, C.byref(used), C.byref(budget)))
        return used.value, budget.value

    def set_timing(self, on, every: int = 1):
        """Phase timing on (the events of every `every`-th evaluation) or off."""
        _check(load().pt_ctx_set_timing(self.h, int(every) if on else 0))

    def phase_times(self, with_count=False):
        """Mean per-evaluation phase times (ms) since set_timing(True): sort+tree+lists
        (with P2M beside them), M2M, M2L kernel, M2L reduce+L2L, P2P kernel, L2P+partials,
        total."""
        ms = np.zeros(7)
        cnt = C.c_int64()
        _check(load().pt_ctx_phase_times(self.h, _ptr(ms), C.byref(cnt)))
        return (ms, cnt.value) if with_count else ms

    def set_near_share(self, per_cu):
        """Near-field workgroups per compute unit beside the far field (0: default)."""
        _check(load().pt_ctx_set_near_share(self.h, int(per_cu)))

    def set_fork(self, mode):
        """Branch that keeps the stream at an early fork: 1 the near field, 0 the
        far field, -1 by the measured balance (the default)."""
        _check(load().pt_ctx_set_fork(self.h, int(mode)))

    def work_counts(self):
        c = np.zeros(6, np.int64)
        _check(load().pt_ctx_work_counts(self.h, _ptr(c, C.c_int64)))
        return c

    def step_stats(self):
        """FMM step evaluations queued on capacities, measured, and queued runs re-run."""
        q, m, r = C.c_int64(), C.c_int64(), C.c_int64()
        _check(load().pt_ctx_step_stats(self.h, C.byref(q), C.byref(m), C.byref(r)))
        return dict(queued=q.value, measured=m.value, reruns=r.value)

    def synchronize(self):
        _check(load().pt_synchronize(self.h))

    def close(self):
        if self.h:
            for c in list(self.crystals):
                c.destroy()
            _check(load().pt_ctx_destroy(self.h))
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Crystal:
    def __init__(self, ctx: Context, h, n: int):
        self.ctx, self.h, self.n = ctx, h, n

    def set_trap(self, B=4.5, omega_z=2 * np.pi * 1.5e6, delta=0.0, omega_r=0.0, dt=1e-9, t0=0.0, damping=0.0):
        p = TrapParams(B, omega_z, delta, omega_r, dt, t0, damping)
        _check(load().pt_set_trap_params(self.h, C.byref(p)))
        return self

    def set_laser(self, mean_per_step=0.0, wavelength=313e-9, mode=None):
        mode = (1 if mean_per_step > 0 else 0) if mode is None else mode
        p = LaserParams(mode, mean_per_step, wavelength)
        _check(load().pt_set_laser_params(self.h, C.byref(p)))
        return self

    def set_beams(self, laser: dict):
        """Beam mode from {wavelength, gamma0, beams: [{khat, detuning, s0, waist_y,
        waist_z, offset_y, uniform}, ...]}."""
        p = LaserParams(2, 0.0, laser["wavelength"], laser["gamma0"], len(laser["beams"]))
        for l, b in enumerate(laser["beams"]):
            p.beam[l] = Beam((C.c_double * 3)(*[float(x) for x in b["khat"]]), b["detuning"], b["s0"],
                             b.get("waist_y", 1.0), b.get("waist_z", 1.0), b.get("offset_y", 0.0),
                             int(b.get("uniform", 0)))
        _check(load().pt_set_laser_params(self.h, C.byref(p)))
        return self

    def set_force(self, method="fmm", p=8, leaf_size=32, precision="fp64"):
        m = {"direct": 0, "fmm": 1}[method] if isinstance(method, str) else int(method)
        pr = {"fp64": 0, "mixed": 1}[precision] if isinstance(precision, str) else int(precision)
        fp = ForceParams(m, int(p), int(leaf_size), pr)
        _check(load().pt_set_force_params(self.h, C.byref(fp)))
        return self

    def set_state(self, pos, vel, step=0):
        p, v = _xyz(pos, self.n), _xyz(vel, self.n)
        _check(load().pt_set_state(self.h, _ptr(p), _ptr(v), int(step)))

    def compute_forces(self):
        F = np.zeros((self.n, 3))
        _check(load().pt_compute_forces(self.h, _ptr(F)))
        return F

    def compute_forces_noalloc(self, F_dev_ptr: int):
        """Direct-sum forces into a caller's device buffer (n x 3 doubles at the
        integer address F_dev_ptr), queued on the context's stream without any
        allocation; call ctx.synchronize() before reading it."""
        _check(load().pt_compute_forces_noalloc(self.h, _vp(F_dev_ptr)))

    def compute_potential(self):
        phi = np.zeros(self.n)
        _check(load().pt_compute_potential(self.h, _ptr(phi)))
        return phi

    def coulomb_energy(self):
        U = C.c_double()
        _check(load().pt_coulomb_energy(self.h, C.byref(U)))
        return U.value

    def rotating_diagnostics(self):
        d = Diagnostics()
        _check(load().pt_rotating_diagnostics(self.h, C.byref(d)))
        return d.as_dict()

    def read_rotating_state(self):
        pos, vel = np.zeros((self.n, 3)), np.zeros((self.n, 3))
        _check(load().pt_read_rotating_state(self.h, _ptr(pos), _ptr(vel)))
        return pos, vel

    def step(self, n_steps: int):
        _check(load().pt_step(self.h, int(n_steps)))

    def read_state(self):
        pos, vel = np.zeros((self.n, 3)), np.zeros((self.n, 3))
        step, t = C.c_int64(), C.c_double()
        ph = np.zeros(self.n, np.int32)
        rc = load().pt_read_state(self.h, _ptr(pos), _ptr(vel), C.byref(step), C.byref(t), _ptr(ph, C.c_int32))
        _check(rc)
        return dict(pos=pos, vel=vel, step=step.value, t=t.value, photons=ph)

    def export_tree(self):
        L = load()
        sz = np.zeros(4, np.int64)
        nul = [None] * 13
        _check(L.pt_debug_export_tree(self.h, _ptr(sz, C.c_int64), *nul))
        nb, nlev, nv, nn = (int(x) for x in sz)
        n = self.n
        out = dict(key=np.zeros(n, np.uint64), perm=np.zeros(n, np.int32), level=np.zeros(nb, np.int32),
                   parent=np.zeros(nb, np.int32), ion_begin=np.zeros(nb, np.int32), ion_end=np.zeros(nb, np.int32),
                   coords=np.zeros((nb, 3), np.int32), is_leaf=np.zeros(nb, np.uint8),
                   v_off=np.zeros(nb + 1, np.int32), v_src=np.zeros(max(nv, 1), np.int32),
                   near_off=np.zeros(nb + 1, np.int32), near_src=np.zeros(max(nn, 1), np.int32), root=np.zeros(4))
        order = ["key", "perm", "level", "parent", "ion_begin", "ion_end", "coords", "is_leaf", "v_off", "v_src",
                 "near_off", "near_src", "root"]
        _check(L.pt_debug_export_tree(self.h, _ptr(sz, C.c_int64), *[out[k].ctypes.data_as(_vp) for k in order]))
        out["v_src"] = out["v_src"][:nv]
        out["near_src"] = out["near_src"][:nn]
        out["nlevels"] = nlev
        return out

    def destroy(self):
        if self.h:
            _check(load().pt_destroy_crystal(self.h))
            self.h = None
            if self in self.ctx.crystals:
                self.ctx.crystals.remove(self)


def step_batch(crystals, n_steps):
    L = load()
    arr = (_vp * len(crystals))(*[c.h for c in crystals])
    ns = np.ascontiguousarray(n_steps if np.ndim(n_steps) else [n_steps] * len(crystals), dtype=np.int64)
    _check(L.pt_step_batch(arr, len(crystals), _ptr(ns, C.c_int64)))


def compute_forces_batch(crystals):
    L = load()
    outs = [np.zeros((c.n, 3)) for c in crystals]
    arr = (_vp * len(crystals))(*[c.h for c in crystals])
    fo = (_dp * len(crystals))(*[_ptr(o) for o in outs])
    _check(L.pt_compute_forces_batch(arr, len(crystals), fo))
    return outs


def compute_potential_batch(crystals):
    L = load()
    outs = [np.zeros(c.n) for c in crystals]
    arr = (_vp * len(crystals))(*[c.h for c in crystals])
    po = (_dp * len(crystals))(*[_ptr(o) for o in outs])
    _check(L.pt_compute_potential_batch(arr, len(crystals), po))
    return outs


def rotating_diagnostics_batch(crystals):
    L = load()
    out = (Diagnostics * len(crystals))()
    arr = (_vp * len(crystals))(*[c.h for c in crystals])
    _check(L.pt_rotating_diagnostics_batch(arr, len(crystals), out))
    return [d.as_dict() for d in out]


def coulomb_energy_batch(crystals):
    L = load()
    U = np.zeros(len(crystals))
    arr = (_vp * len(crystals))(*[c.h for c in crystals])
    _check(L.pt_coulomb_energy_batch(arr, len(crystals), _ptr(U)))
    return U

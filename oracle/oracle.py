"""ctypes binding of the FP64 CPU oracle (``oracle/*.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product package never does.
Every routine restates a passage of Zaris et al., arXiv 2405.13973 (see the
C sources for the equation each follows).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_d = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u32 = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u64 = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


class Trap(C.Structure):
    _fields_ = [("B", C.c_double), ("omega_z", C.c_double), ("delta", C.c_double), ("omega_r", C.c_double),
                ("damping", C.c_double)]


def _trap(trap):
    return Trap(trap["B"], trap["omega_z"], trap.get("delta", 0.0), trap.get("omega_r", 0.0), trap.get("damping", 0.0))


class Beam(C.Structure):
    _fields_ = [("khat", C.c_double * 3), ("detuning", C.c_double), ("s0", C.c_double), ("waist_y", C.c_double),
                ("waist_z", C.c_double), ("offset_y", C.c_double), ("uniform", C.c_int)]


class Laser(C.Structure):
    _fields_ = [("mean_per_step", C.c_double), ("wavelength", C.c_double), ("mode", C.c_int), ("gamma0", C.c_double),
                ("n_beams", C.c_int), ("beam", Beam * 4)]


def laser_struct(laser):
    """Laser from a dict: {mean_per_step, wavelength} (fixed-mean mode) or
    {mode: 2, wavelength, gamma0, beams: [{khat, detuning, s0, waist_y, waist_z,
    offset_y, uniform}, ...]} (beam mode); None: off."""
    la = Laser()
    la.wavelength = 313e-9
    if not laser:
        return la
    la.wavelength = laser["wavelength"]
    if laser.get("mode", 1) == 2:
        la.mode = 2
        la.gamma0 = laser["gamma0"]
        la.n_beams = len(laser["beams"])
        for l, b in enumerate(laser["beams"]):
            la.beam[l].khat[:] = [float(x) for x in b["khat"]]
            la.beam[l].detuning = b["detuning"]
            la.beam[l].s0 = b["s0"]
            la.beam[l].waist_y = b.get("waist_y", 1.0)
            la.beam[l].waist_z = b.get("waist_z", 1.0)
            la.beam[l].offset_y = b.get("offset_y", 0.0)
            la.beam[l].uniform = int(b.get("uniform", 0))
    else:
        la.mode = 1
        la.mean_per_step = laser["mean_per_step"]
    return la


def scattering_rate(laser, l, x, v):
    """gamma_L of beam l at position x with velocity v (eq. scattering_rate), 1/s."""
    la = laser_struct(laser)
    return lib().or_scattering_rate(C.byref(la), int(l), np.ascontiguousarray(x, np.float64),
                                    np.ascontiguousarray(v, np.float64))


class Force(C.Structure):
    _fields_ = [("method", C.c_int), ("p", C.c_int), ("leaf_size", C.c_int)]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C, -ffp-contract=off)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["make", "-s"] + (["-B"] if force else []) + ["liboracle.so"]
        subprocess.run(cmd, cwd=_HERE, check=True)
    return _LIB_PATH


def _nullable(kind):
    """ndpointer type that also accepts None."""
    base = np.ctypeslib.ndpointer(dtype=kind, flags="C_CONTIGUOUS")

    def from_param(cls, obj):
        if obj is None:
            return None
        return base.from_param(obj)

    return type("Nullable" + base.__name__, (base,), {"from_param": classmethod(from_param)})


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(_LIB_PATH)
            L.or_philox4x32_10.argtypes = [_u32, _u32, _u32]
            L.or_poisson_cdf.argtypes = [C.c_double, _d]
            L.or_photon_counts.argtypes = [C.c_int, C.c_uint64, C.c_uint64, C.c_double, _i32]
            L.or_external_force.argtypes = [C.c_double, C.c_double, C.POINTER(Trap), C.c_double, _d, _d]
            L.or_coulomb_direct.argtypes = [C.c_int, _d, C.c_double, _d]
            L.or_coulomb_direct_sampled.argtypes = [C.c_int, _d, C.c_double, C.c_int, _i32, _d]
            L.or_coulomb_energy.argtypes = [C.c_int, _d, C.c_double]
            L.or_rotating_frame.argtypes = [C.c_int, _d, _d, C.c_double, C.c_double, _d, _d]
            L.or_rotating_energy.argtypes = [C.c_int, _d, _d, C.c_double, C.c_double, C.POINTER(Trap), C.c_double, _d]
            L.or_scattering_rate.argtypes = [C.POINTER(Laser), C.c_int, _d, _d]
            L.or_scattering_rate.restype = C.c_double
            L.or_coulomb_potential_direct.argtypes = [C.c_int, _d, C.c_double, _d]
            L.or_coulomb_potential_direct_sampled.argtypes = [C.c_int, _d, C.c_double, C.c_int, _i32, _d]
            L.or_fmm_potential.argtypes = [C.c_int, _d, C.c_double, C.c_int, C.c_int, C.c_int, _nullable(np.int32), _d]
            L.or_fmm_potential.restype = C.c_int
            L.or_coulomb_energy.restype = C.c_double
            L.or_energy.argtypes = [C.c_int, _d, _d, C.c_double, C.c_double, C.POINTER(Trap)]
            L.or_energy.restype = C.c_double
            L.or_u0.argtypes = [C.c_int, _d, _d, C.c_double, C.c_double]
            L.or_step.argtypes = [C.c_int, _d, _d, C.c_double, C.c_double, C.POINTER(Trap), C.POINTER(Laser),
                                  C.POINTER(Force), C.c_double, C.c_double, C.c_uint64, C.c_uint64,
                                  _nullable(np.int32)]
            L.or_run.argtypes = [C.c_int, _d, _d, C.c_double, C.c_double, C.POINTER(Trap), C.POINTER(Laser),
                                 C.POINTER(Force), C.c_double, C.c_double, C.c_uint64, C.c_uint64, C.c_int,
                                 _nullable(np.int32)]
            L.or_root_cube.argtypes = [C.c_int, _d, _d, C.POINTER(C.c_double)]
            L.or_morton_keys.argtypes = [C.c_int, _d, _u64, _d]
            L.or_tree_build.argtypes = [C.c_int, _d, C.c_int]
            L.or_tree_build.restype = C.c_void_p
            L.or_tree_free.argtypes = [C.c_void_p]
            L.or_tree_sizes.argtypes = [C.c_void_p, np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")]
            L.or_tree_export.argtypes = [C.c_void_p, _u64, _i32, _i32, _i32, _i32, _i32, _i32,
                                         np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS"),
                                         _i32, _i32, _i32, _i32, _d]
            L.or_dual_traversal.argtypes = [C.c_void_p, np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS"),
                                            _nullable(np.int32), _nullable(np.int32)]
            L.or_p2m.argtypes = [C.c_int, _d, _d, _d, C.c_int, _d]
            L.or_eval_me.argtypes = [C.c_int, _d, _d, _d]
            L.or_eval_me.restype = C.c_double
            L.or_m2m.argtypes = [C.c_int, _d, _d, _d, _d]
            L.or_m2l_add.argtypes = [C.c_int, _d, _d, _d, _d]
            L.or_l2l.argtypes = [C.c_int, _d, _d, _d, _d]
            L.or_eval_le.argtypes = [C.c_int, _d, _d, _d, C.POINTER(C.c_double), _d]
            L.or_fmm_coulomb.argtypes = [C.c_int, _d, C.c_double, C.c_int, C.c_int, _d]
            L.or_fmm_coulomb.restype = C.c_int
            L.or_fmm_coulomb_sampled.argtypes = [C.c_int, _d, C.c_double, C.c_int, C.c_int, C.c_int, _i32, _d]
            L.or_fmm_coulomb_sampled.restype = C.c_int
            _lib = L
    return _lib


# --------------------------------------------------------------- constants
E_CHARGE = 1.602176634e-19
H_PLANCK = 6.62607015e-34
K_BOLTZ = 1.380649e-23
EPS0 = 8.8541878188e-12
AMU = 1.66053906892e-27
K_E = 1.0 / (4.0 * np.pi * EPS0)


def _pos(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1, 3))


# ------------------------------------------------------------ generators
def philox4x32_10(counter, key):
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(np.asarray(counter, np.uint32), np.asarray(key, np.uint32), out)
    return out


def poisson_cdf(lam):
    F = np.zeros(17)
    lib().or_poisson_cdf(float(lam), F)
    return F


def photon_counts(n, seed, step, mean):
    out = np.zeros(n, np.int32)
    lib().or_photon_counts(int(n), int(seed), int(step), float(mean), out)
    return out


# ------------------------------------------------------------------ forces
def external_force(q, m, trap: dict, t, x):
    F = np.zeros(3)
    tr = _trap(trap)
    lib().or_external_force(q, m, C.byref(tr), t, np.ascontiguousarray(x, dtype=np.float64), F)
    return F


def coulomb_direct(pos, q):
    pos = _pos(pos)
    F = np.zeros_like(pos)
    lib().or_coulomb_direct(len(pos), pos, float(q), F)
    return F


def coulomb_direct_sampled(pos, q, idx):
    pos = _pos(pos)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    F = np.zeros((len(idx), 3))
    lib().or_coulomb_direct_sampled(len(pos), pos, float(q), len(idx), idx, F)
    return F


def coulomb_energy(pos, q):
    pos = _pos(pos)
    return lib().or_coulomb_energy(len(pos), pos, float(q))


def energy(pos, vel, q, m, trap: dict):
    pos, vel = _pos(pos), _pos(vel)
    tr = Trap(trap["B"], trap["omega_z"], 0.0, 0.0, 0.0)
    return lib().or_energy(len(pos), pos, vel, float(q), float(m), C.byref(tr))


def rotating_frame(pos, vel, omega_r, t):
    """Positions and velocities in the frame of eq. (rotation) at time t."""
    pos, vel = _pos(pos), _pos(vel)
    xr, vr = np.zeros_like(pos), np.zeros_like(vel)
    lib().or_rotating_frame(len(pos), pos, vel, float(omega_r), float(t), xr, vr)
    return xr, vr


def rotating_energy(pos, vel, q, m, trap: dict, t):
    """Rotating-frame energy terms (J): axial KE, planar KE, external, Coulomb, total."""
    pos, vel = _pos(pos), _pos(vel)
    tr = _trap(trap)
    out = np.zeros(5)
    lib().or_rotating_energy(len(pos), pos, vel, float(q), float(m), C.byref(tr), float(t), out)
    return out


def fmm_coulomb(pos, q, p, leaf_size):
    pos = _pos(pos)
    F = np.zeros_like(pos)
    rc = lib().or_fmm_coulomb(len(pos), pos, float(q), int(p), int(leaf_size), F)
    if rc:
        raise RuntimeError(f"or_fmm_coulomb failed ({rc})")
    return F


def fmm_coulomb_sampled(pos, q, p, leaf_size, idx):
    pos = _pos(pos)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    F = np.zeros((len(idx), 3))
    rc = lib().or_fmm_coulomb_sampled(len(pos), pos, float(q), int(p), int(leaf_size), len(idx), idx, F)
    if rc:
        raise RuntimeError(f"or_fmm_coulomb_sampled failed ({rc})")
    return F


def coulomb_potential_direct(pos, q, idx=None):
    """phi_i = k_e q sum_{j != i} 1/r_ij (volts); at the ions in idx if given."""
    pos = _pos(pos)
    if idx is None:
        phi = np.zeros(len(pos))
        lib().or_coulomb_potential_direct(len(pos), pos, float(q), phi)
        return phi
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    phi = np.zeros(len(idx))
    lib().or_coulomb_potential_direct_sampled(len(pos), pos, float(q), len(idx), idx, phi)
    return phi


def fmm_potential(pos, q, p, leaf_size, idx=None):
    """FMM potential (volts) at every ion, or at the ions in idx."""
    pos = _pos(pos)
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.int32)
    ns = len(pos) if idx is None else len(idx)
    phi = np.zeros(ns)
    rc = lib().or_fmm_potential(len(pos), pos, float(q), int(p), int(leaf_size), ns, idx, phi)
    if rc:
        raise RuntimeError(f"or_fmm_potential failed ({rc})")
    return phi


def error_pot(phi, phi_dir):
    """Relative RMS potential error of eq. (rms_pot)."""
    phi, phi_dir = np.asarray(phi, np.float64), np.asarray(phi_dir, np.float64)
    return float(np.sqrt(((phi - phi_dir) ** 2).sum() / (phi_dir ** 2).sum()))


# --------------------------------------------------------------- integrator
def u0(pos, vel, wc, tau):
    pos, vel = _pos(pos).copy(), _pos(vel).copy()
    lib().or_u0(len(pos), pos, vel, float(wc), float(tau))
    return pos, vel


def run(pos, vel, q, m, trap: dict, dt, nsteps, *, t0=0.0, step0=0, seed=0, laser=None, method="direct",
        p=8, leaf_size=32, return_photons=False):
    """nsteps oracle steps; returns (pos, vel[, photons of the last step])."""
    pos, vel = _pos(pos).copy(), _pos(vel).copy()
    tr = _trap(trap)
    la = laser_struct(laser)
    fo = Force(0 if method == "direct" else 1, int(p), int(leaf_size))
    ph = np.zeros(len(pos), np.int32)
    rc = lib().or_run(len(pos), pos, vel, float(q), float(m), C.byref(tr), C.byref(la), C.byref(fo), float(t0),
                      float(dt), int(seed), int(step0), int(nsteps), ph)
    if rc:
        raise RuntimeError(f"or_run failed ({rc})")
    return (pos, vel, ph) if return_photons else (pos, vel)


# ---------------------------------------------------------------- tree
def root_cube(pos):
    pos = _pos(pos)
    lo = np.zeros(3)
    W = C.c_double()
    lib().or_root_cube(len(pos), pos, lo, C.byref(W))
    return lo, W.value


def morton_keys(pos):
    pos = _pos(pos)
    keys = np.zeros(len(pos), np.uint64)
    root = np.zeros(4)
    lib().or_morton_keys(len(pos), pos, keys, root)
    return keys, root


def tree(pos, leaf_size):
    """Octree + lists as numpy arrays (boxes in (level, Morton prefix) order)."""
    pos = _pos(pos)
    L = lib()
    h = L.or_tree_build(len(pos), pos, int(leaf_size))
    if not h:
        raise ValueError("or_tree_build rejected its input")
    try:
        sz = np.zeros(4, np.int64)
        L.or_tree_sizes(h, sz)
        nb, nlev, nv, nn = (int(x) for x in sz)
        n = len(pos)
        out = dict(
            key=np.zeros(n, np.uint64), perm=np.zeros(n, np.int32), level=np.zeros(nb, np.int32),
            parent=np.zeros(nb, np.int32), ion_begin=np.zeros(nb, np.int32), ion_end=np.zeros(nb, np.int32),
            coords=np.zeros((nb, 3), np.int32), is_leaf=np.zeros(nb, np.uint8), v_off=np.zeros(nb + 1, np.int32),
            v_src=np.zeros(max(nv, 1), np.int32), near_off=np.zeros(nb + 1, np.int32),
            near_src=np.zeros(max(nn, 1), np.int32), root=np.zeros(4))
        L.or_tree_export(h, out["key"], out["perm"], out["level"], out["parent"], out["ion_begin"], out["ion_end"],
                         out["coords"], out["is_leaf"], out["v_off"], out["v_src"], out["near_off"],
                         out["near_src"], out["root"])
        out["v_src"] = out["v_src"][:nv]
        out["near_src"] = out["near_src"][:nn]
        out["nlevels"] = nlev
        cnt = np.zeros(2, np.int64)
        L.or_dual_traversal(h, cnt, None, None)
        vp = np.zeros((max(int(cnt[0]), 1), 2), np.int32)
        npr = np.zeros((max(int(cnt[1]), 1), 2), np.int32)
        L.or_dual_traversal(h, cnt, vp, npr)
        out["dual_v_pairs"] = vp[: int(cnt[0])]
        out["dual_near_pairs"] = npr[: int(cnt[1])]
        return out
    finally:
        L.or_tree_free(h)


# ------------------------------------------------------------ expansions
def _cplx(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128)).view(np.float64)


def p2m(pos, q, center, p):
    pos = _pos(pos)
    M = np.zeros((p + 1) ** 2, np.complex128)
    lib().or_p2m(len(pos), pos, np.ascontiguousarray(q, dtype=np.float64), np.asarray(center, np.float64), p,
                 M.view(np.float64))
    return M


def eval_me(M, center, x, p):
    return lib().or_eval_me(p, _cplx(M), np.asarray(center, np.float64), np.asarray(x, np.float64))


def m2m(M, c_old, c_new, p):
    out = np.zeros((p + 1) ** 2, np.complex128)
    lib().or_m2m(p, _cplx(M), np.asarray(c_old, np.float64), np.asarray(c_new, np.float64), out.view(np.float64))
    return out


def m2l(M, c_src, c_tgt, p):
    out = np.zeros((p + 1) ** 2, np.complex128)
    lib().or_m2l_add(p, _cplx(M), np.asarray(c_src, np.float64), np.asarray(c_tgt, np.float64),
                     out.view(np.float64))
    return out


def l2l(L, c_old, c_new, p):
    out = np.zeros((p + 1) ** 2, np.complex128)
    lib().or_l2l(p, _cplx(L), np.asarray(c_old, np.float64), np.asarray(c_new, np.float64), out.view(np.float64))
    return out


def eval_le(L, center, x, p):
    phi = C.c_double()
    g = np.zeros(3)
    lib().or_eval_le(p, _cplx(L), np.asarray(center, np.float64), np.asarray(x, np.float64), C.byref(phi), g)
    return phi.value, g

"""Seeded synthetic workloads: ion positions, velocities and trap settings.

This module only draws inputs; it holds none of the method's arithmetic.  It
is the one module shared by the GPU library's callers and by the CPU oracle's
tests, so that both see identical arrays.

The paper benchmarks its code on ions "uniformly distributed within a sphere"
at fixed density with zero initial velocity (Sec. 3), and initialises cooling
runs with Maxwell-Boltzmann velocities, i.e. Gaussian components (Sec. 5,
eq. maxwell_boltzmann).  The workloads below have those shapes; every draw
uses numpy's PCG64 seeded explicitly.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

E_CHARGE = 1.602176634e-19
AMU = 1.66053906892e-27
K_BOLTZ = 1.380649e-23
H_PLANCK = 6.62607015e-34

ION_MASS = 9.0 * AMU          # 9Be+ (the paper's species)
ION_CHARGE = E_CHARGE
COOLING_WAVELENGTH = 313e-9   # photon recoil h/(lambda m) = 0.1417 m/s
GAMMA0 = 2.0 * math.pi * 18e6  # natural linewidth of the cooling transition (rad/s)


def cooling_beams(w_y: float = 2.48e-6, detuning_perp: float = 2.0 * math.pi * 13.6e6, offset: float = 5e-6,
                  s_perp: float = 0.5, w_z: float = 1e-3, s_par: float = 5e-3) -> dict:
    """The cooling set-up of the paper's Sec. 5 and its cooling-setup figure: two
    counter-propagating axial beams of uniform intensity (detuning -gamma0/2,
    peak saturation 5e-3) and a planar Gaussian beam along +x, centred at
    y = offset, z = 0, with waists w_y and w_z (w_z large against the crystal),
    peak saturation 0.5 and detuning detuning_perp (frequencies quoted in MHz
    taken as cyclic, omega = 2 pi f)."""
    return dict(mode=2, wavelength=COOLING_WAVELENGTH, gamma0=GAMMA0, beams=[
        dict(khat=(0.0, 0.0, 1.0), detuning=-0.5 * GAMMA0, s0=s_par, uniform=1),
        dict(khat=(0.0, 0.0, -1.0), detuning=-0.5 * GAMMA0, s0=s_par, uniform=1),
        dict(khat=(1.0, 0.0, 0.0), detuning=detuning_perp, s0=s_perp, waist_y=w_y, waist_z=w_z, offset_y=offset,
             uniform=0),
    ])


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_ball(n: int, radius: float, g: np.random.Generator) -> np.ndarray:
    """n points uniform in a ball: r = R u^(1/3), isotropic direction."""
    d = g.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    r = radius * g.random(n) ** (1.0 / 3.0)
    return d * r[:, None]


def uniform_ellipsoid(n: int, axes, g: np.random.Generator) -> np.ndarray:
    return uniform_ball(n, 1.0, g) * np.asarray(axes, dtype=np.float64)[None, :]


def jittered_lattice_ellipsoid(n: int, axes, jitter: float, g: np.random.Generator) -> np.ndarray:
    """Simple cubic lattice at spacing a = (V/n)^(1/3) clipped to the ellipsoid:
    the n sites with the smallest ellipsoidal radius (ties by site index) are
    kept, then each coordinate moves by U(-jitter a, +jitter a)."""
    axes = np.asarray(axes, dtype=np.float64)
    vol = 4.0 / 3.0 * math.pi * axes.prod()
    a = (vol / n) ** (1.0 / 3.0)
    half = [int(math.ceil(ax / a)) + 2 for ax in axes]
    gx, gy, gz = (np.arange(-h, h + 1) * a for h in half)
    X, Y, Z = np.meshgrid(gx, gy, gz, indexing="ij")
    sites = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    rad = np.sqrt(((sites / axes[None, :]) ** 2).sum(axis=1))
    order = np.lexsort((np.arange(len(sites)), rad))[:n]
    pos = sites[np.sort(order)]
    return pos + g.uniform(-jitter * a, jitter * a, size=pos.shape)


def thermal_velocities(n: int, temperature: float, mass: float, g: np.random.Generator) -> np.ndarray:
    """Maxwell-Boltzmann speeds == independent Gaussian components, sigma = sqrt(kT/m)."""
    return g.normal(0.0, math.sqrt(K_BOLTZ * temperature / mass), size=(n, 3))


@dataclasses.dataclass
class Crystal:
    """One crystal's initial state and parameters (SI units)."""
    pos: np.ndarray
    vel: np.ndarray
    B: float = 4.5
    omega_z: float = 2.0 * math.pi * 1.5e6
    delta: float = 0.0
    omega_r: float = 0.0
    dt: float = 1e-9
    photon_mean: float = 0.0
    beams: dict | None = None   # beam-mode laser (cooling_beams()); overrides photon_mean
    seed: int = 0
    charge: float = ION_CHARGE
    mass: float = ION_MASS

    @property
    def n(self) -> int:
        return len(self.pos)

    def trap(self) -> dict:
        return dict(B=self.B, omega_z=self.omega_z, delta=self.delta, omega_r=self.omega_r)

    def laser(self):
        if self.beams:
            return self.beams
        if self.photon_mean <= 0:
            return None
        return dict(mean_per_step=self.photon_mean, wavelength=COOLING_WAVELENGTH)


def config1(seed: int = 1) -> Crystal:
    """1,000 ions uniform in a 100 um sphere, 10 mK, B = 4.5 T, dt = 1 ns, no laser."""
    g = rng(seed)
    pos = uniform_ball(1000, 100e-6, g)
    vel = thermal_velocities(1000, 10e-3, ION_MASS, g)
    return Crystal(pos, vel, seed=seed)


def config2(seed: int = 2) -> Crystal:
    """10,000 ions uniform in an oblate ellipsoid (300, 300, 150) um, 10 mK,
    photon mean 0.01 per ion per step."""
    g = rng(seed)
    pos = uniform_ellipsoid(10000, (300e-6, 300e-6, 150e-6), g)
    vel = thermal_velocities(10000, 10e-3, ION_MASS, g)
    return Crystal(pos, vel, photon_mean=0.01, seed=seed)


def config3(seed: int = 3, n: int = 100000) -> Crystal:
    """100,000 ions on a 5%-jittered lattice in a prolate ellipsoid (400, 400, 800) um."""
    g = rng(seed)
    pos = jittered_lattice_ellipsoid(n, (400e-6, 400e-6, 800e-6), 0.05, g)
    vel = thermal_velocities(n, 10e-3, ION_MASS, g)
    return Crystal(pos, vel, seed=seed)


def density_radius(n: int) -> float:
    """Sphere radius holding n ions at the density of 1,000 ions in 100 um."""
    return 100e-6 * (n / 1000.0) ** (1.0 / 3.0)


def ensemble(count: int = 256, seed: int = 4, n_lo: int = 100, n_hi: int = 20000) -> list:
    """Independent crystals: N log-uniform in [n_lo, n_hi], B ~ U[2,5] T,
    f_z ~ U[1,2] MHz, photon mean ~ U[0, 0.05]; spheres at fixed density."""
    g = rng(seed)
    out = []
    for k in range(count):
        n = int(round(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
        B = g.uniform(2.0, 5.0)
        fz = g.uniform(1e6, 2e6)
        lam = g.uniform(0.0, 0.05)
        pos = uniform_ball(n, density_radius(n), g)
        vel = thermal_velocities(n, 10e-3, ION_MASS, g)
        out.append(Crystal(pos, vel, B=B, omega_z=2.0 * math.pi * fz, photon_mean=lam, seed=seed * 100003 + k))
    return out


@dataclasses.dataclass
class Request:
    arrival_s: float
    crystal: Crystal
    steps: int


def serving_stream(count: int = 500, rate_hz: float = 50.0, seed: int = 5, n_lo: int = 200,
                   n_hi: int = 50000, k_lo: int = 100, k_hi: int = 2000) -> list:
    """Poisson arrivals; N log-uniform in [n_lo, n_hi]; K ~ U{k_lo..k_hi};
    photon mean 0.01; per-request B and f_z as in the ensemble."""
    g = rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += g.exponential(1.0 / rate_hz)
        n = int(round(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
        steps = int(g.integers(k_lo, k_hi + 1))
        B = g.uniform(2.0, 5.0)
        fz = g.uniform(1e6, 2e6)
        pos = uniform_ball(n, density_radius(n), g)
        vel = thermal_velocities(n, 10e-3, ION_MASS, g)
        c = Crystal(pos, vel, B=B, omega_z=2.0 * math.pi * fz, photon_mean=0.01, seed=seed * 100003 + k)
        out.append(Request(t, c, steps))
    return out

"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds no arithmetic of the method: it only draws initial fields
and turns a workload description (grid size, Fresnel number, reflectivity,
pump ratio, T1) into the physical parameters both sides take as input.

Recipe (used for every workload; the paper's cavity numbers are context only):

* wavelength lambda = 1.064 um and cavity length L = 2 mm, the values of the
  experiment discussed in Sec. 4;
* the Fresnel number F = a^2 / (lambda L) fixes the half-window a, and the grid
  spacing is dx = 2a / N;
* aperture: circular super-Gaussian amplitude exp(-(r/r0)^10), r0 = 0.8 a;
* pump N0 = r * ln(1/R): r times the plane-wave threshold log-gain
  (a mirror of reflectivity R loses ln(1/R) of log-intensity per bounce);
* initial field: circular complex Gaussian noise, <|E|^2> = sigma^2 with
  sigma = 1e-3 (real and imaginary parts N(0, sigma^2/2)), drawn with NumPy's
  PCG64 generator seeded with 14102855 + cavity index; the oracle receives it
  as complex128, the GPU the same array rounded to complex64;
* initial inversion N = N0 everywhere; with m thin gain sheets, N0/m on every
  sheet (the inversion array is then m x N x N, sheet 0 at the mirror);
* mirror roughness (off unless asked for): a phase field psi(x, y) drawn as
  white Gaussian noise (PCG64 seeded with 14102855 + 500009 + cavity index),
  smoothed by a circular moving average `rough_corr` cells wide along each
  axis and scaled to the rms `rough_rms` (rad).  Both sides receive the same
  float64 array.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

LAMBDA = 1.064e-6     # m
L_CAV = 2.0e-3        # m
SEED_BASE = 14102855
ROUGH_SEED_OFFSET = 500009
NOISE_SIGMA = 1.0e-3


@dataclass
class Cavity:
    """One cavity: grid, optics, gain.  Units: metres; gain in log units."""

    N: int
    F: float                 # Fresnel number a^2/(lambda L)
    R: float                 # mirror reflectivity
    pump_ratio: float        # N0 / ln(1/R)
    T1: float                # inversion relaxation time, round trips
    index: int = 0           # cavity index (seeds the noise)
    lam: float = LAMBDA
    L: float = L_CAV
    ap_kind: int = 1         # 0 none, 1 super-Gaussian, 2 Gaussian
    ap_radius_frac: float = 0.8
    ap_order: int = 10
    focal: float = float("inf")
    mod_amp: float = 0.0
    mod_periods: int = 0     # integer number of pump periods across the window
    n0_override: float | None = None
    filter_delta: float = 0.0  # > 0: real renormalization-group filter (m) instead of Fresnel
    model: int = 0             # 0 B class (Euler update), 1 B class (exact update), 2 class A
    slices: int = 1            # thin gain sheets per round trip
    rough_rms: float = 0.0     # rms of the mirror roughness phase (rad); 0 = smooth mirror
    rough_corr: int = 4        # its correlation width (grid cells)

    @property
    def a(self) -> float:
        return math.sqrt(self.F * self.lam * self.L)

    @property
    def dx(self) -> float:
        return 2.0 * self.a / self.N

    @property
    def N0(self) -> float:
        if self.n0_override is not None:
            return self.n0_override
        return self.pump_ratio * math.log(1.0 / self.R)

    @property
    def ap_radius(self) -> float:
        return self.ap_radius_frac * self.a

    @property
    def mod_period(self) -> float:
        return 2.0 * self.a / self.mod_periods if self.mod_periods else 0.0

    def with_(self, **kw) -> "Cavity":
        return replace(self, **kw)


def noise_field(N: int, index: int, sigma: float = NOISE_SIGMA) -> np.ndarray:
    """Seeded circular complex Gaussian noise, complex128 (N, N)."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + index))
    s = sigma / math.sqrt(2.0)
    re = rng.standard_normal((N, N))
    im = rng.standard_normal((N, N))
    return (re * s + 1j * (im * s)).astype(np.complex128)


def roughness_phase(N: int, index: int, rms: float, corr: int = 4) -> np.ndarray:
    """Seeded smooth random phase field psi (rad), float64 (N, N), of rms `rms`:
    white Gaussian noise averaged over a circular window `corr` cells wide
    along each axis, then scaled."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + ROUGH_SEED_OFFSET + index))
    w = rng.standard_normal((N, N))
    k = max(1, int(corr))
    for axis in (0, 1):
        acc = np.zeros_like(w)
        for s in range(k):
            acc += np.roll(w, s, axis=axis)
        w = acc
    w -= w.mean()
    return w * (rms / math.sqrt(np.mean(w * w)))


def rough_field(cav: "Cavity") -> np.ndarray | None:
    """The cavity's roughness phase, or None for a smooth mirror."""
    if not cav.rough_rms:
        return None
    return roughness_phase(cav.N, cav.index, cav.rough_rms, cav.rough_corr)


def initial_state(cav: Cavity):
    """(E0 complex128, Ninv0 float64) for a cavity; Ninv0 is (m, N, N) with
    m > 1 gain sheets."""
    e = noise_field(cav.N, cav.index)
    if cav.slices > 1:
        return e, np.full((cav.slices, cav.N, cav.N), cav.N0 / cav.slices, dtype=np.float64)
    n = np.full((cav.N, cav.N), cav.N0, dtype=np.float64)
    return e, n


def oracle_params(cav: Cavity):
    """The cavity as the oracle's parameter record."""
    from oracle import CavityParams  # test infrastructure; imported lazily

    return CavityParams(N=cav.N, dx=cav.dx, lam=cav.lam, L=cav.L, R=cav.R,
                        N0=cav.N0, T1=cav.T1, focal=cav.focal, ap_kind=cav.ap_kind,
                        ap_radius=cav.ap_radius, ap_order=cav.ap_order,
                        mod_amp=cav.mod_amp, mod_period=cav.mod_period,
                        filter_delta=cav.filter_delta, model=cav.model, slices=cav.slices,
                        rough=rough_field(cav))


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def plain_256() -> Cavity:
    """One cavity, 256^2, F=100, R=0.9, pump 2x threshold, T1=1000 (300 trips)."""
    return Cavity(N=256, F=100.0, R=0.9, pump_ratio=2.0, T1=1000.0)


def plain_1024() -> Cavity:
    """One cavity, 1024^2, F=300, R=0.95, pump 3x threshold, T1=2000 (10000 trips)."""
    return Cavity(N=1024, F=300.0, R=0.95, pump_ratio=3.0, T1=2000.0)


def precision_2048() -> Cavity:
    """One cavity, 2048^2, F=1000, R=0.9, pump 4x threshold, T1=500 (20000 trips)."""
    return Cavity(N=2048, F=1000.0, R=0.9, pump_ratio=4.0, T1=500.0)


SWEEP_SIZES = (256, 384, 512, 768, 1024)


def sweep(count: int = 512, seed: int = 0, sizes=SWEEP_SIZES) -> list[Cavity]:
    """Batched sweep: N uniform over ``sizes``, F log-uniform in [100, 1000],
    pump ratio U[1.2, 4], T1 U[200, 5000], R U[0.8, 0.98]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        n = int(rng.choice(np.asarray(sizes)))
        f = float(10.0 ** rng.uniform(2.0, 3.0))
        r = float(rng.uniform(1.2, 4.0))
        t1 = float(rng.uniform(200.0, 5000.0))
        refl = float(rng.uniform(0.8, 0.98))
        out.append(Cavity(N=n, F=f, R=refl, pump_ratio=r, T1=t1, index=i))
    return out


def sweep_1024(count: int = 64, seed: int = 0) -> list[Cavity]:
    """The sweep's parameter draws with every grid at 1024^2."""
    return [c.with_(N=1024) for c in sweep(count, seed)]


def structured_4096(count: int = 16) -> list[Cavity]:
    """16 cavities at 4096^2, F=1000, R=0.9, pump 2x threshold, T1=1000, pump
    N0 (1 + 0.3 cos(2 pi x/d) cos(2 pi y/d)) with M_i = 45 + round(44 i/15)
    periods across the window, so the cavity length runs from a quarter of the
    Talbot length z_T = 2 d^2 / lambda up to z_T."""
    out = []
    for i in range(count):
        m = 45 + int(round(44.0 * i / max(count - 1, 1)))
        out.append(Cavity(N=4096, F=1000.0, R=0.9, pump_ratio=2.0, T1=1000.0,
                          index=i, mod_amp=0.3, mod_periods=m))
    return out

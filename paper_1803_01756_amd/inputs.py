"""Seeded synthetic inputs shared by the GPU path and the CPU oracle's tests.

This module only draws numbers: the initial density field and the parameter
samples of the batched and served workloads.  It holds none of the lattice
Boltzmann arithmetic.  The noise generator is counter based: cell c of a
field with seed s gets SplitMix64(s XOR c), SplitMix64 being the published
64-bit mixer of Steele, Lea and Flood (OOPSLA 2014, as distributed by Vigna):
    z = x + 0x9E3779B97F4A7C15
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    return z ^ (z >> 31)
so any cell's value can be regenerated on its own.
"""
from __future__ import annotations

import math

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """One SplitMix64 output for each 64-bit state in ``x`` (vectorised)."""
    with np.errstate(over="ignore"):
        z = np.asarray(x, dtype=np.uint64) + _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, count: int) -> np.ndarray:
    """U_c = (SplitMix64(seed XOR c) >> 11) * 2^-53 for c = 0..count-1."""
    c = np.arange(count, dtype=np.uint64)
    z = splitmix64(np.uint64(seed) ^ c)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def density_field(Nx: int, Ny: int, rho_init: float, noise: float, seed: int) -> np.ndarray:
    """Initial density rho(x, y) = rho_init * (1 + noise * (2U - 1)) with the
    counter c = y * Nx + x.  Returned as float64 [Ny, Nx]; the solid plate
    rows are included and ignored by both solvers."""
    u = uniform01(seed, Nx * Ny).reshape(Ny, Nx)
    return rho_init * (1.0 + noise * (2.0 * u - 1.0))


def layer_field(Nx: int, Ny: int, rho_lo: float, rho_hi: float, height: float,
                width: float, noise: float, seed: int) -> np.ndarray:
    """A layer on the lower plate: rho_hi up to row `height`, rho_lo above,
    joined by a tanh profile of the given width, times (1 + noise (2U - 1))
    with the counters of density_field.  float64 [Ny, Nx]."""
    y = np.arange(Ny, dtype=np.float64)[:, None] * np.ones((1, Nx))
    h = 0.5 * (1.0 - np.tanh((y - height) / width))
    return (rho_lo + (rho_hi - rho_lo) * h) * density_field(Nx, Ny, 1.0, noise, seed)


def sample_channels(n: int, seed: int = 1803):
    """Parameter draws of the batched workload: Nx log-uniform on [256, 4096],
    Ny uniform on the multiples of 16 in [32, 256], contact angle uniform on
    [60, 150] degrees, wall temperature uniform on [0.76, 0.84] Tc,
    oscillation period uniform on [1000, 8000] steps, amplitude uniform on
    [5e-7, 5e-6].  Returns a list of dicts (angles in degrees, wall
    temperature as a fraction of Tc)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n):
        nx = int(math.floor(math.exp(rng.uniform(math.log(256.0), math.log(4096.0)))))
        ny = 16 * int(rng.integers(2, 17))
        out.append(dict(Nx=nx, Ny=ny,
                        contact_angle=float(rng.uniform(60.0, 150.0)),
                        Tw_frac=float(rng.uniform(0.76, 0.84)),
                        period=float(rng.uniform(1000.0, 8000.0)),
                        g_osc=float(rng.uniform(5e-7, 5e-6)),
                        seed=int(rng.integers(1, 2 ** 31))))
    return out


def poisson_arrivals(n: int, rate: float, seed: int = 20):
    """Arrival times (seconds) of a Poisson stream and the per-request step
    count, uniform on [2000, 20000]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=n)
    steps = rng.integers(2000, 20001, size=n)
    return np.cumsum(gaps), steps


def droplet_disc(Nx: int, Ny: int, D: float, rho_in: float, rho_out: float,
                 width: float = 5.0) -> np.ndarray:
    """Density field [Ny, Nx] of a disc of diameter D at the centre
    ((Nx-1)/2, (Ny-1)/2): a tanh profile of the given width from rho_in
    inside to rho_out outside."""
    y, x = np.mgrid[0:Ny, 0:Nx].astype(float)
    r = np.hypot(x - (Nx - 1) / 2, y - (Ny - 1) / 2)
    return 0.5 * (rho_in + rho_out) - 0.5 * (rho_in - rho_out) * np.tanh(2 * (r - D / 2) / width)

"""Parameter sets of the workloads the library is measured and tested on.

All are channels between two plates (solid rows y = 0 and y = Ny - 1),
periodic in x, driven by rho * g_osc * sin(2 pi n / period) along x, with the
Peng-Robinson EOS of Eq. 11 (a = 3/49, b = 2/21, R = 1), fluid initially
saturated vapour at T_0 = 0.86 Tc with +-1 % seeded density noise and the
plates at T_w.  Wettability is set through the wall potential: G_w = G and
psi_w = psi(rho_w, T_0) for a virtual wall density rho_w (Eq. 14); the
contact angle that a given rho_w produces is a calibration, see
``CONTACT_ANGLE_TABLE``.
"""
from __future__ import annotations

import math

import numpy as np

from . import inputs
from . import lbm

# Virtual wall density fraction phi_w = (rho_w - rho_g)/(rho_l - rho_g) -> static
# contact angle (degrees) at 0.86 Tc, measured on sessile droplets (see the
# design notes for the recipe).  Filled by the calibration; interpolated
# linearly in between.
CONTACT_ANGLE_TABLE = [
    (0.0, 180.0),
    (0.5, 90.0),
    (1.0, 0.0),
]


def wall_fraction_for_angle(theta_deg: float) -> float:
    """Inverse of CONTACT_ANGLE_TABLE (angles decrease as the fraction grows)."""
    tab = sorted(CONTACT_ANGLE_TABLE, key=lambda t: -t[1])
    angles = [a for _, a in tab]
    fracs = [f for f, _ in tab]
    return float(np.interp(theta_deg, angles[::-1], fracs[::-1]))


def psi_of(p: lbm.lbm_params, rho: float, T: float) -> float:
    """Eq. 10 on the host (used only to turn a wall density into psi_w)."""
    k = 0.37464 + 1.54226 * p.omega - 0.26992 * p.omega ** 2
    phi = (1.0 + k * (1.0 - math.sqrt(T / p.T_c))) ** 2
    br = p.b * rho
    P = rho * p.R * T / (1.0 - br) - p.a * phi * rho * rho / (1.0 + 2.0 * br - br * br)
    arg = 2.0 * (P - rho / 3.0) / p.G
    return math.sqrt(arg) if arg > 0.0 else 0.0


def channel_params(Nx: int, Ny: int, contact_angle: float = 90.0, Tw_frac: float = 0.80,
                   g_osc: float = 1e-6, period: float = 2000.0,
                   precision: int = lbm.LBM_FP32_DEV, flags: int = 0,
                   **overrides) -> lbm.lbm_params:
    p = lbm.lbm_params_default(Nx=Nx, Ny=Ny, g_osc=g_osc, period=period,
                               precision=precision, flags=flags)
    p = lbm.lbm_params_resolve(p)
    p.T_w = Tw_frac * p.T_c
    frac = wall_fraction_for_angle(contact_angle)
    rho_w = p.rho_g + frac * (p.rho_l - p.rho_g)
    p.G_w = p.G
    p.psi_w = psi_of(p, rho_w, p.T_0)
    for k, v in overrides.items():
        setattr(p, "lambda_" if k == "lambda" else k, v)
    return p


def initial_density(p: lbm.lbm_params, seed: int, noise: float = 0.01) -> np.ndarray:
    return inputs.density_field(p.Nx, p.Ny, p.rho_v, noise, seed)


# The workloads (sizes and physics of the measured configurations)
def oracle_size_channel(precision=lbm.LBM_FP32_DEV):
    """128 x 32, contact angle 90 deg, T_w = 0.80 Tc, g = 1e-6, period 2000."""
    return channel_params(128, 32, 90.0, 0.80, 1e-6, 2000.0, precision)


def single_gpu_channel(contact_angle=90.0, precision=lbm.LBM_FP32_DEV):
    """2048 x 256, period 4000, amplitude 2e-6."""
    return channel_params(2048, 256, contact_angle, 0.80, 2e-6, 4000.0, precision)


def large_channel(precision=lbm.LBM_FP32_DEV):
    """8192 x 512 cold-wall condensation: T_w = 0.78 Tc, contact angle 75 deg."""
    return channel_params(8192, 512, 75.0, 0.78, 2e-6, 4000.0, precision)

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

import numpy as np

from . import inputs
from . import lbm

# Virtual wall density fraction phi_w = (rho_w - rho_g)/(rho_l - rho_g) ->
# static contact angle (degrees) at 0.86 Tc, measured on sessile droplets with
# the FP64 oracle (160 x 70 channel, half-disc droplet of radius 22, 12000
# steps, circle fit of the rho = (rho_l + rho_g)/2 contour).  Interpolated
# linearly in between; angles outside the table clamp to its ends.
CONTACT_ANGLE_TABLE = [
    (0.20, 150.72), (0.25, 134.59), (0.30, 121.46), (0.35, 109.91), (0.38, 103.59), (0.41, 97.58),
    (0.43, 93.79), (0.45, 90.13), (0.50, 81.55), (0.55, 73.65), (0.60, 66.44),
    (0.65, 59.84),
]


def wall_fraction_for_angle(theta_deg: float) -> float:
    """Inverse of CONTACT_ANGLE_TABLE (the angle falls as the fraction grows)."""
    tab = sorted(CONTACT_ANGLE_TABLE, key=lambda t: t[1])
    angles = [a for _, a in tab]
    fracs = [f for f, _ in tab]
    return float(np.interp(theta_deg, angles, fracs))


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
    p.psi_w = lbm.lbm_eos_pressure(p, rho_w, p.T_0)[1]
    for k, v in overrides.items():
        setattr(p, "lambda_" if k == "lambda" else k, v)
    return p


def channel_params_cs(Nx: int, Ny: int, wall_fraction: float = 0.45, Tw_frac: float = 0.80,
                      g_osc: float = 1e-6, period: float = 2000.0,
                      precision: int = lbm.LBM_FP32_DEV, flags: int = 0,
                      **overrides) -> lbm.lbm_params:
    """The plate channel with the Carnahan-Starling EOS (a = 1, b = 4, R = 1)
    in place of Eq. 11; T_0 = 0.86 T_c and T_w = Tw_frac T_c of its own
    critical temperature.  The wall potential is set from a virtual wall
    density fraction directly (the contact-angle table is calibrated for
    Eq. 11 only).  lambda defaults to 0.05: the CS vapour is ten times thinner
    than the PR one (rho_g = 0.034 at 0.86 T_c), and the explicit RK4 of the
    energy equation with the nine-point Laplacian (eigenvalues down to -16/3)
    is stable only while lambda / (rho_g C_v) stays below about 0.5."""
    p = lbm.lbm_params_default(Nx=Nx, Ny=Ny, g_osc=g_osc, period=period,
                               precision=precision, flags=flags | lbm.LBM_EOS_CS)
    p.a, p.b, p.R, p.T_c, p.T_0, p.T_w = 1.0, 4.0, 1.0, 0.0, 0.0, 0.0
    p = lbm.lbm_params_resolve(p)
    p.T_w = Tw_frac * p.T_c
    rho_w = p.rho_g + wall_fraction * (p.rho_l - p.rho_g)
    p.G_w = p.G
    p.psi_w = lbm.lbm_eos_pressure(p, rho_w, p.T_0)[1]
    p.lambda_ = 0.05
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


def d2_box(lam: float, precision=lbm.LBM_FP32_DEV, N: int = 200, **overrides):
    """Sec. 3.1 droplet evaporation: an N x N periodic box whose frame is an
    open reservoir at rest (flags FRAME_T | FRAME_RHO) at the surroundings'
    temperature T_c and at the saturation pressure of T_sat = 0.86 T_c (its
    density solves P_EOS(rho, T_c) = P_EOS(rho_g, T_sat) on the vapour side),
    fluid at T_sat, no drive; lambda is the case parameter (1/3 and 2/3 in the
    paper)."""
    p = lbm.lbm_params_default(Nx=N, Ny=N, g_osc=0.0, period=0.0, precision=precision,
                               flags=lbm.LBM_PERIODIC_Y | lbm.LBM_FRAME_T | lbm.LBM_FRAME_RHO)
    p = lbm.lbm_params_resolve(p)
    p.T_w = p.T_c
    p.lambda_ = lam
    p_sat = lbm.lbm_eos_pressure(p, p.rho_g, p.T_0)[0]
    lo, hi = 1e-6, p.rho_g  # P(rho, T_c) rises monotonically on the critical isotherm
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if lbm.lbm_eos_pressure(p, mid, p.T_w)[0] < p_sat:
            lo = mid
        else:
            hi = mid
    p.rho_frame = 0.5 * (lo + hi)
    for k, v in overrides.items():
        setattr(p, "lambda_" if k == "lambda" else k, v)
    return p


def droplet_density(p: lbm.lbm_params, D: float, width: float = 5.0) -> np.ndarray:
    """A disc of diameter D at the box centre: tanh profile of the given width
    between the coexistence densities rho_l (inside) and rho_g."""
    return inputs.droplet_disc(p.Nx, p.Ny, D, p.rho_l, p.rho_g, width)


def open_channel(Nx: int = 1600, Ny: int = 48, contact_angle: float = 137.82,
                 p_amp: float = 0.1, p_period: float = 2000.0, g_x: float = 1e-4,
                 precision=lbm.LBM_FP32_DEV, **overrides) -> lbm.lbm_params:
    """Sec. 3.3: saturated vapour driven through a plate channel by an
    oscillating inlet pressure p0 (1 + 0.1 sin(2 pi n / p_period)) against a
    constant outlet pressure p0 (Zou-He ends, flag OPEN_X); plates at a
    temperature falling linearly from 0.86 T_c at the inlet to 0.56 T_c at the
    outlet; inlet vapour at T_sat = 0.86 T_c and the outlet open onto the
    same saturated vapour (T_out = T_sat: the paper has saturated vapour
    entering through the exit when the flow reverses); gravity g_x = 1e-4
    along +x; the paper's hydrophobic plates (137.82 degrees).  The
    oscillation frequency is not given, so p_period is a parameter.  The
    energy equation is the paper's unless alpha_max > 0 is passed (the
    diffusivity cap, a departure for thin vapour)."""
    p = lbm.lbm_params_default(Nx=Nx, Ny=Ny, g_osc=0.0, period=0.0, precision=precision,
                               flags=lbm.LBM_OPEN_X)
    p = lbm.lbm_params_resolve(p)
    p.T_w = 0.86 * p.T_c
    p.T_w_end = 0.56 * p.T_c
    p.T_in = p.T_0
    p.T_out = p.T_0
    p.p_amp, p.p_period, p.g_x = p_amp, p_period, g_x
    frac = wall_fraction_for_angle(contact_angle)
    p.G_w = p.G
    p.psi_w = lbm.lbm_eos_pressure(p, p.rho_g + frac * (p.rho_l - p.rho_g), p.T_0)[1]
    for k, v in overrides.items():
        setattr(p, "lambda_" if k == "lambda" else k, v)
    return p


def gravity_plate(Nx: int = 100, Ny: int = 300, contact_angle: float = 137.82,
                  Tw_frac: float = 0.65, g: float = 1e-4, cold_band=None,
                  precision=lbm.LBM_FP32_DEV, **overrides) -> lbm.lbm_params:
    """Sec. 3.2: saturated vapour at T_sat = 0.86 T_c between two hydrophobic
    plates, periodic in x, no drive, gravity g toward the bottom plate.  The
    top plate is cold (Tw_frac T_c) on its central band of columns and
    adiabatic on either side (flag TOP_MIXED); the bottom plate is held at
    T_sat.  The band's width is not given (its figure is missing): the
    default is the middle third, [Nx/3, 2Nx/3).  The contact angle is not
    given either: the default is the Sec. 3.3 plates' 137.82 degrees."""
    p = lbm.lbm_params_default(Nx=Nx, Ny=Ny, g_osc=0.0, period=0.0, precision=precision,
                               flags=lbm.LBM_TOP_MIXED)
    p = lbm.lbm_params_resolve(p)
    p.T_w = Tw_frac * p.T_c
    p.T_w_bottom = p.T_0
    p.cold_x0, p.cold_x1 = cold_band if cold_band is not None else (Nx // 3, 2 * Nx // 3)
    p.g_y = -g
    frac = wall_fraction_for_angle(contact_angle)
    p.G_w = p.G
    p.psi_w = lbm.lbm_eos_pressure(p, p.rho_g + frac * (p.rho_l - p.rho_g), p.T_0)[1]
    for k, v in overrides.items():
        setattr(p, "lambda_" if k == "lambda" else k, v)
    return p

"""Shared test helpers: conversion of the library's parameters to the
oracle's and the per-field error measures used by the parity tests.

Error measures (the tolerance of each test is stated where it is used):
  rho, T  max over fluid nodes of |a - b| / |b|
  u       max over fluid nodes of |u_a - u_b| / max |u_b|   (normwise, since u
          passes through zero)
"""
import numpy as np

_MAP = dict(Nx="Nx", Ny="Ny", a="a", b="b", R="R", omega="omega", T_c="Tc", G="G",
            theta="theta", G_w="Gw", psi_w="psiw", s_rho="s_rho", s_e="s_e",
            s_zeta="s_zeta", s_j="s_j", s_q="s_q", tau_g="tau_g", tau_l="tau_l",
            rho_g="rho_g", rho_l="rho_l", C_v="Cv", lambda_="lam", T_0="T0", T_w="Tw",
            g_osc="g_osc", period="period", g_x="gx", g_y="gy", rho_v="rho_v",
            rho_frame="rho_frame", p_amp="p_amp", p_period="p_period", T_w_end="Tw_end",
            T_in="T_in", lambda_l="lam_l", C_v_l="Cv_l", T_w_bottom="Tw_bot",
            cold_x0="cold_x0", cold_x1="cold_x1", flags="flags", alpha_max="alpha_max",
            T_out="T_out")


def to_oracle(orc, p):
    return orc.make_params(**{ov: getattr(p, lv) for lv, ov in _MAP.items()})


def fluid_mask(Nx, Ny, periodic_y=False):
    m = np.ones((Ny, Nx), dtype=bool)
    if not periodic_y:
        m[0] = m[-1] = False
    return m


def field_errors(gpu, ref, mask):
    rho_a, ux_a, uy_a, T_a = gpu[:4]
    rho_b, ux_b, uy_b, T_b = ref[:4]
    e_rho = np.max(np.abs(rho_a - rho_b)[mask] / np.abs(rho_b)[mask])
    e_T = np.max(np.abs(T_a - T_b)[mask] / np.abs(T_b)[mask])
    du = np.hypot(ux_a - ux_b, uy_a - uy_b)[mask]
    umax = np.hypot(ux_b, uy_b)[mask].max()
    e_u = du.max() / umax if umax > 0 else du.max()
    return dict(rho=float(e_rho), u=float(e_u), T=float(e_T), umax=float(umax))

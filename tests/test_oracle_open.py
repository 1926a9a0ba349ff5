"""Pins of the oracle's open channel (Sec. 3.3 boundary set, flag OPEN_X):
Zou-He pressure inlet and outlet, zero-gradient ghosts, linear plate
temperature, held inlet temperature.

* The rebuilt boundary populations give exactly the prescribed density and
  zero transverse momentum; the corner nodes (next to a plate) zero velocity.
* The inlet density is the vapour-branch root of the EOS at the prescribed
  pressure.
* A pressure difference drives plane Poiseuille flow: with the fluid ideal
  (single phase, p = rho/3 in the LB pressure) the centre-line velocity is
  dp/dx H^2 / (8 rho nu), H = Ny - 2, nu = (tau - 1/2)/3.
* Plates hold the linear temperature profile; the inlet column holds T_in.
"""
import numpy as np
import pytest


def _open(orc, Nx, Ny, **kw):
    tc = orc.critical()[1]
    p = orc.default_params(Nx=Nx, Ny=Ny, period=0.0, g_osc=0.0, **kw)
    p.flags |= orc.OPEN_X
    return p, tc


def test_zou_he_sets_density_and_zero_transverse_momentum(orc):
    Nx, Ny = 24, 10
    p, tc = _open(orc, Nx, Ny, flags=orc.SINGLE_PHASE | orc.FREEZE_T)
    p.p_amp, p.p_period = 0.1, 400.0
    rng = np.random.default_rng(3)
    s = orc.Sim(p, rho_uniform=p.rho_v)
    f = s.get_f()
    f[:, 1:-1, :] *= rng.uniform(0.95, 1.05, f[:, 1:-1, :].shape)
    s.set_f(f)
    s.set_time(100)
    rho, ux, uy, _, _, _ = s.moments()
    rin = orc.inlet_density(p, 100)
    np.testing.assert_allclose(rho[2:-2, 0], rin, rtol=1e-14)
    np.testing.assert_allclose(rho[2:-2, -1], p.rho_v, rtol=1e-14)
    assert np.abs(uy[1:-1, 0]).max() < 1e-15 and np.abs(uy[1:-1, -1]).max() < 1e-15
    # corners (next to a plate): the velocity form with u = 0
    for yc in (1, Ny - 2):
        assert abs(ux[yc, 0]) < 1e-15 and abs(ux[yc, -1]) < 1e-15


def test_inlet_density_inverts_the_eos(orc):
    p, tc = _open(orc, 8, 6)
    p.p_amp, p.p_period = 0.1, 1000.0
    p0 = orc.peos(p, p.rho_v, p.T0)
    for n in (0, 125, 250, 600, 750):
        r = orc.inlet_density(p, n)
        target = p0 * (1 + 0.1 * np.sin(2 * np.pi * n / 1000.0))
        assert orc.peos(p, r, p.T0) == pytest.approx(target, rel=1e-12)
        assert orc.dpdrho(p, r, p.T0) > 0 and r < 0.5  # vapour branch
    p.p_period = 0.0
    assert orc.peos(p, orc.inlet_density(p, 7), p.T0) == pytest.approx(1.1 * p0, rel=1e-12)


def test_pressure_driven_poiseuille(orc):
    Nx, Ny, steps = 160, 19, 12000
    p, tc = _open(orc, Nx, Ny, flags=orc.SINGLE_PHASE | orc.FREEZE_T)
    p.p_amp, p.p_period = 0.002, 0.0
    s = orc.Sim(p, rho_uniform=p.rho_v)
    s.step(steps)
    rho, ux, uy, _, _, _ = s.moments()
    rin = orc.inlet_density(p, steps)
    H, nu = Ny - 2, (p.tau_g - 0.5) / 3.0
    xm = Nx // 2
    dpdx = (rin - p.rho_v) / 3.0 / (Nx - 1)
    umax = dpdx * H * H / (8 * rho[Ny // 2, xm] * nu)
    y = np.arange(Ny) - 0.5  # walls at y = 1/2 and Ny - 3/2
    prof = dpdx / (2 * rho[Ny // 2, xm] * nu) * y * (H - y)
    assert ux[Ny // 2, xm] == pytest.approx(umax, rel=0.02)
    np.testing.assert_allclose(ux[1:-1, xm], prof[1:-1], rtol=0, atol=0.03 * umax)
    assert np.abs(uy[1:-1, xm]).max() < 1e-3 * umax


def test_linear_plate_and_inlet_temperature_held(orc):
    Nx, Ny = 30, 8
    p, tc = _open(orc, Nx, Ny)
    p.Tw, p.Tw_end, p.T_in = 0.86 * tc, 0.56 * tc, 0.86 * tc
    s = orc.Sim(p, rho_uniform=p.rho_v)
    s.step(20)
    T = s.moments()[3]
    ramp = 0.86 * tc + (0.56 - 0.86) * tc * np.arange(Nx) / (Nx - 1)
    np.testing.assert_allclose(T[0], ramp, rtol=1e-15)
    np.testing.assert_allclose(T[-1], ramp, rtol=1e-15)
    np.testing.assert_allclose(T[1:-1, 0], p.T_in, rtol=1e-15)
    assert np.abs(T[1:-1, -1] - p.T0).max() > 1e-6  # the outlet column evolves


@pytest.mark.parametrize("hold", [True, False])
def test_held_outlet_keeps_linear_profile(orc, hold):
    """T_out > 0 holds the outlet column at T_out.  Vapour at rest (both ends
    at p0, one phase) between plates carrying the same linear ramp from T_in
    to T_out: the linear field is a fixed point of the nine-point conduction
    term wherever both end columns are held, since every stencil then sees
    the linear field itself.  With the outlet evolving (T_out = 0) the
    zero-gradient ghost past it bends the profile next to it, which tells
    the two readings apart."""
    Nx, Ny = 24, 7
    p, tc = _open(orc, Nx, Ny, flags=orc.SINGLE_PHASE)
    p.p_amp = 0.0
    Tin, Tout = 0.86 * tc, 0.70 * tc
    p.Tw, p.Tw_end, p.T_in = Tin, Tout, Tin
    p.T_out = Tout if hold else 0.0
    s = orc.Sim(p, rho_uniform=p.rho_v)
    lin = Tin + (Tout - Tin) * np.arange(Nx) / (Nx - 1)
    s.set_T(np.broadcast_to(lin, (Ny, Nx)).copy())
    s.step(30)
    rho, ux, uy, T = s.moments()[:4]
    fl = slice(1, -1)
    assert np.abs(ux[fl]).max() < 1e-13 and np.abs(uy[fl]).max() < 1e-13
    if hold:
        np.testing.assert_allclose(T[fl, -1], Tout, rtol=1e-15)
        np.testing.assert_allclose(T[fl], np.broadcast_to(lin, (Ny - 2, Nx)), rtol=1e-13)
    else:
        assert np.abs(T[fl, -1] - Tout).max() > 1e-4 * tc

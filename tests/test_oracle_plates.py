"""Pins of the oracle's Sec. 3.2 plates (flag TOP_MIXED): the top plate holds
T_w on a band of cold columns and is adiabatic elsewhere, the bottom plate
holds its own temperature.

The plates are rows 0 and N = Ny-1.  An adiabatic top node mirrors the fluid
node below it (zero gradient at the half-way wall y = N - 1/2), so in a fluid
at rest (single phase, no drive, no gravity):

* top adiabatic everywhere, bottom held at T_b: T_b + eps cos(a x) sin(k y)
  with k = (2j+1) pi / (2N - 1) satisfies sin(k N) = sin(k (N-1)), hence it is
  an eigenvector of the nine-point Laplacian (diagonal neighbours included)
  with eigenvalue (4/3)(cos a + cos k - 2) + (2/3)(cos a cos k - 1), and the
  coupled step multiplies it by the RK4 factor R(z) exactly up to rounding;
* top cold everywhere at T_w = T_b: the Dirichlet modes sin(j pi y / N);
* top cold everywhere at T_w != T_b: the linear profile between the two
  plate temperatures is a fixed point;
* a band of cold columns: one step reaches four columns (one per RK stage),
  so columns farther than that from the band's ends evolve bit for bit as in
  the all-cold or all-adiabatic case.
"""
import numpy as np
import pytest


def _rk4_factor(z):
    return 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24


def _lap9(a, b):
    return 4 / 3 * (np.cos(a) + np.cos(b) - 2) + 2 / 3 * (np.cos(a) * np.cos(b) - 1)


def _params(orc, Nx, Ny, x0, x1, Tw, Tb, lam=0.3, Cv=1.7):
    p = orc.default_params(Nx=Nx, Ny=Ny, period=0.0, lam=lam, Cv=Cv,
                           flags=orc.SINGLE_PHASE | orc.TOP_MIXED)
    p.Tw, p.Tw_bot, p.cold_x0, p.cold_x1 = Tw, Tb, x0, x1
    return p


def _grid(Nx, Ny):
    y, x = np.mgrid[0:Ny, 0:Nx].astype(float)
    return x, y


@pytest.mark.parametrize("j,m", [(0, 0), (1, 1), (2, 3)])
def test_adiabatic_top_quarter_wave_decay(orc, j, m):
    Nx, Ny, steps, rho = 16, 11, 30, 0.9
    tc = orc.critical()[1]
    Tb = 0.86 * tc
    p = _params(orc, Nx, Ny, 0, 0, 0.65 * tc, Tb)
    N = Ny - 1
    k = (2 * j + 1) * np.pi / (2 * N - 1)
    a = 2 * np.pi * m / Nx
    x, y = _grid(Nx, Ny)
    mode = np.cos(a * x) * np.sin(k * y)
    eps = 1e-3 * Tb
    T0 = Tb + eps * mode
    T0[-1] = p.Tw  # the stored top value, never read on adiabatic columns
    s = orc.Sim(p, rho_uniform=rho)
    s.set_T(T0)
    s.step(steps)
    T = s.moments()[3]
    z = p.lam / (rho * p.Cv) * _lap9(a, k)
    expect = Tb + eps * _rk4_factor(z) ** steps * mode
    np.testing.assert_allclose(T[1:-1], expect[1:-1], rtol=0, atol=1e-13 * Tb)
    assert np.all(T[0] == Tb)


@pytest.mark.parametrize("j,m", [(1, 0), (2, 1)])
def test_cold_top_dirichlet_mode_decay(orc, j, m):
    Nx, Ny, steps, rho = 12, 9, 30, 1.1
    tc = orc.critical()[1]
    Tb = 0.7 * tc
    p = _params(orc, Nx, Ny, 0, Nx, Tb, Tb)
    N = Ny - 1
    k, a = j * np.pi / N, 2 * np.pi * m / Nx
    x, y = _grid(Nx, Ny)
    mode = np.cos(a * x) * np.sin(k * y)
    eps = 1e-3 * Tb
    s = orc.Sim(p, rho_uniform=rho)
    s.set_T(Tb + eps * mode)
    s.step(steps)
    T = s.moments()[3]
    z = p.lam / (rho * p.Cv) * _lap9(a, k)
    np.testing.assert_allclose(T, Tb + eps * _rk4_factor(z) ** steps * mode, rtol=0,
                               atol=1e-13 * Tb)


def test_linear_profile_between_plates_is_fixed(orc):
    Nx, Ny = 10, 13
    tc = orc.critical()[1]
    p = _params(orc, Nx, Ny, 0, Nx, 0.65 * tc, 0.86 * tc)
    _, y = _grid(Nx, Ny)
    lin = p.Tw_bot + (p.Tw - p.Tw_bot) * y / (Ny - 1)
    s = orc.Sim(p, rho_uniform=0.5)
    s.set_T(lin)
    s.step(20)
    np.testing.assert_allclose(s.moments()[3], lin, rtol=1e-14)
    # the same profile under an adiabatic top relaxes toward the bottom value
    q = _params(orc, Nx, Ny, 0, 0, 0.65 * tc, 0.86 * tc)
    s2 = orc.Sim(q, rho_uniform=0.5)
    s2.set_T(lin)
    s2.step(20)
    assert np.all(s2.moments()[3][1:-1] > lin[1:-1] + 1e-9 * tc)


def test_init_plate_temperatures(orc):
    tc = orc.critical()[1]
    p = _params(orc, 14, 7, 4, 9, 0.65 * tc, 0.8 * tc)
    T = orc.Sim(p, rho_uniform=0.4).moments()[3]
    assert np.all(T[0] == p.Tw_bot) and np.all(T[-1] == p.Tw) and np.all(T[1:-1] == p.T0)
    p.Tw_bot = 0.0  # unset: the bottom plate takes T0
    T = orc.Sim(p, rho_uniform=0.4).moments()[3]
    assert np.all(T[0] == p.T0)


def test_cold_band_is_local(orc):
    Nx, Ny, x0, x1 = 40, 12, 12, 28
    tc = orc.critical()[1]
    Tb = 0.86 * tc
    _, y = _grid(Nx, Ny)
    T0 = Tb - 0.05 * tc * (y / (Ny - 1)) ** 2
    out = {}
    for name, (a, b) in dict(mixed=(x0, x1), cold=(0, Nx), adiabatic=(0, 0)).items():
        p = _params(orc, Nx, Ny, a, b, 0.65 * tc, Tb)
        s = orc.Sim(p, rho_uniform=0.6)
        s.set_T(T0)
        s.step(1)
        out[name] = s.moments()[3]
    cols = np.arange(Nx)
    deep_cold = (cols - 4 >= x0) & (cols + 4 < x1)
    deep_adia = np.array([all(not (x0 <= (c + d) % Nx < x1) for d in range(-4, 5))
                          for c in cols])
    assert deep_cold.sum() == 8 and deep_adia.sum() == Nx - (x1 - x0) - 8
    assert np.array_equal(out["mixed"][:, deep_cold], out["cold"][:, deep_cold])
    assert np.array_equal(out["mixed"][:, deep_adia], out["adiabatic"][:, deep_adia])
    # at the band's ends the result lies between the two and differs from both
    edge = np.array([x0 - 1, x0, x1 - 1, x1])
    top = Ny - 2
    assert np.all(out["mixed"][top, edge] != out["cold"][top, edge])
    assert np.all(out["mixed"][top, edge] != out["adiabatic"][top, edge])


@pytest.mark.parametrize("x0,x1", [(7, 8), (5, 11), (6, 14)])
def test_cold_band_position(orc, x0, x1):
    """An x-uniform field under the band [x0, x1) stays symmetric about the
    band's centre (x0 + x1 - 1) / 2 and nowhere else: this fixes both ends,
    the first column in the band and the first one past it."""
    Nx, Ny = 20, 9
    tc = orc.critical()[1]
    Tb = 0.86 * tc
    _, y = _grid(Nx, Ny)
    p = _params(orc, Nx, Ny, x0, x1, 0.65 * tc, Tb)
    s = orc.Sim(p, rho_uniform=0.6)
    s.set_T(Tb - 0.05 * tc * (y / (Ny - 1)) ** 2)
    s.step(3)
    T = s.moments()[3][1:-1]
    cols = np.arange(Nx)
    for shift in (-1, 0, 1):
        refl = (x0 + x1 - 1 + shift - cols) % Nx
        sym = np.allclose(T, T[:, refl], rtol=1e-14, atol=0)
        assert sym == (shift == 0), shift

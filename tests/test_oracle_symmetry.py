"""Symmetry pins of the oracle's full step (arXiv:1803.01756 Eqs. 1-18 with
half-way bounce-back at the plates).

The D2Q9 velocity set, the MRT moments of Eqs. 2-3, the pair-force stencil of
Eq. 9 and the nine-point difference stencils of Eqs. 16-18 are all symmetric
under the lattice's reflections x -> -x and y -> -y, and, on a square box
periodic in both directions, under the exchange of x and y.  A step taken from
a reflected (or transposed) state must therefore give the reflected
(transposed) state, with the velocity components, the drive and gravity
transformed alike.  A wrong sign, a swapped population index or a transposed
operand in any x- or y-odd term (a source-term entry of Eq. 8, an odd moment,
a y-difference of a stencil, the plate adhesion of Eq. 14) breaks one of
these.  Every run starts from random populations about the vapour density
(so u is nonzero and every moment is off equilibrium) and a random
temperature field, two-phase with wall wettability and the oscillating drive
on, and the fields are compared after 40 steps; only the order of
floating-point sums differs between the two runs.
"""
import numpy as np
import pytest

# population index under each map (velocity order of Eq. 2:
# 0 rest, 1 +x, 2 +y, 3 -x, 4 -y, 5 (+,+), 6 (-,+), 7 (-,-), 8 (+,-))
FLIP_Y = [0, 1, 4, 3, 2, 8, 7, 6, 5]
FLIP_X = [0, 3, 2, 1, 4, 6, 5, 8, 7]
SWAP_XY = [0, 2, 1, 4, 3, 5, 8, 7, 6]
STEPS = 40


def _w():
    return np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def _random_state(orc, p, seed):
    rng = np.random.default_rng(seed)
    Ny, Nx = p.Ny, p.Nx
    rho = p.rho_v * (1.0 + 0.02 * (rng.random((Ny, Nx)) - 0.5))
    f = _w()[:, None, None] * rho[None] * (1.0 + 0.05 * (rng.random((9, Ny, Nx)) - 0.5))
    T = p.T0 * (1.0 + 0.01 * (rng.random((Ny, Nx)) - 0.5))
    return f, T


def _run(orc, p, f, T):
    s = orc.Sim(p, rho_uniform=p.rho_v)
    s.set_f(f)
    s.set_T(T)
    s.step(STEPS)
    rho, ux, uy, Tn, _, _ = s.moments()
    return rho, ux, uy, Tn


def _close(a, b, tol=1e-11):
    scale = max(np.abs(b).max(), 1e-300)
    assert np.abs(a - b).max() <= tol * scale, np.abs(a - b).max() / scale


def _params(orc, Nx, Ny, flags=0, **kw):
    tc = orc.critical()[1]
    d = dict(Nx=Nx, Ny=Ny, flags=flags, Tw=0.8 * tc, Gw=-1.0, psiw=0.3, g_osc=2e-5,
             period=60.0)
    d.update(kw)
    return orc.default_params(**d)


@pytest.mark.parametrize("gy", [0.0, -3e-5])
def test_step_commutes_with_y_reflection(orc, gy):
    """Plate channel mirrored about its mid-plane (the plates trade places):
    rho, T, u_x mirror, u_y mirrors with a sign, gravity along y flips."""
    p = _params(orc, 36, 22, gy=gy)
    q = _params(orc, 36, 22, gy=-gy)
    f, T = _random_state(orc, p, 11)
    a = _run(orc, p, f, T)
    b = _run(orc, q, f[FLIP_Y][:, ::-1, :], T[::-1, :])
    _close(b[0], a[0][::-1, :])
    _close(b[1], a[1][::-1, :])
    _close(b[2], -a[2][::-1, :])
    _close(b[3], a[3][::-1, :])


def test_step_commutes_with_x_reflection(orc):
    """Columns reversed (periodic x): u_x and the x drive change sign."""
    p = _params(orc, 36, 22, gx=2e-5)
    q = _params(orc, 36, 22, gx=-2e-5, g_osc=-p.g_osc)
    f, T = _random_state(orc, p, 12)
    a = _run(orc, p, f, T)
    b = _run(orc, q, f[FLIP_X][:, :, ::-1], T[:, ::-1])
    _close(b[0], a[0][:, ::-1])
    _close(b[1], -a[1][:, ::-1])
    _close(b[2], a[2][:, ::-1])
    _close(b[3], a[3][:, ::-1])


def test_step_commutes_with_transpose_on_periodic_box(orc):
    """Square box periodic in x and y: exchanging x and y exchanges u_x and
    u_y, with a body force along x becoming one along y."""
    p = _params(orc, 24, 24, flags=orc.PERIODIC_Y, g_osc=0.0, period=0.0, gx=3e-5, gy=-1e-5)
    q = _params(orc, 24, 24, flags=orc.PERIODIC_Y, g_osc=0.0, period=0.0, gx=-1e-5, gy=3e-5)
    f, T = _random_state(orc, p, 13)
    a = _run(orc, p, f, T)
    b = _run(orc, q, np.transpose(f[SWAP_XY], (0, 2, 1)), T.T)
    _close(b[0], a[0].T)
    _close(b[1], a[2].T)
    _close(b[2], a[1].T)
    _close(b[3], a[3].T)


def test_step_commutes_with_periodic_shift(orc):
    """Translation along the periodic x direction: no term may depend on
    the absolute column."""
    p = _params(orc, 36, 22)
    f, T = _random_state(orc, p, 14)
    a = _run(orc, p, f, T)
    k = 13
    b = _run(orc, p, np.roll(f, k, axis=2), np.roll(T, k, axis=1))
    for x, y in zip(b, a):
        _close(x, np.roll(y, k, axis=1), tol=1e-13)


def test_y_reflection_pin_is_not_vacuous(orc):
    """u_y is far from zero in these runs, so the comparison above would see
    a y-odd quantity that came out with the wrong sign."""
    p = _params(orc, 36, 22)
    f, T = _random_state(orc, p, 15)
    a = _run(orc, p, f, T)
    b = _run(orc, p, f[FLIP_Y][:, ::-1, :], T[::-1, :])
    with pytest.raises(AssertionError):
        _close(b[2], a[2][::-1, :])

"""Pins of the oracle's temperature update (arXiv:1803.01756 Eqs. 16-18).

* K(T) on polynomial fields where the nine-point stencils are exact: the
  advection term on a linear T, the conduction term on a quadratic T and the
  compression term on a linear velocity field, with (dP/dT)_rho taken from
  central differences of P_EOS.
* The full coupled step on Fourier modes of T in a periodic box at rest (and
  in uniform motion): the stencils map exp(ikx) to i sin(k) (gradient) and
  2 (cos k - 1) (Laplacian), so classical RK4 multiplies the mode by
  R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 per step, exactly up to rounding.
  The printed weights (h1 + h2 + h3 + h4)/6 of Eq. 17 would give
  1 + 2z/3 + ... and fail.
* The diffusivity cap alpha_max (a departure from Eq. 17 at delta t = 1 for
  vapour thinner than the RK4 bound allows): the conduction term is linear
  in lambda, so the capped right-hand side is the uncapped one with its
  conduction part scaled by min(1, alpha_max rho C_v / lambda) node by
  node; on modes it turns R(z D) into R(z alpha_max), which decays where
  the uncapped scheme grows.
"""
import numpy as np
import pytest

E = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1),
              (1, 1), (-1, 1), (-1, -1), (1, -1)], dtype=float)
W_EQ = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def _grid(Nx, Ny):
    y, x = np.mgrid[0:Ny, 0:Nx].astype(float)
    return x, y


def test_advection_term_exact_on_linear_field(orc):
    Nx, Ny = 9, 7
    p = orc.default_params(Nx=Nx, Ny=Ny, flags=orc.PERIODIC_Y, lam=0.0)
    x, y = _grid(Nx, Ny)
    rng = np.random.default_rng(0)
    rho = rng.uniform(0.3, 6.0, (Ny, Nx))
    ux, uy = np.full((Ny, Nx), 0.03), np.full((Ny, Nx), -0.02)
    T = p.T0 + 1e-3 * x - 2e-3 * y
    K = orc.heat_rhs(p, rho, ux, uy, T)
    inner = (slice(1, -1), slice(1, -1))
    np.testing.assert_allclose(K[inner], -(0.03 * 1e-3 + 0.02 * 2e-3), rtol=1e-12)


def test_conduction_term_exact_on_quadratic_field(orc):
    Nx, Ny = 9, 7
    p = orc.default_params(Nx=Nx, Ny=Ny, flags=orc.PERIODIC_Y, lam=0.37, Cv=4.0)
    x, y = _grid(Nx, Ny)
    rng = np.random.default_rng(1)
    rho = rng.uniform(0.3, 6.0, (Ny, Nx))
    zero = np.zeros((Ny, Nx))
    T = p.T0 + 1e-4 * (3 * x ** 2 - 2 * x * y + 5 * y ** 2 + x)
    K = orc.heat_rhs(p, rho, zero, zero, T)
    lapT = 1e-4 * (6 + 10)
    inner = (slice(1, -1), slice(1, -1))
    np.testing.assert_allclose(K[inner], (0.37 / (rho * 4.0) * lapT)[inner], rtol=1e-10)


def test_compression_term_on_linear_velocity(orc):
    Nx, Ny = 9, 7
    p = orc.default_params(Nx=Nx, Ny=Ny, flags=orc.PERIODIC_Y)
    x, y = _grid(Nx, Ny)
    rng = np.random.default_rng(2)
    rho = rng.uniform(0.3, 6.0, (Ny, Nx))
    ux = 1e-3 * (2 * x - y)
    uy = 1e-3 * (x + 3 * y)
    T = np.full((Ny, Nx), p.T0)
    K = orc.heat_rhs(p, rho, ux, uy, T)
    div = 1e-3 * (2 + 3)
    h = 1e-6 * p.T0
    inner = (slice(1, -1), slice(1, -1))
    for j in range(1, Ny - 1):
        for i in range(1, Nx - 1):
            r = rho[j, i]
            dpdT = (orc.peos(p, r, p.T0 + h) - orc.peos(p, r, p.T0 - h)) / (2 * h)
            expect = -p.T0 / (r * p.Cv) * dpdT * div
            assert abs(K[j, i] - expect) < 1e-8 * abs(expect)
    assert np.isfinite(K[inner]).all()


def test_walls_hold_dirichlet_temperature(orc):
    """Solid rows keep T_w through a step; a fluid at T_w next to the wall at
    rest stays at T_w (K = 0)."""
    Nx, Ny = 8, 6
    p = orc.default_params(Nx=Nx, Ny=Ny, flags=orc.SINGLE_PHASE, period=0.0,
                           T0=0.8 * orc.critical()[1], Tw=0.8 * orc.critical()[1])
    s = orc.Sim(p, rho_uniform=0.5)
    s.step(5)
    T = s.moments()[3]
    np.testing.assert_allclose(T, p.Tw, rtol=1e-14)


def _rk4_factor(z):
    return 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24


@pytest.mark.parametrize("mode,rho", [(1, 0.38), (3, 1.0), (5, 6.5)])
def test_rk4_conduction_mode_decay(orc, mode, rho):
    Nx, Ny, steps = 24, 3, 40
    p = orc.default_params(Nx=Nx, Ny=Ny, flags=orc.PERIODIC_Y | orc.SINGLE_PHASE,
                           period=0.0, lam=0.2, Cv=1.3)
    s = orc.Sim(p, rho_uniform=rho)
    x, _ = _grid(Nx, Ny)
    k = 2 * np.pi * mode / Nx
    eps = 1e-3 * p.T0
    s.set_T(p.T0 + eps * np.sin(k * x))
    s.step(steps)
    T = s.moments()[3]
    z = p.lam / (rho * p.Cv) * 2 * (np.cos(k) - 1)
    expect = p.T0 + eps * _rk4_factor(z) ** steps * np.sin(k * x)
    np.testing.assert_allclose(T, expect, rtol=0, atol=1e-13 * p.T0)


def test_rk4_advection_mode(orc):
    """Uniform flow U along x (set as the textbook equilibrium) carries the
    mode: z = -i U sin k + D 2 (cos k - 1)."""
    Nx, Ny, steps, U, rho = 20, 3, 60, 0.05, 0.8
    p = orc.default_params(Nx=Nx, Ny=Ny, flags=orc.PERIODIC_Y | orc.SINGLE_PHASE,
                           period=0.0, lam=0.05, Cv=2.0)
    s = orc.Sim(p, rho_uniform=rho)
    eu = E @ np.array([U, 0.0])
    feq = W_EQ * rho * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * U * U)
    s.set_f(np.broadcast_to(feq[:, None, None], (9, Ny, Nx)).copy())
    x, _ = _grid(Nx, Ny)
    k = 2 * np.pi * 2 / Nx
    eps = 1e-3 * p.T0
    s.set_T(p.T0 + eps * np.sin(k * x))
    s.step(steps)
    _, ux, uy, T, _, _ = s.moments()
    np.testing.assert_allclose(ux, U, rtol=1e-13)
    z = -1j * U * np.sin(k) + p.lam / (rho * p.Cv) * 2 * (np.cos(k) - 1)
    expect = p.T0 + np.real(-1j * eps * _rk4_factor(z) ** steps * np.exp(1j * k * x))
    np.testing.assert_allclose(T, expect, rtol=0, atol=1e-13 * p.T0)


@pytest.mark.parametrize("k,l", [(1, 1), (2, 3)])
def test_frame_held_box_mode_decay(orc, k, l):
    """FRAME_T box at rest: the frame holds T_w, and a product of sines that
    vanishes on the frame is an eigenvector of the nine-point Laplacian with
    eigenvalue (4/3)(cos a + cos b - 2) + (2/3)(cos a cos b - 1), so the
    coupled step multiplies it by R(z) exactly up to rounding."""
    Nx, Ny, steps, rho = 12, 9, 30, 0.9
    p = orc.default_params(Nx=Nx, Ny=Ny, period=0.0, lam=0.3, Cv=1.7,
                           flags=orc.PERIODIC_Y | orc.SINGLE_PHASE | orc.FRAME_T)
    p.Tw = 0.9 * orc.critical()[1]
    s = orc.Sim(p, rho_uniform=rho)
    x, y = _grid(Nx, Ny)
    a, b = k * np.pi / (Nx - 1), l * np.pi / (Ny - 1)
    eps = 1e-3 * p.Tw
    mode = np.sin(a * x) * np.sin(b * y)
    s.set_T(p.Tw + eps * mode)
    s.step(steps)
    T = s.moments()[3]
    lam9 = 4 / 3 * (np.cos(a) + np.cos(b) - 2) + 2 / 3 * (np.cos(a) * np.cos(b) - 1)
    z = p.lam / (rho * p.Cv) * lam9
    np.testing.assert_allclose(T, p.Tw + eps * _rk4_factor(z) ** steps * mode, rtol=0,
                               atol=1e-13 * p.Tw)


def test_frame_temperature_held_with_flow(orc):
    """A two-phase box with FRAME_T: the frame nodes keep T_w exactly while
    the interior evolves; without the flag the frame nodes move."""
    Nx, Ny = 16, 12
    tc = orc.critical()[1]
    p = orc.default_params(Nx=Nx, Ny=Ny, period=0.0, flags=orc.PERIODIC_Y | orc.FRAME_T)
    p.Tw = tc
    x, y = _grid(Nx, Ny)
    r = np.hypot(x - Nx / 2, y - Ny / 2)
    rho0 = 0.5 * (p.rho_l + p.rho_g) - 0.5 * (p.rho_l - p.rho_g) * np.tanh(2 * (r - 4) / 3)
    s = orc.Sim(p, rho0)
    s.step(20)
    T = s.moments()[3]
    frame = np.zeros((Ny, Nx), dtype=bool)
    frame[0] = frame[-1] = True
    frame[:, 0] = frame[:, -1] = True
    assert np.all(T[frame] == p.Tw)
    assert np.abs(T[~frame] - p.T0).max() > 1e-6
    q = orc.default_params(Nx=Nx, Ny=Ny, period=0.0, flags=orc.PERIODIC_Y)
    q.Tw = tc
    s2 = orc.Sim(q, rho0)
    s2.step(20)
    assert np.abs(s2.moments()[3][frame] - p.Tw).min() > 1e-3 * tc


def test_reservoir_frame_uniform_equilibrium(orc):
    """FRAME_RHO | FRAME_T box whose interior already matches the reservoir
    (rho = rho_frame, T = T_w, at rest): nothing moves, with the two-phase
    EOS and forces on (uniform psi gives no force)."""
    Nx, Ny = 10, 8
    tc = orc.critical()[1]
    p = orc.default_params(Nx=Nx, Ny=Ny, period=0.0,
                           flags=orc.PERIODIC_Y | orc.FRAME_T | orc.FRAME_RHO)
    p.Tw = p.T0 = 0.9 * tc
    p.rho_frame = 0.3
    s = orc.Sim(p, rho_uniform=0.3)
    s.step(25)
    rho, ux, uy, T, _, _ = s.moments()
    np.testing.assert_allclose(rho, 0.3, rtol=1e-14)
    assert np.abs(ux).max() < 1e-15 and np.abs(uy).max() < 1e-15
    np.testing.assert_allclose(T, p.Tw, rtol=1e-14)


def test_reservoir_frame_values_held(orc):
    """A droplet in a FRAME_RHO | FRAME_T box: the frame keeps rho_frame,
    u = 0 and T_w exactly; mass leaves or enters through it (the interior
    vapour starts at rho_g, the reservoir is thinner)."""
    Nx, Ny = 18, 14
    tc = orc.critical()[1]
    p = orc.default_params(Nx=Nx, Ny=Ny, period=0.0,
                           flags=orc.PERIODIC_Y | orc.FRAME_T | orc.FRAME_RHO)
    p.Tw = tc
    p.rho_frame = 0.29
    x, y = _grid(Nx, Ny)
    r = np.hypot(x - (Nx - 1) / 2, y - (Ny - 1) / 2)
    rho0 = 0.5 * (p.rho_l + p.rho_g) - 0.5 * (p.rho_l - p.rho_g) * np.tanh(2 * (r - 4) / 3)
    s = orc.Sim(p, rho0)
    s.step(30)
    rho, ux, uy, T, _, _ = s.moments()
    frame = np.zeros((Ny, Nx), dtype=bool)
    frame[0] = frame[-1] = True
    frame[:, 0] = frame[:, -1] = True
    assert np.all(rho[frame] == 0.29) and np.all(ux[frame] == 0) and np.all(uy[frame] == 0)
    assert np.all(T[frame] == p.Tw)
    assert abs(rho[~frame].sum() - rho0[~frame].sum()) > 1e-6 * rho0.sum()


def test_phase_props_reduce_to_constant_properties(orc):
    """PHASE_PROPS with equal gas and liquid values is the constant-property
    energy equation."""
    Nx, Ny = 11, 9
    p = orc.default_params(Nx=Nx, Ny=Ny, flags=orc.PERIODIC_Y, lam=0.2, Cv=3.0)
    x, y = _grid(Nx, Ny)
    rng = np.random.default_rng(5)
    rho = rng.uniform(0.3, 6.5, (Ny, Nx))
    ux, uy = rng.uniform(-0.05, 0.05, (2, Ny, Nx))
    T = p.T0 * (1 + 0.01 * rng.uniform(-1, 1, (Ny, Nx)))
    K0 = orc.heat_rhs(p, rho, ux, uy, T)
    p.flags |= orc.PHASE_PROPS
    p.lam_l, p.Cv_l = p.lam, p.Cv
    np.testing.assert_allclose(orc.heat_rhs(p, rho, ux, uy, T), K0, rtol=1e-13, atol=1e-18)


def test_phase_props_conduction_exact_on_polynomials(orc):
    """rho linear in x inside (rho_g, rho_l) makes lambda(rho) linear,
    T = T0 + b x^2: the nine-point form lambda lap T + grad(lambda) . grad(T)
    equals d/dx[(l0 + a x) 2 b x] = 2 b lambda(x) + 2 a b x exactly; divided
    by rho C_v(rho) with C_v interpolated the same way."""
    Nx, Ny = 15, 7
    p = orc.default_params(Nx=Nx, Ny=Ny, flags=orc.PERIODIC_Y | orc.PHASE_PROPS,
                           lam=0.1, Cv=4.0)
    p.lam_l, p.Cv_l = 0.6, 2.5
    x, y = _grid(Nx, Ny)
    frac = 0.1 + 0.05 * x
    rho = p.rho_g + frac * (p.rho_l - p.rho_g)
    bT = 1e-5
    T = p.T0 + bT * x * x
    K = orc.heat_rhs(p, rho, np.zeros_like(rho), np.zeros_like(rho), T)
    lam = p.lam + (p.lam_l - p.lam) * frac
    a = (p.lam_l - p.lam) * 0.05
    cv = p.Cv + (p.Cv_l - p.Cv) * frac
    expect = (2 * bT * lam + a * 2 * bT * x) / (rho * cv)
    inner = (slice(None), slice(1, -1))
    np.testing.assert_allclose(K[inner], expect[inner], rtol=1e-10)


@pytest.mark.parametrize("D", [0.50, 0.55])
def test_rk4_stability_bound_on_checkerboard(orc, D):
    """The checkerboard mode (-1)^(x+y) is the nine-point Laplacian's extreme
    eigenvector (eigenvalue -16/3), so the step multiplies it by R(-16 D / 3)
    with D = lambda / (rho C_v): it decays for D below 2.785 * 3 / 16 = 0.522
    and grows above; the stated bound on the thin-vapour stability follows."""
    Nx = Ny = 8
    rho, Cv = 0.4, 5.0
    p = orc.default_params(Nx=Nx, Ny=Ny, flags=orc.PERIODIC_Y | orc.SINGLE_PHASE,
                           period=0.0, lam=D * rho * Cv, Cv=Cv)
    s = orc.Sim(p, rho_uniform=rho)
    x, y = _grid(Nx, Ny)
    mode = (-1.0) ** (x + y)
    eps = 1e-6 * p.T0
    s.set_T(p.T0 + eps * mode)
    s.step(10)
    T = s.moments()[3]
    r = _rk4_factor(-16.0 * D / 3.0)
    np.testing.assert_allclose(T, p.T0 + eps * r ** 10 * mode, rtol=0, atol=1e-12 * p.T0)
    assert (abs(r) < 1) == (D < 0.522)


@pytest.mark.parametrize("D,cap", [(1.0, 0.25), (11.7, 0.5)])
@pytest.mark.parametrize("mode", ["checkerboard", "sine"])
def test_diffusivity_cap_on_modes(orc, D, cap, mode):
    """D = 11.7 is lambda / (rho C_v) of saturated vapour at 0.56 T_c with the
    paper's lambda and C_v; uncapped, the checkerboard mode grows at both D
    (|R| > 1), the longest sine mode at D = 11.7."""
    Nx = Ny = 8
    rho, Cv = 0.4, 5.0
    p = orc.default_params(Nx=Nx, Ny=Ny, flags=orc.PERIODIC_Y | orc.SINGLE_PHASE,
                           period=0.0, lam=D * rho * Cv, Cv=Cv)
    p.alpha_max = cap
    s = orc.Sim(p, rho_uniform=rho)
    x, y = _grid(Nx, Ny)
    if mode == "checkerboard":
        f, ev = (-1.0) ** (x + y), -16.0 / 3.0
    else:
        k = 2 * np.pi / Nx
        f, ev = np.sin(k * x), 2 * (np.cos(k) - 1)
    eps = 1e-6 * p.T0
    s.set_T(p.T0 + eps * f)
    s.step(10)
    T = s.moments()[3]
    r = _rk4_factor(ev * cap)
    np.testing.assert_allclose(T, p.T0 + eps * r ** 10 * f, rtol=0, atol=1e-12 * p.T0)
    assert abs(r) < 1
    if mode == "checkerboard":
        assert abs(_rk4_factor(ev * D)) > 1


@pytest.mark.parametrize("props", [False, True])
def test_diffusivity_cap_scales_conduction_node_by_node(orc, props):
    """K(T) with the cap against its decomposition: K with lambda = 0 (and
    lambda_l = 0) is the advection and compression part, the rest is the
    conduction part, which the cap scales by min(1, alpha_max / alpha) with
    alpha = lambda(rho) / (rho C_v(rho)); densities from vapour to liquid put
    alpha on both sides of the cap."""
    Nx, Ny = 13, 9
    p = orc.default_params(Nx=Nx, Ny=Ny, flags=orc.PERIODIC_Y, lam=0.25, Cv=5.0)
    if props:
        p.flags |= orc.PHASE_PROPS
        p.lam_l, p.Cv_l = 0.6, 2.5
    rng = np.random.default_rng(17)
    rho = np.exp(rng.uniform(np.log(0.03), np.log(6.5), (Ny, Nx)))
    ux, uy = rng.uniform(-0.05, 0.05, (2, Ny, Nx))
    T = p.T0 * (1 + 0.01 * rng.uniform(-1, 1, (Ny, Nx)))
    full = orc.heat_rhs(p, rho, ux, uy, T)
    lam, lam_l = p.lam, p.lam_l
    p.lam, p.lam_l = 0.0, 0.0
    rest = orc.heat_rhs(p, rho, ux, uy, T)
    p.lam, p.lam_l = lam, lam_l
    if props:
        fr = np.clip((rho - p.rho_g) / (p.rho_l - p.rho_g), 0, 1)
        alpha = (lam + (lam_l - lam) * fr) / (rho * (p.Cv + (p.Cv_l - p.Cv) * fr))
    else:
        alpha = lam / (rho * p.Cv)
    cap = 0.4
    assert (alpha > cap).sum() > 5 and (alpha < cap).sum() > 5
    p.alpha_max = cap
    capped = orc.heat_rhs(p, rho, ux, uy, T)
    expect = rest + (full - rest) * np.minimum(1.0, cap / alpha)
    np.testing.assert_allclose(capped, expect, rtol=1e-12, atol=1e-14 * np.abs(full).max())
    # a cap above every node's diffusivity changes nothing, bit for bit
    p.alpha_max = 1.01 * alpha.max()
    assert np.array_equal(orc.heat_rhs(p, rho, ux, uy, T), full)

"""Pins of the oracle's lattice algebra (arXiv:1803.01756 Eqs. 2, 6-8, 13)
against definitions that do not come from the oracle's own tables.

* The rows of M are checked against the polynomial moment definitions of
  Lallemand & Luo (the paper's ref. [15]), built here from the verbal
  velocity set of Eq. 2.
* With every relaxation rate equal to 1/tau and theta = 0 the MRT collision
  with Li's source must reduce to textbook BGK with Guo's forcing term
  (Guo, Zheng & Shi, PRE 65, 046308, 2002) and the textbook second-order
  equilibrium.  A dropped 1/rho in the equilibrium moments, a sign or an
  antisymmetric p_xy source term (the two printed forms of Eq. 6/8 that the
  oracle reads differently) fail this comparison.
"""
import numpy as np
import pytest

# Eq. 2 in words: rest, then the four axis directions counter-clockwise from
# +x, then the four diagonals counter-clockwise from (1, 1).
E = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1),
              (1, 1), (-1, 1), (-1, -1), (1, -1)], dtype=float)
W_EQ = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)  # textbook D2Q9 weights


def textbook_feq(rho, u):
    eu = E @ u
    return W_EQ * rho * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * (u @ u))


def guo_forcing(u, F, tau):
    eu = E @ u
    return (1 - 0.5 / tau) * W_EQ * (3 * ((E - u) @ F) + 9 * eu * (E @ F))


def test_M_rows_are_lallemand_luo_moments(orc):
    M = orc.matrix_M()
    e2 = (E ** 2).sum(1)
    ex, ey = E[:, 0], E[:, 1]
    rows = [np.ones(9), -4 + 3 * e2, 4 - 10.5 * e2 + 4.5 * e2 ** 2, ex, (-5 + 3 * e2) * ex,
            ey, (-5 + 3 * e2) * ey, ex ** 2 - ey ** 2, ex * ey]
    np.testing.assert_array_equal(M, np.array(rows))


def test_Minv_is_inverse_and_orthogonal_form(orc):
    M, Mi = orc.matrix_M(), orc.matrix_Minv()
    np.testing.assert_allclose(M @ Mi, np.eye(9), atol=1e-14)
    norms = (M * M).sum(1)
    np.testing.assert_array_equal(norms, [9, 36, 36, 6, 12, 6, 12, 4, 4])
    np.testing.assert_allclose(Mi, M.T / norms, atol=1e-15)


def test_rest_equilibrium_has_textbook_weights(orc):
    p = orc.default_params(Nx=3, Ny=3, flags=orc.PERIODIC_Y)
    s = orc.Sim(p, rho_uniform=0.7)
    f = s.get_f()
    for i in range(9):
        np.testing.assert_allclose(f[i], 0.7 * W_EQ[i], rtol=1e-15)


@pytest.mark.parametrize("rho", [0.3796, 1.0, 6.4992])
def test_equilibrium_moments_are_textbook_feq(orc, rho):
    """All rates 1 and no force: f* = M^-1 m_eq(rho, rho u) must be the
    second-order polynomial equilibrium, for rho != 1 too (pins the 1/rho)."""
    p = orc.default_params(s_rho=1.0, s_e=1.0, s_zeta=1.0, s_j=1.0, s_q=1.0, theta=0.0)
    rng = np.random.default_rng(3)
    f = W_EQ * rho * (1 + 0.05 * rng.standard_normal(9))
    r = f.sum()
    u = (E.T @ f) / r
    out = orc.collide_node(p, f, r, u[0], u[1], 0, 0, 0, 0, 0.4, 1.0)
    np.testing.assert_allclose(out, textbook_feq(r, u), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_bgk_guo_special_case(orc, tau):
    p = orc.default_params(s_rho=1 / tau, s_e=1 / tau, s_zeta=1 / tau, s_j=1 / tau,
                           s_q=1 / tau, theta=0.0)
    rng = np.random.default_rng(int(tau * 10))
    for rho in (0.38, 2.0, 6.5):
        f = W_EQ * rho * (1 + 0.1 * rng.standard_normal(9))
        F = 1e-2 * rng.standard_normal(2)
        r = f.sum()
        u = (E.T @ f + 0.5 * F) / r
        out = orc.collide_node(p, f, r, u[0], u[1], F[0], F[1], 0.3 * F[0], 0.3 * F[1],
                               0.5, tau)
        ref = f - (f - textbook_feq(r, u)) / tau + guo_forcing(u, F, tau)
        np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-14)


def test_collision_conserves_mass_and_adds_momentum(orc):
    """Eq. 7 with arbitrary rates: sum f* = sum f and sum e f* = sum e f + F
    (m_3 and m_5 are relaxed towards j = rho u, which already holds F/2)."""
    p = orc.default_params(s_rho=0.7, s_e=1.3, s_zeta=1.3, s_j=0.9, s_q=1.6, theta=0.104)
    rng = np.random.default_rng(11)
    for _ in range(20):
        rho = rng.uniform(0.2, 7.0)
        f = W_EQ * rho * (1 + 0.2 * rng.standard_normal(9))
        F = 1e-2 * rng.standard_normal(2)
        Fm = 1e-2 * rng.standard_normal(2)
        r = f.sum()
        u = (E.T @ f + 0.5 * F) / r
        out = orc.collide_node(p, f, r, u[0], u[1], F[0], F[1], Fm[0], Fm[1],
                               rng.uniform(0.2, 0.6), rng.uniform(0.6, 1.5))
        assert abs(out.sum() - f.sum()) <= 1e-14 * abs(f).sum()
        np.testing.assert_allclose(E.T @ out, E.T @ f + F, rtol=0, atol=1e-14 * abs(f).sum())


def test_theta_term_acts_on_energy_moments_only(orc):
    """Eq. 7-8: (1 - s/2) * 12 theta |F_m|^2 / (psi^2 (tau - 1/2)) equals
    s * 12 theta |F_m|^2 / psi^2 for s = 1/tau, so switching theta on moves
    m*_1 by +s_e c and m*_2 by -s_zeta c (c = 12 theta |F_m|^2 / psi^2) and
    leaves every other moment unchanged."""
    M = orc.matrix_M()
    rng = np.random.default_rng(5)
    f = W_EQ * 1.3 * (1 + 0.1 * rng.standard_normal(9))
    F, Fm, psi = np.array([3e-3, -2e-3]), np.array([2e-3, 1e-3]), 0.45
    r = f.sum()
    u = (E.T @ f + 0.5 * F) / r
    outs = []
    for th in (0.0, 0.2):
        p = orc.default_params(s_e=0.8, s_zeta=1.2, theta=th)
        outs.append(orc.collide_node(p, f, r, u[0], u[1], F[0], F[1], Fm[0], Fm[1], psi, 1.0))
    dm = M @ (outs[1] - outs[0])
    c = 12 * 0.2 * (Fm @ Fm) / psi ** 2
    expect = np.zeros(9)
    expect[1], expect[2] = 0.8 * c, -1.2 * c
    np.testing.assert_allclose(dm, expect, atol=1e-15)


def test_force_weights_are_isotropic():
    """Eq. 9 weights: sum_i w_i e_i e_i^T = I and sum_i w_i e_i = 0."""
    w = np.array([0] + [1 / 3] * 4 + [1 / 12] * 4)
    np.testing.assert_allclose((w[:, None, None] * E[:, :, None] * E[:, None, :]).sum(0),
                               np.eye(2), atol=1e-15)
    np.testing.assert_allclose((w[:, None] * E).sum(0), 0.0, atol=1e-15)

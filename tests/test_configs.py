"""The paper-case parameter builders hold the readings they document (host
only, no GPU): the Sec. 3.1 evaporation box, the Sec. 3.2 gravity box, the
Sec. 3.3 open channel, the Carnahan-Starling channel and the measured
channel workloads."""
import pytest

from paper_1803_01756_amd import configs, lbm


def _psi_w_for(p, angle):
    frac = configs.wall_fraction_for_angle(angle)
    return lbm.lbm_eos_pressure(p, p.rho_g + frac * (p.rho_l - p.rho_g), p.T_0)[1]


def test_gravity_plate_readings():
    p = configs.gravity_plate()
    assert (p.Nx, p.Ny) == (100, 300)
    assert p.flags == lbm.LBM_TOP_MIXED
    assert (p.cold_x0, p.cold_x1) == (33, 66)  # the middle third
    assert p.T_w == pytest.approx(0.65 * p.T_c, rel=1e-15)
    assert p.T_0 == pytest.approx(0.86 * p.T_c, rel=1e-15)
    assert p.T_w_bottom == p.T_0
    assert (p.g_x, p.g_y, p.g_osc) == (0.0, -1e-4, 0.0)
    assert p.G_w == p.G and p.psi_w == pytest.approx(_psi_w_for(p, 137.82), rel=1e-12)


def test_open_channel_readings():
    p = configs.open_channel()
    assert (p.Nx, p.Ny) == (1600, 48)
    assert p.flags == lbm.LBM_OPEN_X
    assert p.T_w == pytest.approx(0.86 * p.T_c, rel=1e-15)
    assert p.T_w_end == pytest.approx(0.56 * p.T_c, rel=1e-15)
    assert p.T_in == p.T_0
    assert (p.p_amp, p.g_x, p.g_y, p.g_osc) == (0.1, 1e-4, 0.0, 0.0)
    assert p.psi_w == pytest.approx(_psi_w_for(p, 137.82), rel=1e-12)


@pytest.mark.parametrize("lam", [1.0 / 3.0, 2.0 / 3.0])
def test_d2_box_readings(lam):
    p = configs.d2_box(lam, N=200)
    assert (p.Nx, p.Ny) == (200, 200)
    assert p.flags == lbm.LBM_PERIODIC_Y | lbm.LBM_FRAME_T | lbm.LBM_FRAME_RHO
    assert p.T_w == p.T_c and p.lambda_ == lam and p.g_osc == 0.0
    # the reservoir is at the saturation pressure of T_sat = T_0, at T_c
    p_sat = lbm.lbm_eos_pressure(p, p.rho_g, p.T_0)[0]
    assert lbm.lbm_eos_pressure(p, p.rho_frame, p.T_c)[0] == pytest.approx(p_sat, rel=1e-12)
    assert 0 < p.rho_frame < p.rho_g


def test_cs_channel_readings():
    p = configs.channel_params_cs(96, 24)
    assert p.flags & lbm.LBM_EOS_CS
    assert (p.a, p.b, p.R) == (1.0, 4.0, 1.0)
    assert p.T_c == pytest.approx(0.0943, abs=5e-5)
    assert p.lambda_ == 0.05


def test_measured_channels():
    big = configs.large_channel()
    assert (big.Nx, big.Ny, big.precision) == (8192, 512, lbm.LBM_FP32_DEV)
    assert big.T_w == pytest.approx(0.78 * big.T_c, rel=1e-15)
    assert big.psi_w == pytest.approx(_psi_w_for(big, 75.0), rel=1e-12)
    assert (big.g_osc, big.period) == (2e-6, 4000.0)
    mid = configs.single_gpu_channel(60.0)
    assert (mid.Nx, mid.Ny, mid.period) == (2048, 256, 4000.0)
    small = configs.oracle_size_channel()
    assert (small.Nx, small.Ny, small.g_osc, small.period) == (128, 32, 1e-6, 2000.0)

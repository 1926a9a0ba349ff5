"""CPU checks of the C-ABI boundary: the library loads, exports every entry
point that include/lbm.h declares, and the host-side parameter logic
(resolution, validation, EOS solvers) works without a GPU."""
import os
import re

import numpy as np
import pytest

from paper_1803_01756_amd import configs, lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", txt)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(lbm.LIB_PATH):
        from paper_1803_01756_amd import build
        build.build()
    return lbm.lib()


def test_library_exports_every_declared_symbol(L):
    names = _declared()
    assert "lbm_create" in names and "lbm_step" in names
    for n in names:
        assert hasattr(L, n), n


def test_binding_names_match_header():
    assert set(lbm.exported_symbols()) <= set(_declared())


def test_params_default_and_resolve(L, orc):
    p = lbm.lbm_params_resolve(lbm.lbm_params_default())
    _, tc = orc.critical()
    assert abs(p.T_c / tc - 1) < 1e-12
    op = orc.default_params()
    g, l, _ = orc.maxwell(op, 0.86 * tc)
    assert abs(p.rho_g / g - 1) < 1e-10 and abs(p.rho_l / l - 1) < 1e-10
    assert p.rho_v == p.rho_g and p.rho_ref == p.rho_v
    assert abs(p.T_0 - 0.86 * tc) < 1e-15 and abs(p.T_w - 0.80 * tc) < 1e-15


@pytest.mark.parametrize("frac", [0.56, 0.65, 0.78, 0.9])
def test_library_coexistence_matches_oracle(L, orc, frac):
    p = lbm.lbm_params_resolve(lbm.lbm_params_default())
    g1, l1, p1 = lbm.lbm_eos_coexistence(p, frac * p.T_c)
    g2, l2, p2 = orc.maxwell(orc.default_params(), frac * p.T_c)
    assert abs(g1 / g2 - 1) < 1e-9 and abs(l1 / l2 - 1) < 1e-9 and abs(p1 / p2 - 1) < 1e-9


@pytest.mark.parametrize("bad", [dict(Nx=2), dict(Ny=3), dict(s_e=0.9), dict(s_q=2.0),
                                 dict(tau_g=0.5), dict(G=0.0), dict(precision=7),
                                 dict(flags=128), dict(flags=512), dict(flags=256 | 4),
                                 dict(flags=256 | 64), dict(flags=256, cold_x1=129),
                                 dict(flags=256, cold_x0=5, cold_x1=3),
                                 dict(flags=256, cold_x0=-1, cold_x1=3),
                                 dict(flags=256, T_w_end=0.05)])
def test_workspace_bytes_rejects_invalid(L, bad):
    p = lbm.lbm_params_default(**bad)
    assert lbm.lbm_workspace_bytes(p) == 0
    assert len(lbm.lib().lbm_last_error()) > 0


@pytest.mark.parametrize("prec,bytes_per_node", [(lbm.LBM_FP32_DEV, 80), (lbm.LBM_FP64, 160)])
def test_workspace_bytes_size_limit(L, prec, bytes_per_node):
    """The step reaches its buffers by 32-bit byte offsets: a 16384-wide
    channel is accepted while its step buffers (bytes_per_node per stored
    node) stay below 4 GiB and refused beyond, without allocating."""
    rows_max = (1 << 32) // (bytes_per_node * 16384)
    ok = lbm.lbm_params_default(Nx=16384, Ny=rows_max - 20 + 2, precision=prec)
    assert lbm.lbm_workspace_bytes(ok) > (rows_max - 20) * 16384 * bytes_per_node
    big = lbm.lbm_params_default(Nx=16384, Ny=rows_max + 1 + 2, precision=prec)
    assert lbm.lbm_workspace_bytes(big) == 0
    assert b"too large" in lbm.lib().lbm_last_error()


def test_workspace_bytes_layout(L):
    p = lbm.lbm_params_default(Nx=100, Ny=10)
    n32 = lbm.lbm_workspace_bytes(p)
    p.precision = lbm.LBM_FP64
    n64 = lbm.lbm_workspace_bytes(p)
    p.precision = lbm.LBM_FP32_DEV_MASSEXACT
    nmx = lbm.lbm_workspace_bytes(p)
    pitch, rows = 128, 8
    pops = 2 * 9 * pitch * rows
    assert n64 - n32 >= 4 * (pops + 2 * pitch * rows) - 256 * 8
    assert nmx - n32 >= 2 * 4 * pitch * rows


def test_eos_pressure_matches_oracle(L, orc):
    p = lbm.lbm_params_resolve(lbm.lbm_params_default())
    op = orc.default_params()
    for rho in (0.2, 0.38, 3.0, 6.5):
        P, ps = lbm.lbm_eos_pressure(p, rho, p.T_0)
        assert abs(P - orc.peos(op, rho, p.T_0)) < 1e-14
        assert abs(ps - orc.psi(op, rho, p.T_0)) < 1e-13


def test_contact_angle_table_matches_golden():
    """configs.CONTACT_ANGLE_TABLE holds the oracle calibration of
    tests/golden/contact_angle_table.json, and the angle falls monotonically
    as the wall potential grows (more wetting)."""
    import json
    from paper_1803_01756_amd import configs
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "contact_angle_table.json")))
    g = {round(r["frac"], 4): r["angle"] for r in gold["table"] if r["angle"] < 180.0}
    for f, a in configs.CONTACT_ANGLE_TABLE:
        assert abs(g[round(f, 4)] - a) < 1e-6
    angles = [a for _, a in sorted(configs.CONTACT_ANGLE_TABLE)]
    assert all(x > y for x, y in zip(angles, angles[1:]))
    assert abs(configs.wall_fraction_for_angle(90.13) - 0.45) < 1e-9


@pytest.mark.parametrize("frac", [0.56, 0.65, 0.86, 0.95])
def test_latent_heat_matches_oracle(orc, frac):
    """The library's Eq. 19 (written with the log of the free-energy term)
    against the oracle's (the printed log ratio), and Eq. 20."""
    p = lbm.lbm_params_resolve(lbm.lbm_params_default())
    q = orc.default_params()
    T = frac * p.T_c
    h = lbm.lbm_eos_latent_heat(p, T)
    assert h == pytest.approx(orc.latent_heat(q, T), rel=1e-9)
    assert lbm.jacob_number(p, T, 0.5 * p.T_c) == pytest.approx(
        orc.jacob(q, T, 0.5 * p.T_c), rel=1e-9)


def test_latent_heat_rejects_supercritical():
    p = lbm.lbm_params_resolve(lbm.lbm_params_default())
    with pytest.raises(lbm.LBMError):
        lbm.lbm_eos_latent_heat(p, 1.01 * p.T_c)


def test_cs_eos_matches_oracle(orc):
    """Carnahan-Starling option: critical point, coexistence and latent heat
    from the library's host EOS against the oracle's."""
    rc, tc = lbm.lbm_eos_critical_cs()
    orc_rc, orc_tc = orc.critical_cs()
    assert tc == pytest.approx(orc_tc, rel=1e-12)
    assert rc == pytest.approx(orc_rc, rel=1e-6)  # flat maximum: T_c is sharp, rho_c is not
    p = configs.channel_params_cs(32, 8)
    q = orc.default_params_cs()
    for frac in (0.6, 0.86, 0.95):
        T = frac * tc
        g, l, ps = lbm.lbm_eos_coexistence(p, T)
        og, ol, ops = orc.maxwell(q, T)
        assert g == pytest.approx(og, rel=1e-9) and l == pytest.approx(ol, rel=1e-10)
        assert lbm.lbm_eos_latent_heat(p, T) == pytest.approx(orc.latent_heat(q, T), rel=1e-9)
    for rho in (0.02, 0.13, 0.3):
        P, psi = lbm.lbm_eos_pressure(p, rho, 0.8 * tc)
        assert P == pytest.approx(orc.peos(q, rho, 0.8 * tc), rel=1e-13)


def test_null_handles_are_refused_without_a_device(L):
    """Every entry point that takes a simulation or pool handle refuses a
    null one with LBM_EINVAL (destroy accepts it) before touching the GPU;
    this runs on a machine without one."""
    import ctypes as C
    f = lbm.lib()
    d = C.c_double()
    i32 = C.c_int32()
    EINVAL = lbm.LBM_EINVAL
    assert f.lbm_step(None, 1) == EINVAL
    assert f.lbm_moments(None, None, None, None, None) == EINVAL
    assert f.lbm_reduce(None, C.byref(d)) == EINVAL
    assert f.lbm_synchronize(None) == EINVAL
    assert f.lbm_destroy(None) == lbm.LBM_OK
    assert f.lbm_time(None) == -1
    assert f.lbm_get_params(None, C.byref(lbm.lbm_params())) == EINVAL
    assert f.lbm_state_bytes(None) == 0
    assert f.lbm_save(None, None, 0) == EINVAL
    assert f.lbm_load(None, None, 0) == EINVAL
    assert f.lbm_set_launch(None, 26) == EINVAL
    assert f.lbm_get_launch(None, C.byref(i32), C.byref(i32)) == EINVAL
    assert f.lbm_autotune(None, 3, C.byref(d)) == EINVAL
    assert f.lbm_pool_admit(None, C.byref(lbm.lbm_params_default()), None, 10, C.byref(i32)) == EINVAL
    assert f.lbm_pool_run(None, 10) == EINVAL
    assert f.lbm_pool_wait(None, 0) == EINVAL
    assert f.lbm_pool_poll(None, None, 0, C.byref(i32)) == EINVAL
    assert f.lbm_pool_moments(None, 0, None, None, None, None) == EINVAL
    assert f.lbm_pool_release(None, 0) == EINVAL
    assert f.lbm_pool_destroy(None) == lbm.LBM_OK
    assert f.lbm_pool_info(None, None, None, None) == EINVAL
    assert f.lbm_pool_slot_time(None, 0) == -1
    assert f.lbm_pool_set_launch(None, 26) == EINVAL
    assert f.lbm_pool_synchronize(None) == EINVAL
    assert f.lbm_pool_create(0, None, None) == EINVAL
    assert f.lbm_health(None, None, None) == EINVAL
    assert f.lbm_pool_slot_health(None, 0, None, None) == EINVAL
    assert len(f.lbm_last_error()) > 0


def test_jacob_number_matches_oracle(L, orc):
    """Eq. 20 computed by the library (lbm_eos_jacob) against the oracle's."""
    p = lbm.lbm_params_resolve(lbm.lbm_params_default())
    q = orc.default_params()
    for ts, tw in ((0.86, 0.80), (0.86, 0.56), (0.7, 0.65)):
        ja = lbm.lbm_eos_jacob(p, ts * p.T_c, tw * p.T_c)
        assert ja == pytest.approx(orc.jacob(q, ts * p.T_c, tw * p.T_c), rel=1e-9)
    with pytest.raises(lbm.LBMError):
        lbm.lbm_eos_jacob(p, 1.01 * p.T_c, 0.8 * p.T_c)


@pytest.mark.parametrize("where", ["fluid", "frame_t"])
def test_create_refuses_initial_density_without_real_psi(L, orc, where):
    """An initial density for which the Eq. 10 argument 2 (P - rho/3) / G is
    negative at the node's initial temperature (P - rho/3 > 0 with G < 0,
    first at rho = 8.97 at 0.86 T_c) is refused with LBM_EINVAL before any
    device call; a density just below the limit is not the reason for a
    refusal.  The limit is located with the oracle's EOS.  With FRAME_T the
    frame starts at T_w, so the limit there is the one at T_w."""
    import ctypes as C
    flags = lbm.LBM_FRAME_T if where == "frame_t" else 0
    p = configs.channel_params(16, 8, 90.0, 0.60, 0.0, 0.0, lbm.LBM_FP32_DEV, flags)
    q = orc.default_params()
    T = p.T_w if where == "frame_t" else p.T_0
    lo, hi = 5.0, 10.4
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if orc.peos(q, mid, T) - mid / 3.0 > 0:
            hi = mid
        else:
            lo = mid
    x = 0 if where == "frame_t" else 7
    for rho, expect_refusal in ((hi * (1 + 1e-6), True), (lo * (1 - 1e-6), False)):
        r0 = np.full((8, 16), p.rho_v)
        r0[3, x] = rho
        h = C.c_void_p()
        st = L.lbm_create(C.byref(p), r0.ctypes.data_as(C.POINTER(C.c_double)), None, 0, None,
                          C.byref(h))
        msg = L.lbm_last_error().decode()
        if expect_refusal:
            assert st == lbm.LBM_EINVAL and "Eq. 10" in msg, msg
            assert h.value is None
        else:
            # on this machine the call then fails at the device (or succeeds
            # on a GPU machine); either way not for the density
            assert "Eq. 10" not in msg
            if st == lbm.LBM_OK:
                L.lbm_destroy(h)

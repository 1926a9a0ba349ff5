"""The allocation-free reduction (lbm_reduce_noalloc) through the C-ABI
against lbm_reduce on the same state: two calls in a row, the second on a
smaller channel, so the shared file-scope scratch holds the first call's
partials when the second starts.

Tolerance: both sum the same FP64 node values (the read-out's per-node
arithmetic is shared) in different orders, so the totals agree to FP64
rounding of the sums: 1e-12 relative on sum rho and sum rho C_v T, 1e-12 of
sum |rho u| on the momenta; the non-finite count exactly.
"""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1803_01756_amd import configs, lbm

pytestmark = pytest.mark.gpu


def _check_against_reduce(p, seed, steps):
    s = lbm.Sim(p, configs.initial_density(p, seed=seed))
    s.step(steps)
    out = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    st = lbm.lib().lbm_reduce_noalloc(C.c_void_p(s.h), C.c_void_p(out.data_ptr()))
    assert st == lbm.LBM_OK, lbm.lib().lbm_last_error()
    s.synchronize()
    got = out.cpu().numpy()
    ref = s.reduce()
    rho, ux, uy, _ = s.moments()
    s.close()
    jscale = np.abs(rho * np.hypot(ux, uy)).sum()
    print(dict(Nx=p.Nx, Ny=p.Ny, got=got.tolist(), ref=ref.tolist()), flush=True)
    assert abs(got[0] - ref[0]) <= 1e-12 * ref[0]
    assert abs(got[1] - ref[1]) <= 1e-12 * jscale
    assert abs(got[2] - ref[2]) <= 1e-12 * jscale
    assert abs(got[3] - ref[3]) <= 1e-12 * ref[3]
    assert got[4] == ref[4] == 0


def test_reduce_noalloc_matches_reduce_two_calls():
    print("\n[case] lbm_reduce_noalloc: 2048x256 fp32 then 130x40 fp64", flush=True)
    _check_against_reduce(configs.single_gpu_channel(60.0), 3, 200)
    _check_against_reduce(configs.channel_params(130, 40, 120.0, 0.78, 2e-4, 300.0,
                                                 lbm.LBM_FP64), 5, 150)


@pytest.mark.parametrize("flags", [lbm.LBM_PERIODIC_Y, lbm.LBM_OPEN_X,
                                   lbm.LBM_FRAME_T | lbm.LBM_FRAME_RHO | lbm.LBM_PERIODIC_Y])
def test_reduce_noalloc_boundary_variants(flags):
    """The tile ring follows the read-out's neighbours: periodic y, open ends
    (the end column stands for the missing neighbour) and reservoir frames."""
    print("\n[case] lbm_reduce_noalloc flags=%d" % flags, flush=True)
    if flags & lbm.LBM_OPEN_X:
        p = configs.open_channel(131, 24, p_period=300.0, precision=lbm.LBM_FP32_DEV)
    else:
        extra = dict(rho_frame=0.3) if flags & lbm.LBM_FRAME_RHO else {}
        p = configs.channel_params(70, 21, 120.0, 0.8, 1e-4, 100.0, lbm.LBM_FP32_DEV_MASSEXACT,
                                   flags, **extra)
    _check_against_reduce(p, 7, 60)

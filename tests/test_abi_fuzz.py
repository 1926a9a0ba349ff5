"""Random parameter sets through the host-only entry points of the C-ABI
(CPU, no device): lbm_params_resolve, lbm_workspace_bytes,
lbm_pool_footprint, the EOS helpers and lbm_create's checks.  Every field
is drawn from a mix of ordinary values, zero, negative, huge, infinite and
NaN values; each call must return a status or a size (never crash), a
refused set must leave a message, and an accepted set must describe a grid
whose step buffers fit the 32-bit offsets."""
import ctypes as C
import math

import numpy as np
import pytest

from paper_1803_01756_amd import lbm

SPECIAL = [0.0, -1.0, 1e300, -1e300, math.inf, -math.inf, math.nan, 1e-300]


def _draw(rng, base):
    p = lbm.lbm_params.from_buffer_copy(base)
    for name, ctype in lbm.lbm_params._fields_:
        if rng.random() > 0.15:
            continue
        if ctype is C.c_double:
            v = SPECIAL[rng.integers(len(SPECIAL))] if rng.random() < 0.5 else \
                getattr(base, name) * rng.uniform(-2.0, 3.0)
            setattr(p, name, v)
        elif ctype is C.c_int32:
            setattr(p, name, int(rng.choice([0, -1, 1, 2, 3, 4, 5, 1 << 20, -(1 << 31), (1 << 31) - 1,
                                              int(rng.integers(0, 4096))])))
        elif ctype is C.c_uint32:
            setattr(p, name, int(rng.integers(0, 1 << 10)))
    return p


@pytest.mark.parametrize("seed", range(4))
def test_random_parameters_never_crash(seed):
    L = lbm.lib()
    rng = np.random.default_rng(seed)
    base = lbm.lbm_params_resolve(lbm.lbm_params_default(Nx=96, Ny=24))
    accepted = 0
    for _ in range(400):
        p = _draw(rng, base)
        q = lbm.lbm_params.from_buffer_copy(p)
        L.lbm_params_resolve(C.byref(q))
        ws = int(L.lbm_workspace_bytes(C.byref(p)))
        fp = int(L.lbm_pool_footprint(C.byref(p)))
        if ws == 0:
            assert len(L.lbm_last_error()) > 0
        else:
            accepted += 1
            assert 0 < ws < (1 << 33) and fp > 0
            assert p.Nx >= 3 and p.Ny >= 3
        g, l, ps = C.c_double(), C.c_double(), C.c_double()
        L.lbm_eos_coexistence(C.byref(p), base.T_0, C.byref(g), C.byref(l), C.byref(ps))
        L.lbm_eos_latent_heat(C.byref(p), base.T_0, C.byref(g))
        if 3 <= p.Nx <= 4096 and 3 <= p.Ny <= 4096:
            h = C.c_void_p()
            st = L.lbm_create(C.byref(p), None, None, C.c_size_t(0), None, C.byref(h))
            assert st != lbm.LBM_OK and not h.value  # no device here, or refused
    assert accepted > 0

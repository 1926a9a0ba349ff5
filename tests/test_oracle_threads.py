"""The OpenMP-over-rows build of the oracle (used to time it on all host
cores) gives bitwise the results of the sequential build: every sweep
writes each node from the previous fields only, and the one cross-node sum
(the psi clamp count) is an integer.  Checked on the channel, the open
channel and a case with psi clamps, with several threads."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_SCRIPT = r"""
import sys, numpy as np
sys.path.insert(0, %r); sys.path.insert(0, %r)
from helpers import to_oracle
from oracle import oracle as O
from paper_1803_01756_amd import configs, inputs, lbm
cases = []
p = configs.oracle_size_channel(lbm.LBM_FP64)
cases.append((p, configs.initial_density(p, seed=1), 60))
p = configs.open_channel(131, 24, p_period=300.0, precision=lbm.LBM_FP64)
cases.append((p, configs.initial_density(p, seed=21), 40))
p = configs.channel_params(64, 24, 90.0, 0.8, 2e-5, 200.0, lbm.LBM_FP64, 0)
p.T_0, p.T_w, p.rho_v, p.rho_ref = 1.15 * p.T_c, 1.6 * p.T_c, 7.8, 7.8
cases.append((p, inputs.density_field(64, 24, 7.8, 0.01, 3), 24))
assert O.threads(True) == 4, O.threads(True)
for p, r0, n in cases:
    a = O.Sim(to_oracle(O, p), r0)
    b = O.Sim(to_oracle(O, p), r0, omp=True)
    a.step(n); b.step(n)
    for x, y in zip(a.moments(), b.moments()):
        assert np.array_equal(x, y)
    assert np.array_equal(a.get_f(), b.get_f())
    assert a.psi_clamps == b.psi_clamps
print("OK", cases[-1][2], a.psi_clamps)
"""


def test_openmp_build_is_bitwise_sequential(orc):
    orc.build(omp=True)
    env = dict(os.environ, OMP_NUM_THREADS="4")
    out = subprocess.run([sys.executable, "-c", _SCRIPT % (ROOT, os.path.join(ROOT, "tests"))],
                         env=env, capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    ok, _, clamps = out.stdout.split()
    assert ok == "OK" and int(clamps) > 1000

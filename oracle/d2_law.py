"""Droplet evaporation (Sec. 3.1, the D^2 law) with the FP64 oracle.

TEST INFRASTRUCTURE: runs only the oracle.  Writes
tests/golden/d2_law_<N>.json: the equivalent diameter D(t) of a droplet in an
N x N periodic box whose frame is an open reservoir at T_c and at the
saturation pressure of T_sat = 0.86 T_c (flags FRAME_T | FRAME_RHO), fluid
initially at T_sat, for lambda = 1/3 and 2/3, and the slope K of
(D/D0)^2 = a - K t fitted where 0.2 < (D/D0)^2 < 0.8 (the first samples carry
the start-up transient of the interface and of the heat front).

D is the diameter of the disc holding the same liquid: the liquid fraction
(rho - rho_g)/(rho_l - rho_g), clipped to [0, 1], summed over the box.

    python oracle/d2_law.py N D steps every      (e.g. 100 30 60000 1000)
"""
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)


def run(args):
    lam, N, D, steps, every = args
    from oracle import oracle as O
    from paper_1803_01756_amd import inputs
    tc = O.critical()[1]
    p = O.default_params(Nx=N, Ny=N, g_osc=0.0, period=0.0, lam=lam, Tw=tc,
                         flags=O.PERIODIC_Y | O.FRAME_T | O.FRAME_RHO)
    # reservoir density: P_EOS(rho, T_c) = P_EOS(rho_g, T_sat), vapour side
    p_sat = O.peos(p, p.rho_g, p.T0)
    lo, hi = 1e-6, p.rho_g
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if O.peos(p, mid, p.Tw) < p_sat else (lo, mid)
    p.rho_frame = 0.5 * (lo + hi)
    rho0 = inputs.droplet_disc(N, N, D, p.rho_l, p.rho_g)
    s = O.Sim(p, rho0)

    def diam(rho):
        frac = np.clip((rho - p.rho_g) / (p.rho_l - p.rho_g), 0.0, 1.0)
        return float(np.sqrt(4.0 * frac.sum() / np.pi))

    t, d = [0], [diam(s.moments()[0])]
    while s.n < steps:
        s.step(every)
        t.append(int(s.n))
        d.append(diam(s.moments()[0]))
        print("lambda %.4f n %d D %.4f" % (lam, s.n, d[-1]), flush=True)
        if d[-1] < 0.3 * d[0]:
            break
    t_a, d2 = np.array(t, float), (np.array(d) / d[0]) ** 2
    sel = (d2 > 0.2) & (d2 < 0.8)
    if sel.sum() < 3:
        return dict(lam=lam, t=t, D=d, K=None, R2=None, fit_points=int(sel.sum()),
                    rho_frame=p.rho_frame)
    A = np.column_stack([np.ones(sel.sum()), -t_a[sel]])
    coef, *_ = np.linalg.lstsq(A, d2[sel], rcond=None)
    res = d2[sel] - A @ coef
    r2 = 1 - float(res @ res) / float(((d2[sel] - d2[sel].mean()) ** 2).sum())
    return dict(lam=lam, t=t, D=d, K=float(coef[1]), R2=r2, fit_points=int(sel.sum()),
                rho_frame=p.rho_frame)


def main():
    N, D, steps, every = int(sys.argv[1]), float(sys.argv[2]), int(sys.argv[3]), int(sys.argv[4])
    with ProcessPoolExecutor(max_workers=2) as ex:
        cases = list(ex.map(run, [(1.0 / 3.0, N, D, steps, every), (2.0 / 3.0, N, D, steps, every)]))
    out = dict(source="oracle/d2_law.py (FP64 oracle only)", N=N, D=D, every=every,
               recipe=__doc__.split("\n\n")[1].replace("\n", " "), cases=cases)
    path = os.path.join(ROOT, "tests", "golden", "d2_law_%d.json" % N)
    json.dump(out, open(path, "w"), indent=1)
    print("wrote", path, [(c["lam"], c["K"], c["R2"]) for c in cases])


if __name__ == "__main__":
    main()

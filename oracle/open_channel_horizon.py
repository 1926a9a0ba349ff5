"""How far the Sec. 3.3 channel runs before it diverges, from the FP64 oracle.

TEST INFRASTRUCTURE: runs only the oracle (its OpenMP build).  Writes
tests/golden/open_channel_horizon_1600x48.json, the record behind the
statements about the channel's divergence and its two remedies.

Set-up (the case as the paper describes it, with the readings for what it
leaves out): 1600 x 48, Zou-He ends, inlet pressure p0 (1 + 0.1 sin(2 pi n /
2000)) against a constant p0 at the outlet (p0 the saturation pressure at
T_in = T_0 = 0.86 T_c), plates linear from 0.86 T_c to 0.56 T_c, gravity
1e-4 along +x, plates at the wall density fraction of 137.82 degrees, vapour
with +-1 % noise (seed 1).  Four variants: the outlet temperature evolving
(zero-gradient) or held at T_sat (T_out), each with and without the
diffusivity cap alpha_max = 0.25.  Every 250 steps up to `steps`: whether
the state is sound (every fluid density finite and positive), the least
fluid density, and how many fluid nodes have lambda / (rho C_v) above the
RK4 bound 0.522; a variant stops at its first unsound sample.

    python oracle/open_channel_horizon.py [steps]     (default 14000)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

NX, NY, SEED, ANGLE, EVERY = 1600, 48, 1, 137.82, 250


def params(O, held_outlet, alpha_max):
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "contact_angle_table.json")))
    tab = sorted((r["angle"], r["frac"]) for r in gold["table"] if r["angle"] < 180.0)
    frac = float(np.interp(ANGLE, [a for a, _ in tab], [f for _, f in tab]))
    tc = O.critical()[1]
    p = O.default_params(Nx=NX, Ny=NY, Tw=0.86 * tc, g_osc=0.0, period=0.0, gx=1e-4,
                         flags=O.OPEN_X)
    p.Tw_end = 0.56 * tc
    p.T_in = p.T0
    p.T_out = p.T0 if held_outlet else 0.0
    p.p_amp, p.p_period = 0.1, 2000.0
    p.alpha_max = alpha_max
    p.Gw = p.G
    p.psiw = O.psi(p, p.rho_g + frac * (p.rho_l - p.rho_g), p.T0)
    return p


def run(O, held_outlet, alpha_max, steps):
    from paper_1803_01756_amd import inputs
    p = params(O, held_outlet, alpha_max)
    s = O.Sim(p, inputs.density_field(NX, NY, p.rho_v, 0.01, SEED), omp=True)
    hist = []
    t0 = time.time()
    while s.n < steps:
        s.step(EVERY)
        rho = s.moments()[0][1:-1]
        fin = bool(np.isfinite(rho).all() and rho.min() > 0.0)
        rec = dict(step=int(s.n), sound=fin)
        if fin:
            rec["min_rho"] = float(rho.min())
            rec["nodes_above_rk4_bound"] = int((p.lam / (rho * p.Cv) > 0.522).sum())
        hist.append(rec)
        print(held_outlet, alpha_max, json.dumps(rec), "%.0f s" % (time.time() - t0), flush=True)
        if not fin:
            break
    last = max([r["step"] for r in hist if r["sound"]], default=0)
    return dict(outlet="held at T_sat" if held_outlet else "evolving", alpha_max=alpha_max,
                sound_through=last, diverged=not hist[-1]["sound"], history=hist)


def main():
    from oracle import oracle as O
    steps = int(sys.argv[1]) if len(sys.argv) > 1 else 14000
    out = dict(source="oracle/open_channel_horizon.py (FP64 oracle only)", Nx=NX, Ny=NY,
               seed=SEED, contact_angle=ANGLE, sample_every=EVERY, steps=steps,
               variants=[run(O, h, a, steps) for h in (False, True) for a in (0.0, 0.25)])
    path = os.path.join(ROOT, "tests", "golden", "open_channel_horizon_%dx%d.json" % (NX, NY))
    json.dump(out, open(path, "w"), indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()

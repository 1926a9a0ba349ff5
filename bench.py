#!/usr/bin/env python3
"""Throughput of the fused FP32 pseudopotential MRT-LBM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the 8192 x 512 plate channel (4.18 M fluid nodes), FP32 deviation
storage, cold plates at 0.78 Tc with a 75 degree wall, drive amplitude 2e-6
and period 4000 steps, saturated vapour with +-1 % seeded noise.  It is the
HBM-bound configuration: its 2 x 36 B populations + 2 x 4 B temperature per
node (352 MB) exceed the 256 MB Infinity Cache.  One step = one launch of the
fused kernel over the whole channel.  Inputs are resident in HBM before the
timed region starts.  After tuning the launch shape the channel runs 0.1 s of
untimed steps, then the W warm-up steps, then the K timed steps.

Prints one JSON line.  `value` is MLUPS (million fluid-node updates per
second).  `roofline` compares the algorithmic bytes of one launch (80 B per
node: 9 FP32 populations read and written, T read and written) per average
launch time with the 8 TB/s HBM peak; `traffic` is the HBM traffic the
rocprofv3 FETCH_SIZE / WRITE_SIZE counters measured for the same kernel
(committed under profiles/), scaled by what those counters read for a plain
copy of known size, or null when the kernel source changed since.
`cpu_baseline` times the FP64 CPU oracle on a bounded sample of the same
workload on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_LUP = {0: 80.0, 1: 160.0, 2: 88.0}  # FP32_DEV, FP64, FP32_DEV_MASSEXACT
# headline storage: name -> (lbm precision code, dtype label, description, profile tag)
PRECISIONS = {"fp32": (0, "f32", "FP32 deviation storage", "fp32"),
              "fp64": (1, "f64", "FP64 storage", "fp64"),
              "fp32-massexact": (2, "f32", "mass-exact FP32 deviation storage", "fp32_massexact")}


def pmc_file(tag):
    return os.path.join(ROOT, "profiles", "pmc_step_8192x512_%s.json" % tag)
# the sources that decide what a step launch reads and writes: the kernels and
# the device layout (plane stride, pitch, buffer offsets)
TRAFFIC_SRCS = [os.path.join(ROOT, "paper_1803_01756_amd", "csrc", f)
                for f in ("lbm_kernels.hip", "lbm_runtime.cpp", "lbm_host.h")]


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def host_info():
    """Logical CPUs and CPU model of the host the CPU baseline ran on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(nproc=os.cpu_count(), model=model)


def kernel_sha():
    """sha256 over the kernel and layout sources, in order; a counter summary
    taken from other sources is not used."""
    h = hashlib.sha256()
    for path in TRAFFIC_SRCS:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(tag="fp32"):
    """HBM bytes per launch from the committed counter summary of this
    storage, or None (no summary, or one taken from other kernel source)."""
    path = pmc_file(tag)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_sha256") != kernel_sha():
        return None
    fetch = d["fetch_kib_per_dispatch"] * 1024.0 / d["copy_fetch_factor"]
    write = d["write_kib_per_dispatch"] * 1024.0 / d["copy_write_factor"]
    return fetch + write


# Untimed steps run after the launch-shape tuning and before the W warm-up
# steps, in wall-clock seconds.  The GPU reaches its sustained clock state
# only after some tens of milliseconds of continuous work: a short timed
# region straight after host-side setup (the autotune, whose trials are
# timed one by one) or after an idle pause measures that transient instead
# (20 timed steps of the 8192 x 512 channel: 98-106 us each there, 95-96 us
# after 0.1 s of sustained steps, 93 us over 2000 steps).
PREHEAT_S = 0.1


def preheat(sim, seconds=PREHEAT_S):
    """Run untimed steps for about `seconds` of wall time, enqueued back to
    back after a first 20 that size them; returns how many."""
    t0 = time.perf_counter()
    sim.step(20)
    sim.synchronize()
    per = max(time.perf_counter() - t0, 1e-6) / 20
    n = int(max(0.0, seconds - (time.perf_counter() - t0)) / per)
    sim.step(n)
    sim.synchronize()
    return 20 + n


def time_steps(sim, steps, warmup):
    import torch
    sim.step(warmup)
    sim.synchronize()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    sim.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1), wall * 1e3


def fluid_nodes(p):
    return p.Nx * (p.Ny if (p.flags & 4) else p.Ny - 2)


def run_config(p, rho0, steps, warmup, tune=True, seg_rows=0):
    from paper_1803_01756_amd import lbm
    sim = lbm.Sim(p, rho0, torch_memory=True)
    if seg_rows > 0:
        sim.set_launch(seg_rows)
    elif tune:
        sim.autotune(10)
    preheat(sim)
    ms, wall_ms = time_steps(sim, steps, warmup)
    seg, waves = sim.launch()
    red = sim.reduce(check=False)
    sim.close()
    return ms, wall_ms, seg, waves, red


def oracle_mlups(p, rho0, steps, omp=False):
    """FP64 oracle on the full grid for `steps`: the sequential build, or
    with omp the OpenMP-over-rows build on OMP_NUM_THREADS threads (bitwise
    the same results).  Returns (MLUPS, seconds, threads)."""
    from oracle import oracle as O
    names = dict(T_c="Tc", G_w="Gw", psi_w="psiw", C_v="Cv", lambda_="lam", T_0="T0",
                 T_w="Tw", g_x="gx", g_y="gy")
    op = O.make_params(**{names.get(k, k): v for k, v in p.as_dict().items()
                          if k not in ("rho_ref", "precision")})
    sim = O.Sim(op, rho0, omp=omp)
    sim.step(1)  # first-touch of the scratch fields outside the timing
    t0 = time.perf_counter()
    sim.step(steps)
    dt = time.perf_counter() - t0
    return fluid_nodes(p) * steps / dt / 1e6, dt, O.threads(omp)


def batch_and_serve(args):
    """64 channels of uneven size in one pool (launch policy autotuned, and
    the default heuristic for reference) against the same channels run one
    after another alone, each at its own autotuned shape; then a Poisson
    stream of requests served with continuous batching (warm-up requests
    first, the launch policy tuned on the live mix once they are admitted),
    under a cap that never binds and again under one (256 MiB) that makes
    requests wait for admission.  A seeded 10 % sample of the measured
    requests is rerun alone at its full step count and compared bitwise."""
    import numpy as np
    from paper_1803_01756_amd import inputs, lbm, serve
    chans = [serve.channel_request(d, args.batch_steps)
             for d in inputs.sample_channels(64, seed=1803)]
    lups = sum(serve.lup(p, args.batch_steps) for p, _ in chans)
    log("batched: 64 channels x %d steps (%.2e node updates), pool autotuned"
        % (args.batch_steps, lups))
    info = {}
    tb, _ = serve.run_batch(chans, args.batch_steps, chunk=1000, tune_steps=10, info=info)
    log("batched %.3f s (tuned %.3f ms/step); default launch policy next" % (tb, info["tuned_ms_per_step"]))
    tb0, _ = serve.run_batch(chans, args.batch_steps, chunk=1000)
    log("default policy %.3f s; now the same channels one after another, each autotuned" % tb0)
    alone_shapes = []
    ta, _ = serve.run_alone(chans, args.batch_steps, tune_steps=3, shapes=alone_shapes)
    seg = [sr for sr, _ in info["shapes"]]
    batched = dict(channels=64, steps=args.batch_steps, node_updates=lups,
                   seconds=round(tb, 4), mlups=round(lups / tb / 1e6, 1),
                   hbm_gbs_algorithmic=round(lups / tb * BYTES_PER_LUP[lbm.LBM_FP32_DEV] / 1e9, 1),
                   roofline_frac=round(lups / tb * BYTES_PER_LUP[lbm.LBM_FP32_DEV] / 1e9
                                       / HBM_PEAK_GBS, 4),
                   sims_per_s=round(64 / tb, 3),
                   launch="lbm_pool_autotune (per bucket of fluid rows)",
                   tuned_ms_per_step=round(info["tuned_ms_per_step"], 4),
                   waves_per_step=sum(w for _, w in info["shapes"]),
                   seg_rows_min_median_max=[min(seg), int(np.median(seg)), max(seg)],
                   default_policy_seconds=round(tb0, 4),
                   default_policy_mlups=round(lups / tb0 / 1e6, 1),
                   alone_seconds=round(ta, 4), alone_mlups=round(lups / ta / 1e6, 1),
                   alone_launch="lbm_autotune per channel",
                   speedup_vs_alone=round(ta / tb, 3))
    log("batched: %s" % batched)

    n_warm, n_meas = args.serve_warmup, args.serve_requests
    rng = np.random.default_rng(1803)
    sample = set((n_warm + rng.choice(n_meas, max(1, n_meas // 10), replace=False)).tolist())

    def keep_sampled(r):
        if r.rid not in sample:
            r.result = None

    def stream(cap, rate=None, warm=None, nmeas=None):
        rate = args.serve_rate if rate is None else rate
        warm = n_warm if warm is None else warm
        nmeas = n_meas if nmeas is None else nmeas
        reqs = serve.make_requests(warm + nmeas, rate)
        pool = lbm.Pool(cap)
        serve.serve(reqs, pool, chunk=500, on_done=keep_sampled, tune_after=warm)
        pool.close()
        meas = reqs[warm:]
        st = serve.latency_stats(meas)
        lat = np.array([r.finished - r.arrival for r in meas])
        wait = np.array([r.admitted - r.arrival for r in meas])
        lu = sum(serve.lup(r.params, r.steps) for r in meas)
        arr_span = meas[-1].arrival - meas[0].arrival
        fifths = [round(float(np.percentile(c, 50)), 3) for c in np.array_split(lat, 5)]
        out = dict(p50_latency_s=round(st["p50_s"], 4), p99_latency_s=round(st["p99_s"], 4),
                   mean_latency_s=round(st["mean_s"], 4),
                   p50_latency_by_arrival_fifth_s=fifths,
                   admission_wait_s=dict(mean=round(float(wait.mean()), 4),
                                         p50=round(float(np.percentile(wait, 50)), 4),
                                         p99=round(float(np.percentile(wait, 99)), 4),
                                         max=round(float(wait.max()), 4)),
                   sims_per_s=round(st["sims_per_s"], 3),
                   mlups=round(lu / st["span_s"] / 1e6, 1),
                   offered_mlups=round(lu / arr_span / 1e6, 1),
                   errors=sum(1 for r in reqs if r.error))
        return reqs, out

    log("served: %d requests at %.0f/s (first %d are warm-up), cap 200 GB"
        % (n_warm + n_meas, args.serve_rate, n_warm))
    reqs, out = stream(200 << 30)
    served = dict(requests=n_meas, warmup_requests=n_warm, rate_per_s=args.serve_rate,
                  cap_bytes=200 << 30, chunk_steps=500, tuned_after_admissions=n_warm, **out)
    log("served: %s" % out)
    # the sampled results against the same requests run alone
    same = 0
    checked = sorted(sample)
    for rid in checked:
        r = reqs[rid]
        s = lbm.Sim(r.params, r.rho0)
        s.step(r.steps)
        ref = s.moments()
        s.close()
        same += int(r.result is not None and all(np.array_equal(a, b) for a, b in zip(r.result, ref)))
    served["checked_alone"] = dict(sampled=len(checked), bitwise_equal=same,
                                   sample="seeded 10 % of the measured requests (numpy "
                                          "default_rng(1803)), each rerun alone for its full "
                                          "step count")
    log("served: %d of %d sampled results bitwise equal to their runs alone" % (same, len(checked)))
    cap = 256 << 20
    log("served again under a %d MiB cap" % (cap >> 20))
    _, out = stream(cap)
    served["capped"] = dict(cap_bytes=cap, **out)
    log("capped: %s" % served["capped"])
    # below capacity: the offered load at the specified rate is just above
    # what the pool sustains, so the latency there keeps creeping up; at a
    # lower rate it is stationary
    rate2 = args.serve_rate_steady
    log("served below capacity: %d requests at %.0f/s (first %d are warm-up)"
        % (args.serve_requests_steady + n_warm // 2, rate2, n_warm // 2))
    _, out = stream(200 << 30, rate=rate2, warm=n_warm // 2, nmeas=args.serve_requests_steady)
    served["below_capacity"] = dict(rate_per_s=rate2, requests=args.serve_requests_steady,
                                    warmup_requests=n_warm // 2, cap_bytes=200 << 30, **out)
    log("below capacity: %s" % served["below_capacity"])
    return batched, served


def precision_study():
    """2048x256 channels with contact angles 60/90/120 degrees (seeds 1-3),
    and a liquid-rich one (90 degrees, a liquid layer filling the lower 40 %
    of the channel, seed 4): FP32 deviation storage (and, for the liquid
    layer, mass-exact FP32) against the FP64 build on the GPU, per-field
    differences at steps 100, 1000 and 20000, and the throughput of both."""
    import torch
    from paper_1803_01756_amd import analysis, configs, inputs, lbm
    out = {}
    cases = [(1, 60.0, False, lbm.LBM_FP32_DEV), (2, 90.0, False, lbm.LBM_FP32_DEV),
             (3, 120.0, False, lbm.LBM_FP32_DEV), (4, 90.0, True, lbm.LBM_FP32_DEV),
             (4, 90.0, True, lbm.LBM_FP32_DEV_MASSEXACT)]
    for seed, ca, liquid, prec in cases:
        p32 = configs.single_gpu_channel(ca, prec)
        p64 = configs.single_gpu_channel(ca, lbm.LBM_FP64)
        if liquid:
            rho0 = inputs.layer_field(p32.Nx, p32.Ny, p32.rho_g, p32.rho_l, 0.4 * p32.Ny, 2.0,
                                      0.01, seed)
        else:
            rho0 = configs.initial_density(p32, seed=seed)
        a, b = lbm.Sim(p32, rho0), lbm.Sim(p64, rho0)
        a.autotune(5)
        b.autotune(5)
        n, errs, t32, t64 = 0, {}, 0.0, 0.0
        for target in (100, 1000, 20000):
            for s, which in ((a, 32), (b, 64)):
                s.synchronize()
                t0 = time.perf_counter()
                s.step(target - n)
                s.synchronize()
                if which == 32:
                    t32 += time.perf_counter() - t0
                else:
                    t64 += time.perf_counter() - t0
            n = target
            errs[str(target)] = {k: float("%.3e" % v) for k, v in
                                 analysis.field_differences(a.moments(), b.moments()).items()}
        fl = fluid_nodes(p32) * 20000
        name = "%g deg" % ca
        if liquid:
            name += ", liquid layer 40 %%, %s" % ("mass-exact" if prec == lbm.LBM_FP32_DEV_MASSEXACT
                                                 else "FP32 deviations")
        out[name] = dict(errors_fp32_vs_fp64=errs, fp32_mlups=round(fl / t32 / 1e6, 1),
                         fp64_mlups=round(fl / t64 / 1e6, 1))
        a.close()
        b.close()
        log("precision study %s: %s" % (name, errs))
    return out


def large_mass_run(steps=50000, every=1000):
    """8192x512, mass-exact FP32 storage: FP64 total mass every `every` steps
    (max relative drift) and the droplets on the plates at the end."""
    from paper_1803_01756_amd import analysis, configs, lbm
    p = configs.large_channel(lbm.LBM_FP32_DEV_MASSEXACT)
    rho0 = configs.initial_density(p, seed=1)
    s = lbm.Sim(p, rho0)
    s.autotune(5)
    m0 = s.reduce()[0]
    worst = 0.0
    s.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps // every):
        s.step(every)
        worst = max(worst, abs(s.reduce()[0] / m0 - 1.0))
    dt = time.perf_counter() - t0
    rho = s.moments()[0]
    drops = analysis.droplets(rho, 0.5 * (s.params.rho_l + s.params.rho_g))
    s.close()
    res = dict(steps=steps, max_rel_mass_drift=float("%.3e" % worst),
               mlups_incl_reductions=round(fluid_nodes(p) * steps / dt / 1e6, 1),
               droplets=drops)
    log("large run: %s" % res)
    return res


def d2_law_study(N=200, D=60.0, max_steps=320000, every=4000):
    """Sec. 3.1 droplet evaporation on the paper's 200 x 200 box (D = 60,
    frame reservoir at T_c, lambda = 1/3 and 2/3), FP32 deviations: the D^2
    slope K fitted where (D/D0)^2 falls from 0.8 to 0.2, its R^2, the ratio
    of the two slopes, and the oracle's slopes for the same set-up when its
    record (tests/golden/d2_law_200.json) is present."""
    import numpy as np
    from paper_1803_01756_amd import analysis, configs, lbm
    gold_path = os.path.join(ROOT, "tests", "golden", "d2_law_%d.json" % N)
    gold = json.load(open(gold_path)) if os.path.exists(gold_path) else None
    out = {}
    for lam in (1.0 / 3.0, 2.0 / 3.0):
        p = configs.d2_box(lam, lbm.LBM_FP32_DEV, N=N)
        s = lbm.Sim(p, configs.droplet_density(p, D))
        s.autotune(3)
        t, d = [0], [analysis.equivalent_diameter(s.moments()[0], p.rho_l, p.rho_g)]
        s.synchronize()
        t0 = time.perf_counter()
        while s.n < max_steps and d[-1] > 0.3 * d[0]:
            s.step(every)
            t.append(s.n)
            d.append(analysis.equivalent_diameter(s.moments()[0], p.rho_l, p.rho_g))
        dt = time.perf_counter() - t0
        n_done = s.n
        s.close()
        ta, d2 = np.array(t, float), (np.array(d) / d[0]) ** 2
        sel = (d2 > 0.2) & (d2 < 0.8)
        K, r2 = analysis.d2_fit(ta[sel], d2[sel]) if sel.sum() >= 3 else (None, None)
        rec = dict(K=K, R2=None if r2 is None else round(r2, 5), steps=int(n_done),
                   mlups_incl_readout=round(N * N * n_done / dt / 1e6, 1))
        if gold:
            ref = [c for c in gold["cases"] if abs(c["lam"] - lam) < 1e-12][0]
            rec["oracle_K"] = ref["K"]
            if K and ref["K"]:
                rec["K_rel_diff"] = float("%.3e" % (K / ref["K"] - 1))
        out["lambda=%.4f" % lam] = rec
        log("d2 law lambda %.4f: %s" % (lam, rec))
    ks = [v["K"] for v in out.values()]
    if all(ks):
        out["K_ratio_2_over_1"] = round(ks[1] / ks[0], 4)
    return out


def open_channel_run(steps=10500, every=500, alpha_max=0.25):
    """Sec. 3.3 on the paper's 1600 x 48 channel (Zou-He oscillating-pressure
    inlet, constant-pressure outlet open onto saturated vapour, plates
    0.86 -> 0.56 T_c, gravity +x, 137.82 degree plates), FP32, through the
    paper's 8500-10500 step window: throughput and, every `every` steps, the
    condensate (liquid nodes; liquid sets on the plates, and those whose
    centroid lies past x = 1500, the paper's exit region).  With the paper's
    energy equation the run diverges near step 10300 (held outlet); the
    diffusivity cap alpha_max (departure for thin vapour) keeps it finite
    past 13000 steps in the oracle."""
    import numpy as np
    from paper_1803_01756_amd import analysis, configs, lbm
    p = configs.open_channel(alpha_max=alpha_max)
    s = lbm.Sim(p, configs.initial_density(p, seed=1))
    s.autotune(3)
    out = dict(steps=steps, alpha_max=alpha_max, T_out_over_Tc=round(p.T_out / p.T_c, 4),
               paper="first droplets at the exit at ~8500 steps, more upstream by 9000, the two "
                     "nearest the exit merge and leave past X = 1550 by ~10500",
               samples=[])
    thr = 0.5 * (p.rho_l + p.rho_g)
    s.synchronize()
    dt_steps = 0.0
    while s.n < steps:
        t1 = time.perf_counter()
        s.step(min(every, steps - s.n))
        try:
            s.synchronize()
        except lbm.LBMError as e:  # non-finite state: report where it stopped
            out["diverged_by_step"] = int(s.n)
            log("open channel 1600x48 stopped: %s" % e)
            break
        dt_steps += time.perf_counter() - t1
        rho = s.moments()[0]
        sets = analysis.liquid_sets_open(rho, thr)
        on_plate = [r for r in sets if r[3] or r[4]]
        exit_sets = [r for r in on_plate if r[2] > 1500]
        out["samples"].append(dict(
            step=int(s.n), liquid_nodes=int((rho[1:-1] > thr).sum()),
            plate_sets=len(on_plate),
            exit_sets=[[r[0], round(r[2], 1), "top" if r[3] else "bottom"] for r in exit_sets],
            liquid_nodes_x_gt_1500=int((rho[1:-1, 1500:] > thr).sum()),
            min_rho=round(float(rho[1:-1].min()), 4)))
    out["mlups"] = round(fluid_nodes(p) * s.n / dt_steps / 1e6, 1)
    s.close()
    # the same run in FP64 storage: liquid nodes at the paper's marks, next
    # to the FP32 run's, to show the timeline does not hinge on the storage
    q = configs.open_channel(alpha_max=alpha_max, precision=lbm.LBM_FP64)
    s = lbm.Sim(q, configs.initial_density(q, seed=1))
    s.autotune(3)
    fp64 = []
    for mark in (2500, 5000, 8500, 10500):
        if mark > steps:
            break
        s.step(mark - s.n)
        try:
            rho = s.moments()[0]
        except lbm.LBMError:
            fp64.append(dict(step=mark, diverged=True))
            break
        fp64.append(dict(step=mark, liquid_nodes=int((rho[1:-1] > thr).sum()),
                         liquid_nodes_x_gt_1500=int((rho[1:-1, 1500:] > thr).sum())))
    s.close()
    out["fp64_check"] = fp64
    log("open channel 1600x48: %s" % out)
    return out


def open_channel_wettability(steps=10500, marks=(2500, 5000, 8500, 10500),
                             angles=(115.0, 145.0), alpha_max=0.25):
    """Sec. 3.3 wettability comparison (the paper's 115 and 145 degree
    plates) on the 1600 x 48 open channel, FP32, with the setting of
    open_channel_run: liquid nodes and the liquid sets on the plates (all,
    and past x = 1500) at the paper's 8500 and 10500 steps and earlier marks
    (the paper finds more condensate, in more closely spaced droplets, on the
    more wettable plate)."""
    import numpy as np
    from paper_1803_01756_amd import analysis, configs, lbm
    out = {}
    for ang in angles:
        p = configs.open_channel(contact_angle=ang, alpha_max=alpha_max)
        s = lbm.Sim(p, configs.initial_density(p, seed=1))
        s.autotune(3)
        thr = 0.5 * (p.rho_l + p.rho_g)
        rec = []
        for m in marks:
            if m > steps:
                break
            s.step(m - s.n)
            try:
                rho = s.moments()[0]
            except lbm.LBMError:
                rec.append(dict(step=m, diverged=True))
                break
            sets = [r for r in analysis.liquid_sets_open(rho, thr) if r[3] or r[4]]
            xs = sorted(r[2] for r in sets)
            rec.append(dict(step=m, liquid_nodes=int((rho[1:-1] > thr).sum()),
                            plate_sets=len(sets),
                            plate_sets_x_gt_1500=sum(1 for x in xs if x > 1500),
                            mean_spacing=round(float(np.mean(np.diff(xs))), 1) if len(xs) > 1
                            else None))
        s.close()
        out["%g deg" % ang] = rec
    log("open channel wettability: %s" % out)
    return out


def gravity_plate_run(steps=40000, every=2500):
    """Sec. 3.2 condensation under gravity on the paper's 100 x 300 box (cold
    middle third of the top plate at 0.65 T_c, adiabatic sides, bottom plate
    at T_sat, gravity 1e-4 toward it, 137.82 degree plates), FP32: throughput
    and, every `every` steps, the liquid and its largest connected set (node
    count, centroid height); the first sample at which that set's centroid
    has left the top tenth of the box (the droplet has come off the cold
    band), and the first at which it lies in the bottom tenth (landed)."""
    from paper_1803_01756_amd import analysis, configs, lbm
    p = configs.gravity_plate()
    s = lbm.Sim(p, configs.initial_density(p, seed=32))
    s.autotune(3)
    out = dict(steps=steps, samples=[], detached_at=None, landed_at=None, seg_rows=s.launch()[0])
    thr = 0.5 * (p.rho_l + p.rho_g)
    dt_steps = 0.0
    while s.n < steps:
        s.synchronize()
        t1 = time.perf_counter()
        s.step(every)
        s.synchronize()
        dt_steps += time.perf_counter() - t1
        sets = analysis.liquid_sets(s.moments()[0], thr)
        big = sets[0] if sets else [0, 0.0, 0.0, 0, 0]
        out["samples"].append(dict(step=int(s.n), liquid_nodes=int(sum(r[0] for r in sets)),
                                   largest=big[0], largest_y=round(big[1], 1)))
        if sets and out["detached_at"] is None and big[1] < 0.9 * p.Ny:
            out["detached_at"] = int(s.n)
        if sets and out["landed_at"] is None and big[1] < p.Ny / 10:
            out["landed_at"] = int(s.n)
    out["mlups"] = round(fluid_nodes(p) * steps / dt_steps / 1e6, 1)
    s.close()
    log("gravity plate 100x300: %s" % out)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--cpu-steps-omp", type=int, default=40,
                    help="oracle steps on the full grid for the all-threads CPU baseline")
    ap.add_argument("--cpu-steps", type=int, default=6,
                    help="oracle steps on the full grid for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the secondary precisions and the cache-resident size")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--seg-rows", type=int, default=0,
                    help="force the launch shape (rows per wave) instead of autotuning")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched and served runs")
    ap.add_argument("--batch-steps", type=int, default=10000)
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="measured requests of the served stream (after the warm-up ones)")
    ap.add_argument("--serve-warmup", type=int, default=100)
    ap.add_argument("--serve-rate-steady", type=float, default=16.0,
                    help="rate of the below-capacity served stream")
    ap.add_argument("--serve-requests-steady", type=int, default=500)
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--precision", choices=sorted(PRECISIONS), default="fp32",
                    help="storage of the headline 8192x512 run (default fp32)")
    args = ap.parse_args()
    prec, dtype, storage, tag = PRECISIONS[args.precision]

    if args.gpus != 1:
        print("bench.py measures one GPU only: the step runs on a single MI355X and this "
              "build has no multi-GPU path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1803_01756_amd import configs, lbm

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    lbm.lib()

    log("bandwidth probe (plain copy, 1 GiB)")
    probe_gbs, _ = lbm.lbm_bandwidth_probe(1 << 30, 20)

    p = configs.large_channel(prec)
    rho0 = configs.initial_density(p, seed=1)
    n = fluid_nodes(p)
    log("8192x512 %s: tune + %.2f s of untimed steps + %d warmup + %d timed steps"
        % (args.precision, PREHEAT_S, args.warmup, args.steps))
    ms, wall_ms, seg, waves, red = run_config(p, rho0, args.steps, args.warmup,
                                              tune=not args.no_tune, seg_rows=args.seg_rows)
    ms_step = ms / args.steps
    mlups = n * args.steps / (ms * 1e-3) / 1e6
    achieved = BYTES_PER_LUP[prec] * n / (ms_step * 1e-3) / 1e9
    traffic = counter_traffic(tag)
    log("%s %.4f ms/step  %.0f MLUPS  %.0f GB/s algorithmic" % (args.precision, ms_step, mlups, achieved))

    extra = {}
    if not args.no_extra:
        k = max(200, args.steps // 4)
        for name, prec2 in (("fp64", lbm.LBM_FP64), ("fp32_massexact", lbm.LBM_FP32_DEV_MASSEXACT)):
            q = configs.large_channel(prec2)
            log("8192x512 %s: %d steps" % (name, k))
            m2, _, s2, _, _ = run_config(q, rho0, k, 20, tune=not args.no_tune)
            extra[name] = dict(mlups=round(n * k / (m2 * 1e-3) / 1e6, 1),
                               ms_per_step=round(m2 / k, 5), seg_rows=s2,
                               hbm_gbs_algorithmic=round(BYTES_PER_LUP[prec2] * n / (m2 / k * 1e-3) / 1e9, 1))
        q = configs.single_gpu_channel(90.0, lbm.LBM_FP32_DEV)
        r2 = configs.initial_density(q, seed=1)
        log("2048x256 fp32 (cache-resident): %d steps" % (4 * k))
        m3, _, s3, _, _ = run_config(q, r2, 4 * k, 50, tune=not args.no_tune)
        n3 = fluid_nodes(q)
        extra["2048x256_fp32"] = dict(mlups=round(n3 * 4 * k / (m3 * 1e-3) / 1e6, 1),
                                      ms_per_step=round(m3 / (4 * k), 5), seg_rows=s3)

    if not args.no_extra:
        extra["precision_2048x256"] = precision_study()
        extra["mass_run_8192x512"] = large_mass_run()
        extra["d2_law_200x200"] = d2_law_study()
        extra["open_channel_1600x48"] = open_channel_run()
        extra["gravity_plate_100x300"] = gravity_plate_run()
        extra["open_channel_wettability"] = open_channel_wettability()

    batched = served = None
    if not args.no_batch:
        batched, served = batch_and_serve(args)

    cpu = None
    if not args.no_cpu_baseline:
        log("CPU oracle, all host threads: %d steps on the full 8192x512 grid"
            % args.cpu_steps_omp)
        cm_n, dt_n, thr = oracle_mlups(p, rho0, args.cpu_steps_omp, omp=True)
        log("CPU oracle, one thread: %d steps on the full 8192x512 grid" % args.cpu_steps)
        cm, dt, _ = oracle_mlups(p, rho0, args.cpu_steps)
        cpu = dict(value=round(cm_n, 3), unit="MLUPS", cores=thr, kind="oracle",
                   sample="FP64 oracle, OpenMP over rows on %d threads, %d steps of the full "
                          "8192x512 grid (%.1f s)" % (thr, args.cpu_steps_omp, dt_n),
                   single_thread=dict(value=round(cm, 3), unit="MLUPS", cores=1,
                                      sample="the sequential build, %d steps of the full "
                                             "8192x512 grid (%.1f s)" % (args.cpu_steps, dt)),
                   host=host_info())

    line = {
        "metric": "MLUPS & % HBM roofline (FP32 fused step); batched sims/s + p50/p99 latency",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": "plate channel 8192x512, %s, Tw=0.78Tc, "
                               "75 deg wall, drive 2e-6 / 4000 steps, seeded vapour noise" % storage,
                   "Nx": p.Nx, "Ny": p.Ny, "fluid_nodes": n, "seg_rows": seg, "waves": waves,
                   "untimed_preheat_s": PREHEAT_S},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "bytes_per_lup": BYTES_PER_LUP[prec],
                     "copy_probe_gbs": round(probe_gbs, 1),
                     "frac_of_copy_probe": round(achieved / probe_gbs, 4),
                     # HBM bytes the counters saw per launch, over the same time
                     "counter_gbs": None if traffic is None else round(traffic / (ms_step * 1e-3) / 1e9, 1),
                     "counter_frac": None if traffic is None else round(traffic / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "cpu_baseline": cpu,
        "wall_ms_timed": round(wall_ms, 3),
        "mass": red[0],
        "extra": extra,
        "batched": batched,
        "served": served,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

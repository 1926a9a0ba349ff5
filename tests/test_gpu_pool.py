"""GPU tests of the slot pool (batched and served runs) through the C-ABI.

A channel stepped inside a batch, admitted while other channels are already
running, must give bitwise the result of the same channel run alone: the
batched launch runs the same per-node arithmetic, only the work list
differs.  Admission must respect the byte cap."""
import numpy as np
import pytest

from helpers import field_errors, fluid_mask, to_oracle
from paper_1803_01756_amd import configs, inputs, lbm, serve

pytestmark = pytest.mark.gpu


def _case(name):
    print("\n[case] %s" % name, flush=True)


def _chan(Nx, Ny, ca, tw, g, per, seed, flags=0):
    p = configs.channel_params(Nx, Ny, ca, tw, g, per, lbm.LBM_FP32_DEV, flags)
    return p, configs.initial_density(p, seed)


def _alone(p, rho0, steps):
    s = lbm.Sim(p, rho0)
    s.step(steps)
    out = s.moments()
    s.close()
    return out


def test_pool_staggered_admission_equals_alone():
    _case("pool staggered admission")
    chans = [_chan(300, 34, 120.0, 0.80, 2e-6, 400.0, 1), _chan(140, 48, 150.0, 0.78, 5e-6, 300.0, 2),
             _chan(64, 20, 100.0, 0.84, 1e-6, 700.0, 3),
             _chan(515, 40, 130.0, 0.80, 3e-6, 250.0, 4, lbm.LBM_FREEZE_T)]
    steps = [400, 250, 330, 200]
    pool = lbm.Pool(1 << 30)
    sl = [pool.admit(chans[0][0], chans[0][1], steps[0]), pool.admit(chans[1][0], chans[1][1], steps[1])]
    pool.run(150)
    sl.append(pool.admit(chans[2][0], chans[2][1], steps[2]))
    pool.run(100)
    sl.append(pool.admit(chans[3][0], chans[3][1], steps[3]))
    done = set()
    for _ in range(20):
        pool.run(90)
        pool.wait(0)
        done |= set(pool.poll())
        if len(done) == 4:
            break
    assert done == set(sl)
    for (p, r0), s, n in zip(chans, sl, steps):
        assert pool.slot_time(s) == n
        got = pool.moments(s, p.Nx, p.Ny)
        ref = _alone(p, r0, n)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
    pool.close()


def test_pool_mixed_features_equal_alone():
    """One batch holding a plain channel and channels with each optional
    feature (Sec. 3.2 plates, phase-dependent properties, Carnahan-Starling,
    open ends, a held reservoir frame): a feature in any slot makes the whole
    batch run the kernel build with the optional features, and every slot,
    the plain one included, still gives bitwise its result alone.  A second
    batch holds a plain channel and one whose only option is the diffusivity
    cap, which alone selects that build."""
    _case("pool with optional features")
    prec = lbm.LBM_FP32_DEV
    plain = _chan(200, 30, 110.0, 0.80, 2e-6, 300.0, 11)
    grav = configs.gravity_plate(90, 40, cold_band=(30, 60), precision=prec)
    props = configs.channel_params(120, 26, 90.0, 0.78, 2e-5, 200.0, prec, lbm.LBM_PHASE_PROPS,
                                   lambda_l=0.6, C_v_l=3.0)
    cs = configs.channel_params_cs(96, 24, 0.45, 0.8, 1e-4, 400.0, prec)
    opn = configs.open_channel(131, 24, p_period=300.0, precision=prec)
    box = configs.d2_box(1.0 / 3.0, prec, N=60)
    chans = [plain, (grav, configs.initial_density(grav, 12)),
             (props, configs.initial_density(props, 13)), (cs, configs.initial_density(cs, 14)),
             (opn, configs.initial_density(opn, 15)), (box, configs.droplet_density(box, 20.0))]
    steps = [300, 260, 220, 280, 240, 200]
    pool = lbm.Pool(1 << 30)
    sl = [pool.admit(p, r0, n) for (p, r0), n in zip(chans, steps)]
    done = set()
    for _ in range(20):
        pool.run(100)
        pool.wait(0)
        done |= set(pool.poll())
        if len(done) == len(sl):
            break
    assert done == set(sl)
    for (p, r0), s, n in zip(chans, sl, steps):
        assert pool.slot_time(s) == n
        got = pool.moments(s, p.Nx, p.Ny)
        ref = _alone(p, r0, n)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
    pool.close()
    capped = configs.channel_params(150, 28, 100.0, 0.78, 2e-5, 200.0, prec, 0, alpha_max=0.1)
    chans = [_chan(170, 22, 120.0, 0.80, 2e-6, 300.0, 16), (capped, configs.initial_density(capped, 17))]
    pool = lbm.Pool(1 << 30)
    sl = [pool.admit(p, r0, 150) for p, r0 in chans]
    pool.run(150)
    pool.wait(0)
    for (p, r0), s in zip(chans, sl):
        for a, b in zip(pool.moments(s, p.Nx, p.Ny), _alone(p, r0, 150)):
            assert np.array_equal(a, b)
    pool.close()


def test_sampled_batch_channels_match_oracle(orc):
    """The eight smallest channels of the batched workload's draw (seed 1803:
    uneven sizes, contact angles 80-146 degrees, wall temperatures
    0.76-0.83 Tc, different drive periods and amplitudes), stepped together
    in one pool: each matches the oracle within 1e-5 after 100 steps."""
    _case("sampled batch channels vs oracle, 100 steps")
    draws = sorted(inputs.sample_channels(64, 1803), key=lambda d: d["Nx"] * d["Ny"])[:8]
    chans = [serve.channel_request(d, 100) for d in draws]
    pool = lbm.Pool(1 << 30)
    try:
        slots = [pool.admit(p, r0, 100) for p, r0 in chans]
        assert None not in slots
        pool.run(100)
        pool.wait(0)
        for (p, r0), s in zip(chans, slots):
            got = pool.moments(s, p.Nx, p.Ny)
            o = orc.Sim(to_oracle(orc, p), r0)
            o.step(100)
            e = field_errors(got, o.moments(), fluid_mask(p.Nx, p.Ny))
            print(p.Nx, p.Ny, e, flush=True)
            assert e["rho"] < 1e-5 and e["u"] < 1e-5 and e["T"] < 1e-5
    finally:
        pool.close()


def test_pool_autotune_leaves_states_and_results_unchanged():
    """lbm_pool_autotune on a batch whose slots span every row bucket (fluid
    rows 18 to 298) and carry an optional feature: the states, time levels
    and counters are those before the call (the trials step copies), every
    slot's shape follows the chosen policy (segments of about the bucket's
    target, balanced over its rows, seg + 10 a multiple of 6), and the
    finished results equal the runs alone bitwise."""
    _case("pool autotune")
    chans = [_chan(300, 20, 120.0, 0.80, 2e-6, 400.0, 1), _chan(140, 60, 150.0, 0.78, 5e-6, 300.0, 2),
             _chan(700, 100, 100.0, 0.84, 1e-6, 700.0, 3), _chan(96, 200, 130.0, 0.80, 3e-6, 250.0, 4),
             _chan(200, 300, 90.0, 0.80, 2e-6, 500.0, 5, lbm.LBM_PHASE_PROPS)]
    chans[-1][0].lambda_l, chans[-1][0].C_v_l = 0.6, 3.0
    steps = 120
    pool = lbm.Pool(1 << 31)
    with pytest.raises(lbm.LBMError) as ei:  # nothing admitted: nothing to tune
        pool.autotune(2)
    assert ei.value.status == lbm.LBM_EINVAL
    slots = [pool.admit(p, r0, steps) for p, r0 in chans]
    pool.run(40)
    before = [pool.moments(sl, p.Nx, p.Ny) for sl, (p, _) in zip(slots, chans)]
    health = [pool.slot_health(sl) for sl in slots]
    shapes0 = [pool.slot_launch(sl) for sl in slots]
    ms = pool.autotune(4)
    assert ms > 0
    shapes = [pool.slot_launch(sl) for sl in slots]
    print(dict(ms=ms, before=shapes0, after=shapes), flush=True)
    for sl, (p, r0), b, h in zip(slots, chans, before, health):
        assert pool.slot_time(sl) == 40 and pool.slot_health(sl) == h
        for x, y in zip(pool.moments(sl, p.Nx, p.Ny), b):
            assert np.array_equal(x, y)
    for (sr, waves), (p, _) in zip(shapes, chans):
        rows = p.Ny - 2
        assert 1 <= sr <= rows and (sr == rows or (sr + 10) % 6 == 0)
        assert waves == -(-p.Nx // 54) * -(-rows // sr)
    while True:
        pool.run(50)
        pool.wait(0)
        if all(pool.slot_time(sl) == steps for sl in slots):
            break
    for sl, (p, r0) in zip(slots, chans):
        got = pool.moments(sl, p.Nx, p.Ny)
        for x, y in zip(got, _alone(p, r0, steps)):
            assert np.array_equal(x, y)
    pool.close()


def test_pool_refuses_other_precisions():
    """Slots hold FP32 deviations only: FP64 and mass-exact requests are
    refused with LBM_EINVAL and leave the pool empty."""
    _case("pool precision check")
    pool = lbm.Pool(1 << 28)
    try:
        for prec in (lbm.LBM_FP64, lbm.LBM_FP32_DEV_MASSEXACT):
            p = configs.channel_params(64, 20, 90.0, 0.8, 1e-6, 500.0, prec)
            with pytest.raises(lbm.LBMError) as ei:
                pool.admit(p, configs.initial_density(p, 1), 10)
            assert ei.value.status == lbm.LBM_EINVAL
        assert pool.poll() == []
    finally:
        pool.close()


def test_pool_admission_by_footprint():
    _case("pool cap")
    a, b = _chan(256, 32, 120.0, 0.8, 1e-6, 500.0, 5), _chan(512, 64, 120.0, 0.8, 1e-6, 500.0, 6)
    fa, fb = lbm.lbm_pool_footprint(a[0]), lbm.lbm_pool_footprint(b[0])
    assert fa >= 256 * 30 * 80 and fb >= 512 * 62 * 80
    pool = lbm.Pool(fa + fb - 1)
    sa = pool.admit(a[0], a[1], 10)
    assert sa is not None
    assert pool.admit(b[0], b[1], 10) is None
    pool.run(10)
    pool.wait(0)
    pool.release(sa)
    sb = pool.admit(b[0], b[1], 10)
    assert sb is not None
    assert pool.info()[1] == fb
    pool.close()


def test_served_stream_results_equal_alone():
    """A served stream whose launch policy is tuned on the live mix after
    four admissions: every request's result equals its run alone."""
    _case("served stream, tuned after 4 admissions")
    reqs = serve.make_requests(10, rate=40.0, steps_scale=0.02)
    pool = lbm.Pool(8 << 30)
    serve.serve(reqs, pool, chunk=100, tune_after=4, tune_steps=2)
    pool.close()
    assert all(r.finished > r.arrival and not r.error for r in reqs)
    for r in reqs:
        ref = _alone(r.params, r.rho0, r.steps)
        for a, b in zip(r.result, ref):
            assert np.array_equal(a, b)

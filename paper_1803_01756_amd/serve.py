"""Batched and served runs on a slot pool.

``run_batch``  -- many independent channels of uneven size stepped together
                  in one batched launch per step (lbm_pool_run), timed, next
                  to the same channels run one after another alone.
``serve``      -- continuous batching: requests arrive as a Poisson stream,
                  are admitted into free slots as device memory allows
                  (footprint against a byte cap), are stepped together in
                  chunks while later requests keep arriving, and return
                  rho, u, T on the host when they finish.  Latency is arrival
                  to results on the host.  A request whose state turns
                  non-finite is retired by the pool and returns an error
                  (``Request.error``) instead of results; the loop goes on.

The scheduling logic works against any object with the ``lbm.Pool``
interface, so it can be exercised on the CPU with a fake pool.
"""
from __future__ import annotations

import collections
import os
import time
from dataclasses import dataclass, field

import numpy as np

from . import configs, inputs, lbm


class _Ranges:
    """roctx ranges around the serving loop's phases (admission, chunk
    enqueue, read-out, tuning) for rocprofv3 --marker-trace, enabled by the
    environment variable LBM_ROCTX=1; otherwise every call is a no-op."""

    def __init__(self):
        self.lib = None
        if os.environ.get("LBM_ROCTX") == "1":
            import ctypes
            # the rocprofiler-sdk library is the one rocprofv3 traces; the
            # older roctx library is the fallback
            for name in ("librocprofiler-sdk-roctx.so.1", "libroctx64.so"):
                try:
                    self.lib = ctypes.CDLL(name)
                    break
                except OSError:
                    continue
            if self.lib is None:
                raise OSError("LBM_ROCTX=1 but no roctx library could be loaded")
            self.lib.roctxRangePushA.argtypes = [ctypes.c_char_p]

    def push(self, name: str):
        if self.lib is not None:
            self.lib.roctxRangePushA(name.encode())

    def pop(self):
        if self.lib is not None:
            self.lib.roctxRangePop()


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    params: object          # lbm_params
    rho0: np.ndarray
    steps: int
    admitted: float = -1.0
    finished: float = -1.0
    slot: int = -1
    result: tuple = field(default=None, repr=False)
    error: str = ""         # set when the request was retired with a non-finite state


def channel_request(d: dict, steps: int, rid: int = 0) -> tuple:
    """Parameters and initial density of one sampled channel (a dict from
    inputs.sample_channels)."""
    p = configs.channel_params(d["Nx"], d["Ny"], d["contact_angle"], d["Tw_frac"], d["g_osc"],
                               d["period"], lbm.LBM_FP32_DEV)
    rho0 = configs.initial_density(p, seed=d["seed"])
    return p, rho0


def lup(p, steps: int) -> int:
    rows = p.Ny if (p.flags & lbm.LBM_PERIODIC_Y) else p.Ny - 2
    return p.Nx * rows * steps


def run_batch(channels, steps: int, chunk: int = 1000, cap_bytes: int = 200 << 30,
              seg_rows: int = 0, keep_results: bool = False, tune_steps: int = 0,
              info: dict = None):
    """Step every channel `steps` times in one pool; returns (seconds, results).
    tune_steps > 0: lbm_pool_autotune with that many steps per trial before
    the timed run (untimed); `info` then receives the tuned time per step
    and the slots' launch shapes."""
    pool = lbm.Pool(cap_bytes)
    if seg_rows:
        pool.set_launch(seg_rows)
    slots = []
    for p, rho0 in channels:
        s = pool.admit(p, rho0, steps)
        if s is None:
            raise RuntimeError("batch does not fit under the cap")
        slots.append(s)
    if tune_steps > 0:
        ms = pool.autotune(tune_steps)
        if info is not None:
            info["tuned_ms_per_step"] = ms
            info["shapes"] = [pool.slot_launch(s) for s in slots]
    elif info is not None:
        info["shapes"] = [pool.slot_launch(s) for s in slots]
    pool.synchronize()
    t0 = time.perf_counter()
    left = steps
    while left > 0:
        pool.run(min(chunk, left))
        left -= min(chunk, left)
    pool.synchronize()
    dt = time.perf_counter() - t0
    res = None
    if keep_results:
        res = [pool.moments(s, p.Nx, p.Ny) for s, (p, _) in zip(slots, channels)]
    pool.close()
    return dt, res


def run_alone(channels, steps: int, keep_results: bool = False, tune_steps: int = 0,
              shapes: list = None):
    """The same channels one after another with lbm_create/lbm_step;
    tune_steps > 0: each is autotuned first (lbm_autotune, untimed), and
    `shapes` receives each one's (rows per wave, waves)."""
    total = 0.0
    res = []
    for p, rho0 in channels:
        s = lbm.Sim(p, rho0)
        if tune_steps > 0:
            s.autotune(tune_steps)
        if shapes is not None:
            shapes.append(s.launch())
        s.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        s.synchronize()
        total += time.perf_counter() - t0
        if keep_results:
            res.append(s.moments())
        s.close()
    return total, (res if keep_results else None)


def serve(requests, pool, chunk: int = 500, max_pending: int = 2, clock=time.perf_counter,
          sleep=time.sleep, on_done=None, tune_after: int = 0, tune_steps: int = 4):
    """Continuous-batching loop.  ``requests`` sorted by arrival.  Returns the
    requests with admission / finish times and results filled in.
    tune_after > 0: once that many requests have been admitted, the pool's
    launch policy is tuned on the live mix (lbm_pool_autotune, tune_steps
    per trial; it blocks until the enqueued chunks are done)."""
    rg = _Ranges()
    t0 = clock()
    queue = collections.deque()
    by_slot = {}
    i, finished, admitted = 0, 0, 0
    tuned = tune_after <= 0
    n = len(requests)
    while finished < n:
        now = clock() - t0
        while i < n and requests[i].arrival <= now:
            queue.append(requests[i])
            i += 1
        # admit in arrival order while the footprint fits
        rg.push("serve: admit")
        while queue:
            r = queue[0]
            slot = pool.admit(r.params, r.rho0, r.steps)
            if slot is None:
                if not by_slot:  # an empty pool cannot hold it: it never will
                    raise ValueError("request of %dx%d needs more than the pool's cap"
                                     % (r.params.Nx, r.params.Ny))
                break
            queue.popleft()
            r.slot, r.admitted = slot, clock() - t0
            by_slot[slot] = r
            admitted += 1
        rg.pop()
        if not tuned and admitted >= tune_after and by_slot:
            rg.push("serve: tune")
            try:
                pool.autotune(tune_steps)
            except lbm.LBMError as e:  # no device memory for the trial copies:
                if e.status != lbm.LBM_ENOMEM:  # keep the default policy
                    raise
            rg.pop()
            tuned = True
        if by_slot:
            rg.push("serve: chunk")
            pool.run(chunk)
            pool.wait(max_pending)
            rg.pop()
        elif i < n:
            sleep(max(0.0, requests[i].arrival - (clock() - t0)))
        done = pool.poll()
        if done:
            rg.push("serve: read-out")
        for slot in done:
            r = by_slot.pop(slot)
            try:
                r.result = pool.moments(slot, r.params.Nx, r.params.Ny)
            except lbm.LBMError as e:
                if e.status != lbm.LBM_EUNSTABLE:
                    raise
                r.error = str(e)  # retired: its state became non-finite
            r.finished = clock() - t0
            pool.release(slot)
            finished += 1
            if on_done:
                on_done(r)
        if done:
            rg.pop()
        if by_slot and not done:
            sleep(0.0002)  # remaining slots are finishing their last chunk
    return requests


def latency_stats(reqs):
    lat = np.array([r.finished - r.arrival for r in reqs])
    span = max(r.finished for r in reqs) - min(r.arrival for r in reqs)
    return dict(p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                mean_s=float(lat.mean()), sims_per_s=len(reqs) / span if span > 0 else 0.0,
                span_s=span)


def make_requests(n: int, rate: float, seed_arrivals: int = 20, seed_params: int = 1803,
                  steps_scale: float = 1.0):
    arrivals, steps = inputs.poisson_arrivals(n, rate, seed_arrivals)
    chans = inputs.sample_channels(n, seed_params)
    reqs = []
    for k in range(n):
        st = max(1, int(round(int(steps[k]) * steps_scale)))
        p, rho0 = channel_request(chans[k], st, k)
        reqs.append(Request(rid=k, arrival=float(arrivals[k]), params=p, rho0=rho0, steps=st))
    return reqs

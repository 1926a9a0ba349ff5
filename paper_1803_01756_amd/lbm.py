"""Python binding of the C-ABI in ``include/lbm.h`` (ctypes, argument
marshalling only).  Every step of the method runs in the HIP library
``liblbm_hip.so``; when that library is missing or cannot be loaded, the
calls raise instead of falling back to anything else.

The functions keep the C names (``lbm_create``, ``lbm_step``, ...); ``Sim``
wraps them for convenience and can take its device memory and stream from
PyTorch.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblbm_hip.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LBM_FP32_DEV, LBM_FP64, LBM_FP32_DEV_MASSEXACT = 0, 1, 2
LBM_FREEZE_T, LBM_SINGLE_PHASE, LBM_PERIODIC_Y, LBM_FRAME_T, LBM_FRAME_RHO, LBM_EOS_CS = 1, 2, 4, 8, 16, 32
LBM_OPEN_X, LBM_PHASE_PROPS, LBM_TOP_MIXED = 64, 128, 256

_STATUS = {LBM_EINVAL: "EINVAL", LBM_ENOMEM: "ENOMEM", LBM_EDEVICE: "EDEVICE",
           LBM_EUNSTABLE: "EUNSTABLE", LBM_ESTATE: "ESTATE"}


class LBMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


class lbm_params(C.Structure):
    _fields_ = [
        ("Nx", C.c_int32), ("Ny", C.c_int32),
        ("a", C.c_double), ("b", C.c_double), ("R", C.c_double), ("omega", C.c_double),
        ("T_c", C.c_double), ("G", C.c_double), ("theta", C.c_double),
        ("G_w", C.c_double), ("psi_w", C.c_double),
        ("s_rho", C.c_double), ("s_e", C.c_double), ("s_zeta", C.c_double),
        ("s_j", C.c_double), ("s_q", C.c_double),
        ("tau_g", C.c_double), ("tau_l", C.c_double),
        ("rho_g", C.c_double), ("rho_l", C.c_double),
        ("C_v", C.c_double), ("lambda_", C.c_double),
        ("T_0", C.c_double), ("T_w", C.c_double),
        ("g_osc", C.c_double), ("period", C.c_double),
        ("g_x", C.c_double), ("g_y", C.c_double), ("rho_v", C.c_double),
        ("rho_ref", C.c_double), ("rho_frame", C.c_double),
        ("p_amp", C.c_double), ("p_period", C.c_double),
        ("T_w_end", C.c_double), ("T_in", C.c_double),
        ("lambda_l", C.c_double), ("C_v_l", C.c_double),
        ("T_w_bottom", C.c_double), ("cold_x0", C.c_int32), ("cold_x1", C.c_int32),
        ("precision", C.c_int32), ("flags", C.c_uint32),
        ("alpha_max", C.c_double), ("T_out", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load the HIP library (raises if it has not been built).

    PyTorch-ROCm carries its own HIP runtime.  Importing torch first makes the
    dynamic loader bind this library to that same runtime, so a process that
    also uses torch (for device memory, streams or events) holds a single HIP
    runtime; loading the system runtime first would leave torch unable to
    initialise the GPU."""
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is not built; run "
                               "`python -m paper_1803_01756_amd.build`" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        P = C.POINTER(lbm_params)
        vp, dp = C.c_void_p, C.POINTER(C.c_double)
        sig = {
            "lbm_params_default": (None, [P]),
            "lbm_params_resolve": (C.c_int, [P]),
            "lbm_eos_critical": (C.c_int, [C.c_double, C.c_double, C.c_double, dp, dp]),
            "lbm_eos_critical_cs": (C.c_int, [C.c_double, C.c_double, C.c_double, dp, dp]),
            "lbm_eos_coexistence": (C.c_int, [P, C.c_double, dp, dp, dp]),
            "lbm_eos_pressure": (C.c_int, [P, C.c_double, C.c_double, dp, dp]),
            "lbm_eos_latent_heat": (C.c_int, [P, C.c_double, dp]),
            "lbm_eos_jacob": (C.c_int, [P, C.c_double, C.c_double, dp]),
            "lbm_health": (C.c_int, [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
            "lbm_reduce_noalloc": (C.c_int, [vp, vp]),
            "lbm_pool_slot_health": (C.c_int, [vp, C.c_int32, C.POINTER(C.c_int64),
                                               C.POINTER(C.c_int64)]),
            "lbm_workspace_bytes": (C.c_size_t, [P]),
            "lbm_create": (C.c_int, [P, dp, vp, C.c_size_t, vp, C.POINTER(vp)]),
            "lbm_step": (C.c_int, [vp, C.c_int64]),
            "lbm_moments": (C.c_int, [vp, dp, dp, dp, dp]),
            "lbm_reduce": (C.c_int, [vp, dp]),
            "lbm_synchronize": (C.c_int, [vp]),
            "lbm_destroy": (C.c_int, [vp]),
            "lbm_time": (C.c_int64, [vp]),
            "lbm_get_params": (C.c_int, [vp, P]),
            "lbm_last_error": (C.c_char_p, []),
            "lbm_state_bytes": (C.c_size_t, [vp]),
            "lbm_save": (C.c_int, [vp, vp, C.c_size_t]),
            "lbm_load": (C.c_int, [vp, vp, C.c_size_t]),
            "lbm_set_launch": (C.c_int, [vp, C.c_int32]),
            "lbm_get_launch": (C.c_int, [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
            "lbm_autotune": (C.c_int, [vp, C.c_int32, dp]),
            "lbm_bandwidth_probe": (C.c_int, [C.c_size_t, C.c_int32, dp, dp]),
            "lbm_pool_footprint": (C.c_size_t, [P]),
            "lbm_pool_create": (C.c_int, [C.c_size_t, vp, C.POINTER(vp)]),
            "lbm_pool_admit": (C.c_int, [vp, P, dp, C.c_int64, C.POINTER(C.c_int32)]),
            "lbm_pool_run": (C.c_int, [vp, C.c_int32]),
            "lbm_pool_poll": (C.c_int, [vp, C.POINTER(C.c_int32), C.c_int32,
                                        C.POINTER(C.c_int32)]),
            "lbm_pool_moments": (C.c_int, [vp, C.c_int32, dp, dp, dp, dp]),
            "lbm_pool_release": (C.c_int, [vp, C.c_int32]),
            "lbm_pool_destroy": (C.c_int, [vp]),
            "lbm_pool_info": (C.c_int, [vp, C.POINTER(C.c_int32), C.POINTER(C.c_size_t),
                                        C.POINTER(C.c_size_t)]),
            "lbm_pool_slot_time": (C.c_int64, [vp, C.c_int32]),
            "lbm_pool_set_launch": (C.c_int, [vp, C.c_int32]),
            "lbm_pool_autotune": (C.c_int, [vp, C.c_int32, C.POINTER(C.c_double)]),
            "lbm_pool_slot_launch": (C.c_int, [vp, C.c_int32, C.POINTER(C.c_int32),
                                               C.POINTER(C.c_int32)]),
            "lbm_pool_synchronize": (C.c_int, [vp]),
            "lbm_pool_wait": (C.c_int, [vp, C.c_int32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    """Names the header declares; the CPU tests check the library has them."""
    return ["lbm_params_default", "lbm_params_resolve", "lbm_eos_critical", "lbm_eos_critical_cs",
            "lbm_eos_coexistence", "lbm_eos_pressure", "lbm_eos_latent_heat", "lbm_eos_jacob",
            "lbm_workspace_bytes", "lbm_create", "lbm_step",
            "lbm_moments", "lbm_reduce", "lbm_reduce_noalloc", "lbm_synchronize",
            "lbm_health", "lbm_destroy",
            "lbm_time",
            "lbm_get_params", "lbm_last_error", "lbm_state_bytes", "lbm_save", "lbm_load",
            "lbm_set_launch", "lbm_get_launch", "lbm_autotune", "lbm_bandwidth_probe",
            "lbm_pool_footprint", "lbm_pool_create", "lbm_pool_admit", "lbm_pool_run",
            "lbm_pool_poll", "lbm_pool_moments", "lbm_pool_slot_health", "lbm_pool_release",
            "lbm_pool_destroy",
            "lbm_pool_info", "lbm_pool_slot_time", "lbm_pool_set_launch",
            "lbm_pool_autotune", "lbm_pool_slot_launch",
            "lbm_pool_synchronize", "lbm_pool_wait"]


def _check(st: int):
    if st != LBM_OK:
        raise LBMError(st, lib().lbm_last_error().decode())


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


# ---- thin wrappers with the C names ----------------------------------------
def lbm_params_default(**overrides) -> lbm_params:
    p = lbm_params()
    lib().lbm_params_default(C.byref(p))
    for k, v in overrides.items():
        setattr(p, "lambda_" if k == "lambda" else k, v)
    return p


def lbm_params_resolve(p: lbm_params) -> lbm_params:
    q = lbm_params.from_buffer_copy(p)
    _check(lib().lbm_params_resolve(C.byref(q)))
    return q


def lbm_eos_critical(a=3.0 / 49.0, b=2.0 / 21.0, R=1.0):
    rc, tc = C.c_double(), C.c_double()
    _check(lib().lbm_eos_critical(a, b, R, C.byref(rc), C.byref(tc)))
    return rc.value, tc.value


def lbm_eos_critical_cs(a=1.0, b=4.0, R=1.0):
    rc, tc = C.c_double(), C.c_double()
    _check(lib().lbm_eos_critical_cs(a, b, R, C.byref(rc), C.byref(tc)))
    return rc.value, tc.value


def lbm_eos_coexistence(p: lbm_params, T: float):
    g, l, ps = C.c_double(), C.c_double(), C.c_double()
    _check(lib().lbm_eos_coexistence(C.byref(p), T, C.byref(g), C.byref(l), C.byref(ps)))
    return g.value, l.value, ps.value


def lbm_eos_latent_heat(p: lbm_params, T: float) -> float:
    """h_fg of Eq. 19 at T < T_c."""
    h = C.c_double()
    _check(lib().lbm_eos_latent_heat(C.byref(p), T, C.byref(h)))
    return h.value


def lbm_eos_jacob(p: lbm_params, T_sat: float, T_w: float) -> float:
    """Eq. 20: Ja = C_v (T_sat - T_w) / h_fg(T_sat) (computed by the library)."""
    ja = C.c_double()
    _check(lib().lbm_eos_jacob(C.byref(p), T_sat, T_w, C.byref(ja)))
    return ja.value


jacob_number = lbm_eos_jacob


def lbm_eos_pressure(p: lbm_params, rho: float, T: float):
    """(P_EOS, psi) at (rho, T)."""
    P, ps = C.c_double(), C.c_double()
    _check(lib().lbm_eos_pressure(C.byref(p), rho, T, C.byref(P), C.byref(ps)))
    return P.value, ps.value


def lbm_workspace_bytes(p: lbm_params) -> int:
    return int(lib().lbm_workspace_bytes(C.byref(p)))


def lbm_create(p: lbm_params, rho0=None, workspace: int = 0, ws_bytes: int = 0,
               stream: int = 0) -> int:
    h = C.c_void_p()
    r = None
    if rho0 is not None:
        r = np.ascontiguousarray(rho0, dtype=np.float64)
        if r.size != p.Nx * p.Ny:
            raise ValueError("rho0 must have Nx*Ny entries")
    _check(lib().lbm_create(C.byref(p), _dp(r), C.c_void_p(workspace or None), ws_bytes,
                            C.c_void_p(stream or None), C.byref(h)))
    return h.value


def lbm_step(h: int, n: int):
    _check(lib().lbm_step(C.c_void_p(h), int(n)))


def lbm_moments(h: int, Nx: int, Ny: int):
    outs = [np.empty((Ny, Nx)) for _ in range(4)]
    _check(lib().lbm_moments(C.c_void_p(h), *[_dp(o) for o in outs]))
    return tuple(outs)


def lbm_reduce(h: int, check: bool = True):
    out = np.zeros(5)
    st = lib().lbm_reduce(C.c_void_p(h), _dp(out))
    if check or st != LBM_EUNSTABLE:
        _check(st)
    return out


def lbm_reduce_noalloc(h: int, out_dev: int):
    """Enqueue the lbm_reduce totals into 5 doubles of device memory at
    out_dev (allocation-free, asynchronous)."""
    _check(lib().lbm_reduce_noalloc(C.c_void_p(h), C.c_void_p(out_dev)))


def lbm_synchronize(h: int):
    _check(lib().lbm_synchronize(C.c_void_p(h)))


def lbm_health(h: int):
    """(non-finite readings, psi clamps) counted by the steps so far."""
    a, b = C.c_int64(), C.c_int64()
    _check(lib().lbm_health(C.c_void_p(h), C.byref(a), C.byref(b)))
    return a.value, b.value


def lbm_destroy(h: int):
    _check(lib().lbm_destroy(C.c_void_p(h)))


def lbm_time(h: int) -> int:
    return int(lib().lbm_time(C.c_void_p(h)))


def lbm_get_params(h: int) -> lbm_params:
    p = lbm_params()
    _check(lib().lbm_get_params(C.c_void_p(h), C.byref(p)))
    return p


def lbm_save(h: int) -> bytes:
    n = int(lib().lbm_state_bytes(C.c_void_p(h)))
    buf = C.create_string_buffer(n)
    _check(lib().lbm_save(C.c_void_p(h), buf, n))
    return buf.raw


def lbm_load(h: int, blob: bytes):
    buf = C.create_string_buffer(blob, len(blob))
    _check(lib().lbm_load(C.c_void_p(h), buf, len(blob)))


def lbm_set_launch(h: int, seg_rows: int):
    _check(lib().lbm_set_launch(C.c_void_p(h), int(seg_rows)))


def lbm_get_launch(h: int):
    s, w = C.c_int32(), C.c_int32()
    _check(lib().lbm_get_launch(C.c_void_p(h), C.byref(s), C.byref(w)))
    return s.value, w.value


def lbm_autotune(h: int, steps_per_trial: int = 10) -> float:
    ms = C.c_double()
    _check(lib().lbm_autotune(C.c_void_p(h), int(steps_per_trial), C.byref(ms)))
    return ms.value


def lbm_bandwidth_probe(nbytes: int, iters: int = 20):
    """(GB/s counting read + write, ms per copy) of a plain device copy."""
    g, ms = C.c_double(), C.c_double()
    _check(lib().lbm_bandwidth_probe(int(nbytes), int(iters), C.byref(g), C.byref(ms)))
    return g.value, ms.value


class Sim:
    """One simulation.  With ``torch_memory=True`` the device workspace is a
    torch tensor and the work is ordered on torch's current stream."""

    def __init__(self, params: lbm_params, rho0=None, torch_memory: bool = False):
        self._ws = None
        ws_ptr, ws_bytes, stream = 0, 0, 0
        if torch_memory:
            import torch
            ws_bytes = lbm_workspace_bytes(params)
            if ws_bytes == 0:
                raise LBMError(LBM_EINVAL, lib().lbm_last_error().decode())
            self._ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
            ws_ptr = self._ws.data_ptr()
            stream = torch.cuda.current_stream().cuda_stream
        self.h = lbm_create(params, rho0, ws_ptr, ws_bytes, stream)
        self.params = lbm_get_params(self.h)
        self.Nx, self.Ny = self.params.Nx, self.params.Ny

    def step(self, n: int = 1):
        """Enqueue n steps (lbm_step); returns before they run."""
        lbm_step(self.h, n)

    def moments(self):
        """(rho, ux, uy, T) as float64 [Ny, Nx] host arrays."""
        return lbm_moments(self.h, self.Nx, self.Ny)

    def reduce(self, check: bool = True):
        """FP64 totals of the fluid nodes (lbm_reduce); with check, a
        non-finite state raises LBMError(LBM_EUNSTABLE)."""
        return lbm_reduce(self.h, check)

    def synchronize(self):
        """Wait for the enqueued steps (lbm_synchronize); a non-finite state
        read by a step raises LBMError(LBM_EUNSTABLE)."""
        lbm_synchronize(self.h)

    def health(self):
        """(non-finite node readings, psi clamps) counted by the steps so far
        (lbm_health)."""
        return lbm_health(self.h)

    @property
    def n(self) -> int:
        """Current time level (lbm_time)."""
        return lbm_time(self.h)

    def save(self) -> bytes:
        """Checkpoint of the time level, parameters and state (lbm_save)."""
        return lbm_save(self.h)

    def load(self, blob: bytes):
        """Restore a checkpoint of a channel of the same grid and precision
        (lbm_load)."""
        lbm_load(self.h, blob)

    def set_launch(self, seg_rows: int):
        """Rows per wave of the step kernel; <= 0 restores the default
        (lbm_set_launch).  Results do not depend on it."""
        lbm_set_launch(self.h, seg_rows)

    def launch(self):
        """(seg_rows, waves) of the current launch shape (lbm_get_launch)."""
        return lbm_get_launch(self.h)

    def autotune(self, steps_per_trial: int = 10) -> float:
        """Time candidate launch shapes on this channel, keep the fastest and
        restore the state (lbm_autotune); returns its ms per step."""
        return lbm_autotune(self.h, steps_per_trial)

    def close(self):
        """Free the simulation (lbm_destroy); idempotent."""
        if getattr(self, "h", None):
            lbm_destroy(self.h)
            self.h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ---- slot pool (batched and served runs) ------------------------------------
def lbm_pool_footprint(p: lbm_params) -> int:
    return int(lib().lbm_pool_footprint(C.byref(p)))


class Pool:
    """Wrapper of the lbm_pool_* calls.  ``admit`` returns the slot id or
    None when the footprint does not fit under the cap."""

    def __init__(self, cap_bytes: int, torch_stream: bool = False):
        stream = 0
        if torch_stream:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        h = C.c_void_p()
        _check(lib().lbm_pool_create(int(cap_bytes), C.c_void_p(stream or None), C.byref(h)))
        self.h = h.value

    def admit(self, p: lbm_params, rho0, nsteps: int):
        """Admit a channel for nsteps steps (lbm_pool_admit): its slot id,
        or None while its footprint does not fit under the cap."""
        r = None if rho0 is None else np.ascontiguousarray(rho0, dtype=np.float64)
        slot = C.c_int32()
        st = lib().lbm_pool_admit(C.c_void_p(self.h), C.byref(p), _dp(r), int(nsteps),
                                  C.byref(slot))
        if st == LBM_ENOMEM:
            return None
        _check(st)
        return slot.value

    def run(self, chunk_steps: int):
        """Enqueue up to chunk_steps steps of every unfinished slot
        (lbm_pool_run)."""
        _check(lib().lbm_pool_run(C.c_void_p(self.h), int(chunk_steps)))

    def poll(self, max_n: int = 1024):
        """Slots that finished since the last poll (lbm_pool_poll)."""
        buf = (C.c_int32 * max_n)()
        n = C.c_int32()
        _check(lib().lbm_pool_poll(C.c_void_p(self.h), buf, max_n, C.byref(n)))
        return list(buf[:n.value])

    def moments(self, slot: int, Nx: int, Ny: int):
        """(rho, ux, uy, T) of a slot as float64 [Ny, Nx] arrays
        (lbm_pool_moments)."""
        outs = [np.empty((Ny, Nx)) for _ in range(4)]
        _check(lib().lbm_pool_moments(C.c_void_p(self.h), int(slot), *[_dp(o) for o in outs]))
        return tuple(outs)

    def slot_health(self, slot: int):
        """(non-finite node readings, psi clamps) of a slot
        (lbm_pool_slot_health)."""
        a, b = C.c_int64(), C.c_int64()
        _check(lib().lbm_pool_slot_health(C.c_void_p(self.h), int(slot), C.byref(a),
                                          C.byref(b)))
        return a.value, b.value

    def release(self, slot: int):
        """Free a slot's memory for later admissions (lbm_pool_release)."""
        _check(lib().lbm_pool_release(C.c_void_p(self.h), int(slot)))

    def info(self):
        """(active slots, bytes used, cap bytes) (lbm_pool_info)."""
        a, u, c = C.c_int32(), C.c_size_t(), C.c_size_t()
        _check(lib().lbm_pool_info(C.c_void_p(self.h), C.byref(a), C.byref(u), C.byref(c)))
        return a.value, u.value, c.value

    def slot_time(self, slot: int) -> int:
        """Time level a slot has reached, -1 for no such slot."""
        return int(lib().lbm_pool_slot_time(C.c_void_p(self.h), int(slot)))

    def set_launch(self, seg_rows: int):
        """Rows per wave for every slot; <= 0: per-slot default."""
        _check(lib().lbm_pool_set_launch(C.c_void_p(self.h), int(seg_rows)))

    def autotune(self, steps_per_trial: int = 10) -> float:
        """lbm_pool_autotune: keep the fastest launch policy for the slots
        with steps left; returns its time per batched step in ms."""
        ms = C.c_double()
        _check(lib().lbm_pool_autotune(C.c_void_p(self.h), int(steps_per_trial), C.byref(ms)))
        return ms.value

    def slot_launch(self, slot: int):
        """(rows per wave, waves per step) of a slot."""
        sr, w = C.c_int32(), C.c_int32()
        _check(lib().lbm_pool_slot_launch(C.c_void_p(self.h), int(slot), C.byref(sr),
                                          C.byref(w)))
        return sr.value, w.value

    def synchronize(self):
        """Wait for every enqueued chunk."""
        _check(lib().lbm_pool_synchronize(C.c_void_p(self.h)))

    def wait(self, max_pending: int):
        """Block until at most max_pending chunks are still running."""
        _check(lib().lbm_pool_wait(C.c_void_p(self.h), int(max_pending)))

    def close(self):
        """Free the pool and every slot (lbm_pool_destroy); idempotent."""
        if getattr(self, "h", None):
            lib().lbm_pool_destroy(C.c_void_p(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

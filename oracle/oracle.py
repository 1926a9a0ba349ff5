"""ctypes front end of the FP64 CPU oracle (``lbm_oracle.c``).

TEST INFRASTRUCTURE ONLY: the oracle is the plain, slow reference that the GPU
path is checked against.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this module.  It does not import the
GPU package and the GPU package does not import it.

Functions follow arXiv:1803.01756 Section 2 (Eqs. 1-18); see the header of
``lbm_oracle.c`` for the readings taken where the paper is silent or garbled.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")
# the same source built with OpenMP over the rows of every sweep (bitwise the
# same results; used to time the oracle on all host cores)
LIB_OMP = os.path.join(HERE, "liblbm_oracle_omp.so")

FREEZE_T = 1
SINGLE_PHASE = 2
PERIODIC_Y = 4
FRAME_T = 8
FRAME_RHO = 16
EOS_CS = 32
OPEN_X = 64
PHASE_PROPS = 128
TOP_MIXED = 256


def build(force: bool = False, omp: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math); omp: the
    OpenMP-over-rows build."""
    out = LIB_OMP if omp else LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-shared", "-fPIC"] + (["-fopenmp"] if omp else []) +
            ["-o", tmp, SRC, "-lm"])
        os.replace(tmp, out)
    return out


class OrcParams(C.Structure):
    _fields_ = [
        ("Nx", C.c_int32), ("Ny", C.c_int32),
        ("a", C.c_double), ("b", C.c_double), ("R", C.c_double),
        ("omega", C.c_double), ("Tc", C.c_double),
        ("G", C.c_double), ("theta", C.c_double),
        ("Gw", C.c_double), ("psiw", C.c_double),
        ("s_rho", C.c_double), ("s_e", C.c_double), ("s_zeta", C.c_double),
        ("s_j", C.c_double), ("s_q", C.c_double),
        ("tau_g", C.c_double), ("tau_l", C.c_double),
        ("rho_g", C.c_double), ("rho_l", C.c_double),
        ("Cv", C.c_double), ("lam", C.c_double),
        ("T0", C.c_double), ("Tw", C.c_double),
        ("g_osc", C.c_double), ("period", C.c_double),
        ("gx", C.c_double), ("gy", C.c_double), ("rho_v", C.c_double),
        ("rho_frame", C.c_double),
        ("p_amp", C.c_double), ("p_period", C.c_double),
        ("Tw_end", C.c_double), ("T_in", C.c_double),
        ("lam_l", C.c_double), ("Cv_l", C.c_double),
        ("Tw_bot", C.c_double), ("cold_x0", C.c_int32), ("cold_x1", C.c_int32),
        ("flags", C.c_uint32), ("pad_", C.c_int32),
        ("alpha_max", C.c_double), ("T_out", C.c_double),
    ]


_lib = None
_lib_omp = None


def lib(omp: bool = False):
    """The sequential oracle library, or with omp the OpenMP build."""
    global _lib, _lib_omp
    if (_lib_omp if omp else _lib) is None:
        build(omp=omp)
        L = C.CDLL(LIB_OMP if omp else LIB)
        dp = C.POINTER(C.c_double)
        P = C.POINTER(OrcParams)
        L.orc_matrix_M.argtypes = [dp]
        L.orc_matrix_Minv.argtypes = [dp]
        for name in ("orc_peos", "orc_dpdrho", "orc_dpdT", "orc_psi"):
            getattr(L, name).argtypes = [P, C.c_double, C.c_double]
            getattr(L, name).restype = C.c_double
        L.orc_phi.argtypes = [P, C.c_double]
        L.orc_phi.restype = C.c_double
        L.orc_critical.argtypes = [C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_critical_cs.argtypes = [C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_maxwell.argtypes = [P, C.c_double, dp, dp, dp]
        L.orc_maxwell.restype = C.c_int
        L.orc_latent_heat.argtypes = [P, C.c_double, dp]
        L.orc_inlet_density.argtypes = [P, C.c_int64]
        L.orc_inlet_density.restype = C.c_double
        L.orc_latent_heat.restype = C.c_int
        L.orc_collide_node.argtypes = [P, dp] + [C.c_double] * 9 + [dp]
        L.orc_heat_rhs.argtypes = [P, dp, dp, dp, dp, dp]
        L.orc_sim_new.argtypes = [P]
        L.orc_sim_new.restype = C.c_void_p
        L.orc_sim_free.argtypes = [C.c_void_p]
        L.orc_sim_init.argtypes = [C.c_void_p, dp, C.c_double]
        L.orc_sim_set_f.argtypes = [C.c_void_p, dp]
        L.orc_sim_get_f.argtypes = [C.c_void_p, dp]
        L.orc_sim_set_T.argtypes = [C.c_void_p, dp]
        L.orc_sim_set_time.argtypes = [C.c_void_p, C.c_int64]
        L.orc_sim_time.argtypes = [C.c_void_p]
        L.orc_sim_time.restype = C.c_int64
        L.orc_sim_psi_clamps.argtypes = [C.c_void_p]
        L.orc_sim_psi_clamps.restype = C.c_int64
        L.orc_sim_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_sim_moments.argtypes = [C.c_void_p] + [dp] * 6
        L.orc_threads.restype = C.c_int
        if omp:
            _lib_omp = L
        else:
            _lib = L
    return _lib_omp if omp else _lib


def threads(omp: bool = True) -> int:
    """Threads a row sweep of that build uses (OMP_NUM_THREADS)."""
    return int(lib(omp).orc_threads())


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(**kw) -> OrcParams:
    p = OrcParams()
    for k, v in kw.items():
        setattr(p, "lam" if k == "lambda_" else k, v)
    return p


# ---- thermodynamics (Eq. 10-11) ------------------------------------------
def critical(a: float = 3.0 / 49.0, b: float = 2.0 / 21.0, R: float = 1.0):
    """Critical density and temperature of the Peng-Robinson EOS (Eq. 11)."""
    rc, tc = C.c_double(), C.c_double()
    lib().orc_critical(a, b, R, C.byref(rc), C.byref(tc))
    return rc.value, tc.value


def critical_cs(a: float = 1.0, b: float = 4.0, R: float = 1.0):
    """Critical density and temperature of the Carnahan-Starling EOS."""
    rc, tc = C.c_double(), C.c_double()
    lib().orc_critical_cs(a, b, R, C.byref(rc), C.byref(tc))
    return rc.value, tc.value


def default_params_cs(Nx: int = 128, Ny: int = 32, **kw) -> OrcParams:
    """default_params with the Carnahan-Starling EOS (a = 1, b = 4, R = 1),
    T0 = 0.86 Tc and T_w = 0.80 Tc of its own critical temperature."""
    _, tc = critical_cs()
    d = dict(a=1.0, b=4.0, R=1.0, Tc=tc, T0=0.86 * tc, Tw=0.80 * tc, flags=EOS_CS)
    d.update(kw)
    d["flags"] = d["flags"] | EOS_CS
    return default_params(Nx, Ny, **d)


def peos(p: OrcParams, rho: float, T: float) -> float:
    return lib().orc_peos(C.byref(p), rho, T)


def dpdrho(p: OrcParams, rho: float, T: float) -> float:
    return lib().orc_dpdrho(C.byref(p), rho, T)


def dpdT(p: OrcParams, rho: float, T: float) -> float:
    return lib().orc_dpdT(C.byref(p), rho, T)


def psi(p: OrcParams, rho: float, T: float) -> float:
    return lib().orc_psi(C.byref(p), rho, T)


def maxwell(p: OrcParams, T: float):
    """Equal-area coexistence (rho_g, rho_l, p_sat) at T < Tc."""
    g, l, ps = C.c_double(), C.c_double(), C.c_double()
    rc = lib().orc_maxwell(C.byref(p), T, C.byref(g), C.byref(l), C.byref(ps))
    if rc != 0:
        raise ValueError("temperature %g is not below the critical point" % T)
    return g.value, l.value, ps.value


def latent_heat(p: OrcParams, T: float) -> float:
    """Eq. 19 latent heat h_fg at T < Tc."""
    h = C.c_double()
    if lib().orc_latent_heat(C.byref(p), T, C.byref(h)) != 0:
        raise ValueError("temperature %g is not below the critical point" % T)
    return h.value


def inlet_density(p: OrcParams, n: int) -> float:
    """OPEN_X inlet density at time level n (vapour-branch root of the
    oscillating inlet pressure)."""
    return lib().orc_inlet_density(C.byref(p), n)


def jacob(p: OrcParams, T_sat: float, T_w: float) -> float:
    """Eq. 20: Ja = C_v (T_sat - T_w) / h_fg(T_sat)."""
    return p.Cv * (T_sat - T_w) / latent_heat(p, T_sat)


def matrix_M() -> np.ndarray:
    out = np.zeros(81)
    lib().orc_matrix_M(_dp(out))
    return out.reshape(9, 9)


def matrix_Minv() -> np.ndarray:
    out = np.zeros(81)
    lib().orc_matrix_Minv(_dp(out))
    return out.reshape(9, 9)


def collide_node(p: OrcParams, f, rho, ux, uy, Fx, Fy, Fmx, Fmy, psi_, tau_v) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(9)
    lib().orc_collide_node(C.byref(p), _dp(f), rho, ux, uy, Fx, Fy, Fmx, Fmy, psi_, tau_v,
                           _dp(out))
    return out


def heat_rhs(p: OrcParams, rho, ux, uy, T) -> np.ndarray:
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (rho, ux, uy, T)]
    out = np.zeros_like(arrs[3])
    lib().orc_heat_rhs(C.byref(p), *[_dp(a) for a in arrs], _dp(out))
    return out


def default_params(Nx: int = 128, Ny: int = 32, **kw) -> OrcParams:
    """Paper values (Eq. 11: a = 3/49, b = 2/21, R = 1; Sec. 3.2: C_v = 5,
    lambda = 0.25) and the readings for the unstated ones: omega = 0.344,
    G = -1, theta = 0.104, s_rho = s_j = 1, s_e = s_zeta = 0.8, s_q = 1.1,
    tau_g = tau_l = 1, T0 = 0.86 Tc, T_w = 0.80 Tc; rho_g, rho_l, rho_v not
    given (or None) are the Maxwell coexistence densities at T0."""
    _, tc = critical()
    d = dict(Nx=Nx, Ny=Ny, a=3.0 / 49.0, b=2.0 / 21.0, R=1.0, omega=0.344, Tc=tc,
             G=-1.0, theta=0.104, Gw=0.0, psiw=0.0,
             s_rho=1.0, s_e=0.8, s_zeta=0.8, s_j=1.0, s_q=1.1,
             tau_g=1.0, tau_l=1.0, rho_g=None, rho_l=None,
             Cv=5.0, lam=0.25, T0=0.86 * tc, Tw=0.80 * tc,
             g_osc=1e-6, period=2000.0, gx=0.0, gy=0.0, rho_v=None, flags=0)
    d.update({("lam" if k == "lambda_" else k): v for k, v in kw.items()})
    derived = [k for k in ("rho_g", "rho_l", "rho_v") if d[k] is None]
    p = make_params(**{k: v for k, v in d.items() if v is not None})
    if derived:
        g, l, _ = maxwell(p, p.T0)
        vals = dict(rho_g=g, rho_l=l, rho_v=g)
        for k in derived:
            setattr(p, k, vals[k])
    return p


class Sim:
    """Full-field FP64 solver.  State after n steps: f_i(x, n) (post-stream)
    and T(x, n).  Arrays are indexed [y, x].  omp: run on the OpenMP build
    (all threads of OMP_NUM_THREADS; bitwise the same results)."""

    def __init__(self, p: OrcParams, rho0: np.ndarray | None = None, rho_uniform: float = 1.0,
                 omp: bool = False):
        self.p = p
        self.Nx, self.Ny = p.Nx, p.Ny
        self._L = lib(omp)
        self.h = self._L.orc_sim_new(C.byref(p))
        if not self.h:
            raise ValueError("invalid oracle grid")
        if rho0 is not None:
            r = np.ascontiguousarray(rho0, dtype=np.float64).reshape(self.Ny, self.Nx)
            self._L.orc_sim_init(self.h, _dp(r), 0.0)
        else:
            self._L.orc_sim_init(self.h, None, rho_uniform)

    def __del__(self):
        h = getattr(self, "h", None)
        L = getattr(self, "_L", None)
        if h and L is not None:
            L.orc_sim_free(h)
            self.h = None

    @property
    def n(self) -> int:
        return self._L.orc_sim_time(self.h)

    @property
    def psi_clamps(self) -> int:
        return self._L.orc_sim_psi_clamps(self.h)

    def step(self, nsteps: int = 1):
        self._L.orc_sim_step(self.h, int(nsteps))

    def set_f(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(9, self.Ny, self.Nx)
        self._L.orc_sim_set_f(self.h, _dp(f))

    def get_f(self) -> np.ndarray:
        f = np.zeros((9, self.Ny, self.Nx))
        self._L.orc_sim_get_f(self.h, _dp(f))
        return f

    def set_T(self, T: np.ndarray):
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(self.Ny, self.Nx)
        self._L.orc_sim_set_T(self.h, _dp(T))

    def set_time(self, n: int):
        self._L.orc_sim_set_time(self.h, int(n))

    def moments(self):
        """(rho, ux, uy, T, Fx, Fy) at the current time level, each [Ny, Nx]."""
        outs = [np.zeros((self.Ny, self.Nx)) for _ in range(6)]
        self._L.orc_sim_moments(self.h, *[_dp(o) for o in outs])
        return tuple(outs)

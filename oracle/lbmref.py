"""ctypes binding of the plain FP64 CPU oracle (lbmref.c).

TEST INFRASTRUCTURE ONLY.  Tests, the smoke check and the benchmark's CPU
baseline use this module to compute what the method gives, independently of
the HIP path.  It takes and returns NumPy float64 arrays: fields are [ny, nx],
populations [9, ny, nx] (x fastest, D2Q9 order of Eq. VelocitySet) and hold
the post-streaming, pre-collision state f(t).
"""
import ctypes
import os

import numpy as np

from . import build as _build

OK = 0
ERR_INVALID_ARG = -1
ERR_DOMAIN = -2


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("tau", ctypes.c_double), ("G", ctypes.c_double),
        ("epsilon", ctypes.c_double), ("sigma", ctypes.c_double),
        ("eos_a", ctypes.c_double), ("eos_b", ctypes.c_double),
        ("eos_c", ctypes.c_double), ("eos_k", ctypes.c_double), ("T", ctypes.c_double),
        ("force_on", ctypes.c_int32), ("m2_trace_alt", ctypes.c_int32),
        ("storage", ctypes.c_int32), ("rho_ref", ctypes.c_double),
        ("collision", ctypes.c_int32),
        ("tau_rho", ctypes.c_double), ("tau_e", ctypes.c_double), ("tau_zeta", ctypes.c_double),
        ("tau_j", ctypes.c_double), ("tau_q", ctypes.c_double),
    ]


class Fault(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("cell", ctypes.c_int64), ("rho", ctypes.c_double)]


class OracleError(RuntimeError):
    def __init__(self, status, fault=None):
        self.status = status
        self.fault = fault
        msg = {ERR_INVALID_ARG: "invalid argument", ERR_DOMAIN: "EOS domain error"}.get(
            status, f"status {status}")
        if fault is not None and status == ERR_DOMAIN:
            msg += f" at step {fault.step}, cell {fault.cell}, rho={fault.rho!r}"
        super().__init__(msg)


_lib = None
_DP = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER(Params)
        lib.lbmref_eos_pressure.argtypes = [P, ctypes.c_double]
        lib.lbmref_eos_pressure.restype = ctypes.c_double
        lib.lbmref_psi.argtypes = [P, ctypes.c_double, _DP]
        lib.lbmref_equilibrium.argtypes = [ctypes.c_double] * 3 + [_DP]
        lib.lbmref_equilibrium.restype = None
        lib.lbmref_guo_source.argtypes = [ctypes.c_double] * 5 + [_DP]
        lib.lbmref_guo_source.restype = None
        lib.lbmref_guo_term.argtypes = [ctypes.c_double] * 4 + [_DP]
        lib.lbmref_guo_term.restype = None
        lib.lbmref_mrt_matrix.argtypes = [_DP]
        lib.lbmref_mrt_matrix.restype = None
        lib.lbmref_mrt_operators.argtypes = [P, _DP, _DP]
        lib.lbmref_psi_moments.argtypes = [ctypes.c_int32, ctypes.c_int32] + [_DP] * 7
        lib.lbmref_psi_moments.restype = None
        lib.lbmref_force.argtypes = [P, _DP, _DP, _DP]
        lib.lbmref_force.restype = None
        lib.lbmref_force_aij.argtypes = [P, _DP, _DP, _DP]
        lib.lbmref_force_aij.restype = None
        lib.lbmref_init.argtypes = [P, _DP, _DP, _DP, _DP]
        lib.lbmref_moments.argtypes = [P, _DP] + [_DP] * 6 + [ctypes.POINTER(Fault)]
        lib.lbmref_step.argtypes = [P, _DP, ctypes.c_int64, ctypes.POINTER(Fault)]
        lib.lbmref_threads.argtypes = []
        lib.lbmref_set_threads.argtypes = [ctypes.c_int]
        lib.lbmref_set_threads.restype = None
        lib.lbmref_quantize.argtypes = [ctypes.c_int32, ctypes.c_double]
        lib.lbmref_quantize.restype = ctypes.c_double
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


STORE_F64, STORE_F32, STORE_F16, STORE_F16_LOCAL = 0, 1, 2, 3


COLL_BGK, COLL_MRT = 0, 1


def make_params(nx, ny, tau=1.0, G=-1.0, epsilon=1.73, sigma=1.0, eos=(1.0, 1.0, 1.0, 1.0),
                T=0.0, force_on=True, m2_trace_alt=False, storage=0, rho_ref=0.0,
                collision=COLL_BGK, mrt=(1.0, 1.0, 1.0, 1.0, 1.0)) -> Params:
    """mrt = (tau_rho, tau_e, tau_zeta, tau_j, tau_q) of Eq. RelaxationMatrix; the
    stress rows relax with tau."""
    a, b, c, k = eos
    return Params(int(nx), int(ny), float(tau), float(G), float(epsilon), float(sigma),
                  float(a), float(b), float(c), float(k), float(T), int(bool(force_on)),
                  int(bool(m2_trace_alt)), int(storage), float(rho_ref), int(collision),
                  *[float(v) for v in mrt])


def quantize(storage, x):
    """Round x to the storage format (1: binary32, 2: binary16; 0: unchanged)."""
    return _load().lbmref_quantize(int(storage), float(x))


def threads() -> int:
    return _load().lbmref_threads()


def set_threads(n: int) -> None:
    """Use n > 0 OpenMP threads in the following calls (timing only: every
    result is independent of the thread count)."""
    _load().lbmref_set_threads(int(n))


def eos_pressure(p: Params, rho: float) -> float:
    return _load().lbmref_eos_pressure(ctypes.byref(p), float(rho))


def psi(p: Params, rho: float) -> float:
    out = ctypes.c_double(0.0)
    st = _load().lbmref_psi(ctypes.byref(p), float(rho), ctypes.byref(out))
    if st != OK:
        raise OracleError(st)
    return out.value


def equilibrium(rho, ux, uy):
    out = np.zeros(9)
    _load().lbmref_equilibrium(float(rho), float(ux), float(uy), _ptr(out))
    return out


def guo_source(tau, ux, uy, Fx, Fy):
    out = np.zeros(9)
    _load().lbmref_guo_source(float(tau), float(ux), float(uy), float(Fx), float(Fy), _ptr(out))
    return out


def guo_term(ux, uy, Fx, Fy):
    out = np.zeros(9)
    _load().lbmref_guo_term(float(ux), float(uy), float(Fx), float(Fy), _ptr(out))
    return out


def mrt_matrix():
    out = np.zeros(81)
    _load().lbmref_mrt_matrix(_ptr(out))
    return out.reshape(9, 9)


def mrt_operators(p: Params):
    """(K, C) = (M^-1 Lambda M, M^-1 (I - Lambda/2) M) of the parameters."""
    K = np.zeros(81)
    C = np.zeros(81)
    st = _load().lbmref_mrt_operators(ctypes.byref(p), _ptr(K), _ptr(C))
    if st != OK:
        raise OracleError(st)
    return K.reshape(9, 9), C.reshape(9, 9)


def psi_moments(psi_field):
    psi_field = np.ascontiguousarray(psi_field, dtype=np.float64)
    ny, nx = psi_field.shape
    outs = [np.empty_like(psi_field) for _ in range(6)]
    _load().lbmref_psi_moments(nx, ny, _ptr(psi_field), *[_ptr(o) for o in outs])
    return dict(zip(["M0", "M1x", "M1y", "M2xx", "M2xy", "M2yy"], outs))


def force(p: Params, psi_field, aij=False):
    psi_field = np.ascontiguousarray(psi_field, dtype=np.float64)
    assert psi_field.shape == (p.ny, p.nx)
    Fx = np.empty_like(psi_field)
    Fy = np.empty_like(psi_field)
    fn = _load().lbmref_force_aij if aij else _load().lbmref_force
    fn(ctypes.byref(p), _ptr(psi_field), _ptr(Fx), _ptr(Fy))
    return Fx, Fy


def init(p: Params, rho0, ux0=None, uy0=None):
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
    assert rho0.shape == (p.ny, p.nx)
    ux0 = None if ux0 is None else np.ascontiguousarray(ux0, dtype=np.float64)
    uy0 = None if uy0 is None else np.ascontiguousarray(uy0, dtype=np.float64)
    f = np.empty((9, p.ny, p.nx))
    st = _load().lbmref_init(ctypes.byref(p), _ptr(rho0), _ptr(ux0), _ptr(uy0), _ptr(f))
    if st != OK:
        raise OracleError(st)
    return f


def moments(p: Params, f):
    """rho, ux, uy, Fx, Fy, psi of the state f(t) (Eqs. FD, DED, IFT, FMD)."""
    assert f.shape == (9, p.ny, p.nx) and f.dtype == np.float64 and f.flags.c_contiguous
    outs = [np.empty((p.ny, p.nx)) for _ in range(6)]
    fault = Fault()
    st = _load().lbmref_moments(ctypes.byref(p), _ptr(f), *[_ptr(o) for o in outs],
                                ctypes.byref(fault))
    if st != OK:
        raise OracleError(st, fault)
    return dict(zip(["rho", "ux", "uy", "Fx", "Fy", "psi"], outs))


def step(p: Params, f, nsteps=1):
    """Advance f in place by nsteps (Eq. TLBE); raises OracleError on a domain fault."""
    assert f.shape == (9, p.ny, p.nx) and f.dtype == np.float64 and f.flags.c_contiguous
    fault = Fault()
    st = _load().lbmref_step(ctypes.byref(p), _ptr(f), int(nsteps), ctypes.byref(fault))
    if st != OK:
        raise OracleError(st, fault)
    return f


def diagnostics(p: Params, f, rho_prev=None):
    """Mass, total momentum sum(rho u), the numerator and denominator of the
    steady-state criterion (Eq. SSC) against rho_prev, and max |u|."""
    m = moments(p, f)
    rho = m["rho"]
    num = float(np.abs(rho - rho_prev).sum()) if rho_prev is not None else 0.0
    return {
        "mass": float(rho.sum()),
        "mom_x": float((rho * m["ux"]).sum()),
        "mom_y": float((rho * m["uy"]).sum()),
        "ssc_num": num,
        "ssc_den": float(np.abs(rho).sum()),
        "umax": float(np.sqrt(m["ux"] ** 2 + m["uy"] ** 2).max()),
    }

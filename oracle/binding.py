"""ctypes binding of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark import
this module.  The HIP product path never does.  Every function here marshals numpy
arrays into the C++ oracle in ``wenozn_oracle.cpp``; no arithmetic of the method
lives in Python.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None

ORC_ZN, ORC_Z, ORC_JS = 0, 1, 2
SYS_ADV, SYS_EULER1, SYS_EULER2 = 0, 1, 2
BC_PERIODIC, BC_TRANSMISSIVE = 0, 1

# The paper's WENO-ZN parameters: A = 10 (Sec. 3, eq:function), square in C,
# exponent 1 on tau8/(IS_k+eps) (eq:new), eps = 1e-40 (reading fixed by the
# critical-point table of Sec. 4.1).
PAPER_A = 10.0
PAPER_EPS = 1e-40
GAMMA = 1.4


class OrcParams(C.Structure):
    _fields_ = [("scheme", C.c_int32), ("p_C", C.c_int32), ("q", C.c_int32),
                ("pad", C.c_int32), ("A", C.c_double), ("eps", C.c_double)]


class OrcStepInfo(C.Structure):
    _fields_ = [("alpha_used", C.c_double * 3), ("alpha_used_y", C.c_double * 3),
                ("dt", C.c_double)]


def params(scheme=ORC_ZN, p_C=2, q=1, A=PAPER_A, eps=PAPER_EPS):
    return OrcParams(scheme, p_C, q, 0, A, eps)


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(path)
        d, i32, i64, p = C.c_double, C.c_int, C.c_int64, C.c_void_p
        L.orc_reconstruct_f64.argtypes = [p, C.POINTER(OrcParams), p]
        L.orc_reconstruct_f128.argtypes = [p, p, C.POINTER(OrcParams), p, p]
        L.orc_rhs_1d_f64.argtypes = [i32, i32, i64, p, p, d, d, C.POINTER(OrcParams), d, d]
        L.orc_rhs_1d_f64.restype = d
        L.orc_rhs_1d_f128.argtypes = [i32, i32, i64, p, p, p, p, d, d, d,
                                      C.POINTER(OrcParams), d, d]
        L.orc_rhs_1d_c128.argtypes = [i32, i32, i64, p, p, d, d, C.POINTER(OrcParams), d, d]
        L.orc_rk3_step_1d_f64.argtypes = [i32, i32, i64, p, d, d, d, p, C.POINTER(OrcParams),
                                          d, d, C.POINTER(OrcStepInfo)]
        L.orc_rk3_run_1d_f64.argtypes = [i32, i32, i64, p, d, d, C.c_int32, p, p,
                                         C.POINTER(OrcParams), d, d, p, p]
        L.orc_rk3_step_1d_c128.argtypes = [i32, i32, i64, p, d, d, p, C.POINTER(OrcParams),
                                           d, d]
        L.orc_rk3_run_1d_c128.argtypes = [i32, i32, i64, p, d, C.c_int32, p, p,
                                          C.POINTER(OrcParams), d, d]
        L.orc_rk3_run_1d_f128.argtypes = [i32, i32, i64, p, p, d, C.c_int32, p, p,
                                          C.POINTER(OrcParams), d, d]
        L.orc_rhs_2d_f64.argtypes = [i32, i32, i64, i64, p, p, d, d, d, d,
                                     C.POINTER(OrcParams), d, p]
        L.orc_rk3_run_2d_f64.argtypes = [i32, i32, i64, i64, p, d, d, d, C.c_int32, p,
                                         C.POINTER(OrcParams), d, p]
        L.orc_rhs_1d_char_f64.argtypes = [i32, i64, p, p, d, p, C.POINTER(OrcParams), d, p]
        L.orc_roe_eigen_f64.argtypes = [p, p, d, p, p]
        L.orc_rhs_2d_sw_f64.argtypes = [i32, i32, i64, i64, p, p, d, d, C.POINTER(OrcParams), d]
        L.orc_sw_split_f64.argtypes = [p, i32, d, p, p]
        L.orc_rk3_run_2d_sw_f64.argtypes = [i32, i32, i64, i64, p, d, d, d, C.c_int32, p,
                                            C.POINTER(OrcParams), d, p]
        L.orc_rk3_run_1d_char_f64.argtypes = [i32, i64, p, d, d, C.c_int32, p,
                                              C.POINTER(OrcParams), d, p, p]
        L.orc_rhs_2d_char_f64.argtypes = [i32, i32, i64, i64, p, p, d, d, p,
                                          C.POINTER(OrcParams), d, p]
        L.orc_roe_eigen_2d_f64.argtypes = [p, p, i32, d, p, p]
        L.orc_rk3_run_2d_char_f64.argtypes = [i32, i32, i64, i64, p, d, d, d, C.c_int32, p,
                                              C.POINTER(OrcParams), d, p]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        _LIB = L
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


RECON_FIELDS = ("IS0", "IS1", "IS2", "tau5", "tau8", "C", "alpha0", "alpha1", "alpha2",
                "omega0", "omega1", "omega2", "q0", "q1", "q2", "fhat")


def reconstruct(f5, prm=None):
    """All intermediate quantities of one reconstruction, fp64, as a dict."""
    prm = prm or params()
    f5 = _f64(f5)
    out = np.zeros(16)
    lib().orc_reconstruct_f64(_ptr(f5), C.byref(prm), _ptr(out))
    return dict(zip(RECON_FIELDS, out))


def reconstruct_f128(f5_hi, f5_lo, prm=None):
    """Same in __float128; returns (hi, lo) dicts."""
    prm = prm or params()
    hi, lo = _f64(f5_hi), _f64(f5_lo)
    oh, ol = np.zeros(16), np.zeros(16)
    lib().orc_reconstruct_f128(_ptr(hi), _ptr(lo), C.byref(prm), _ptr(oh), _ptr(ol))
    return dict(zip(RECON_FIELDS, oh)), dict(zip(RECON_FIELDS, ol))


def rhs_1d(u, dx, sys=SYS_EULER1, bc=BC_TRANSMISSIVE, alpha=-1.0, prm=None, a=1.0,
           gamma=GAMMA):
    """L(U) for a [nvar, n] state; returns (L, alpha_used)."""
    prm = prm or params()
    u = _f64(u)
    n = u.shape[-1]
    out = np.zeros_like(u)
    al = lib().orc_rhs_1d_f64(sys, bc, n, _ptr(u), _ptr(out), dx, alpha, C.byref(prm), a, gamma)
    return out, al


def rhs_1d_f128(u_hi, u_lo, dx_hi, dx_lo, alpha, sys=SYS_ADV, bc=BC_TRANSMISSIVE, prm=None,
                a=1.0, gamma=GAMMA):
    prm = prm or params()
    uh, ul = _f64(u_hi), _f64(u_lo)
    n = uh.shape[-1]
    dh, dl = np.zeros_like(uh), np.zeros_like(uh)
    lib().orc_rhs_1d_f128(sys, bc, n, _ptr(uh), _ptr(ul), _ptr(dh), _ptr(dl), dx_hi, dx_lo,
                          alpha, C.byref(prm), a, gamma)
    return dh, dl


def rhs_1d_complex(u, dx, alpha, sys=SYS_EULER1, bc=BC_PERIODIC, prm=None, a=1.0, gamma=GAMMA):
    prm = prm or params()
    u = np.ascontiguousarray(u, dtype=np.complex128)
    n = u.shape[-1]
    out = np.zeros_like(u)
    lib().orc_rhs_1d_c128(sys, bc, n, _ptr(u), _ptr(out), dx, alpha, C.byref(prm), a, gamma)
    return out


def rk3_step_1d(u, dx, cfl=0.5, dt=-1.0, alpha3=None, sys=SYS_EULER1, bc=BC_TRANSMISSIVE,
                prm=None, a=1.0, gamma=GAMMA):
    """One TVD-RK3 step; returns (u_new, dt, alphas of the three stages)."""
    prm = prm or params()
    u = _f64(u).copy()
    n = u.shape[-1]
    info = OrcStepInfo()
    al = None if alpha3 is None else _f64(alpha3)
    lib().orc_rk3_step_1d_f64(sys, bc, n, _ptr(u), dx, cfl, dt, _ptr(al), C.byref(prm), a,
                              gamma, C.byref(info))
    return u, info.dt, np.array(info.alpha_used[:])


def rk3_run_1d(u, dx, nsteps, cfl=0.5, dt=None, alpha=None, sys=SYS_EULER1,
               bc=BC_TRANSMISSIVE, prm=None, a=1.0, gamma=GAMMA):
    """nsteps TVD-RK3 steps; dt: None (CFL), scalar or [nsteps]; alpha: None or [nsteps, 3].
    Returns (u_final, dt_history, alpha_history[nsteps, 3])."""
    prm = prm or params()
    u = _f64(u).copy()
    n = u.shape[-1]
    if dt is not None:
        dt = _f64(np.broadcast_to(np.asarray(dt, dtype=np.float64), (nsteps,)))
    if alpha is not None:
        alpha = _f64(alpha).reshape(nsteps * 3)
    dt_out = np.zeros(nsteps)
    al_out = np.zeros(nsteps * 3)
    lib().orc_rk3_run_1d_f64(sys, bc, n, _ptr(u), dx, cfl, nsteps, _ptr(dt), _ptr(alpha),
                             C.byref(prm), a, gamma, _ptr(dt_out), _ptr(al_out))
    return u, dt_out, al_out.reshape(nsteps, 3)


def rk3_step_1d_complex(u, dx, dt, alpha3, sys=SYS_EULER1, bc=BC_PERIODIC, prm=None, a=1.0,
                        gamma=GAMMA):
    prm = prm or params()
    u = np.ascontiguousarray(u, dtype=np.complex128).copy()
    n = u.shape[-1]
    al = _f64(alpha3)
    lib().orc_rk3_step_1d_c128(sys, bc, n, _ptr(u), dx, dt, _ptr(al), C.byref(prm), a, gamma)
    return u


def rk3_run_1d_complex(u, dx, dts, alphas, sys=SYS_EULER1, bc=BC_PERIODIC, prm=None, a=1.0,
                       gamma=GAMMA):
    """len(dts) TVD-RK3 steps of a complex state with the frozen schedule dts [nsteps],
    alphas [nsteps, 3] (complex-step directional derivatives of a whole run)."""
    prm = prm or params()
    u = np.ascontiguousarray(u, dtype=np.complex128).copy()
    n = u.shape[-1]
    dts = _f64(dts).reshape(-1)
    al = _f64(alphas).reshape(-1)
    assert al.size == 3 * dts.size
    lib().orc_rk3_run_1d_c128(sys, bc, n, _ptr(u), dx, int(dts.size), _ptr(dts), _ptr(al),
                              C.byref(prm), a, gamma)
    return u


def rk3_run_1d_f128(u_hi, u_lo, dx, dts, alphas, sys=SYS_EULER1, bc=BC_PERIODIC, prm=None,
                    a=1.0, gamma=GAMMA):
    """len(dts) TVD-RK3 steps in __float128 with the frozen schedule dts [nsteps], alphas
    [nsteps, 3]; the state as (hi, lo) pairs.  Returns (hi, lo)."""
    prm = prm or params()
    uh, ul = _f64(u_hi).copy(), _f64(u_lo).copy()
    n = uh.shape[-1]
    dts = _f64(dts).reshape(-1)
    al = _f64(alphas).reshape(-1)
    assert al.size == 3 * dts.size and ul.shape == uh.shape
    lib().orc_rk3_run_1d_f128(sys, bc, n, _ptr(uh), _ptr(ul), dx, int(dts.size), _ptr(dts),
                              _ptr(al), C.byref(prm), a, gamma)
    return uh, ul


def rhs_2d(u, dx, dy, bcx=BC_TRANSMISSIVE, bcy=BC_TRANSMISSIVE, alpha_x=-1.0, alpha_y=-1.0,
           prm=None, gamma=GAMMA):
    """L(U) for a [4, ny, nx] state; returns (L, (alpha_x, alpha_y))."""
    prm = prm or params()
    u = _f64(u)
    ny, nx = u.shape[-2], u.shape[-1]
    out = np.zeros_like(u)
    al = np.zeros(2)
    lib().orc_rhs_2d_f64(bcx, bcy, nx, ny, _ptr(u), _ptr(out), dx, dy, alpha_x, alpha_y,
                         C.byref(prm), gamma, _ptr(al))
    return out, tuple(al)


def rk3_run_2d(u, dx, dy, nsteps, cfl=0.5, dt=None, bcx=BC_TRANSMISSIVE, bcy=BC_TRANSMISSIVE,
               prm=None, gamma=GAMMA):
    prm = prm or params()
    u = _f64(u).copy()
    ny, nx = u.shape[-2], u.shape[-1]
    if dt is not None:
        dt = _f64(np.broadcast_to(np.asarray(dt, dtype=np.float64), (nsteps,)))
    dt_out = np.zeros(nsteps)
    lib().orc_rk3_run_2d_f64(bcx, bcy, nx, ny, _ptr(u), dx, dy, cfl, nsteps, _ptr(dt),
                             C.byref(prm), gamma, _ptr(dt_out))
    return u, dt_out


def rhs_2d_sw(u, dx, dy, bcx=BC_TRANSMISSIVE, bcy=None, prm=None, gamma=GAMMA):
    """2D Euler L(U) with the Steger-Warming splitting, [4, ny, nx]."""
    prm = prm or params()
    bcy = bcx if bcy is None else bcy
    u = _f64(u)
    ny, nx = u.shape[-2], u.shape[-1]
    out = np.zeros_like(u)
    lib().orc_rhs_2d_sw_f64(bcx, bcy, nx, ny, _ptr(u), _ptr(out), dx, dy, C.byref(prm), gamma)
    return out


def sw_split(U, direction, gamma=GAMMA):
    """(F+, F-) of one 2D state along direction 0 (x) or 1 (y)."""
    Fp, Fm = np.zeros(4), np.zeros(4)
    lib().orc_sw_split_f64(_ptr(_f64(U)), int(direction), gamma, _ptr(Fp), _ptr(Fm))
    return Fp, Fm


def rk3_run_2d_sw(u, dx, dy, nsteps, cfl=0.5, bcx=BC_TRANSMISSIVE, bcy=None, dt=None,
                  prm=None, gamma=GAMMA):
    """nsteps TVD-RK3 steps with the Steger-Warming splitting; returns (u, dt[nsteps])."""
    prm = prm or params()
    bcy = bcx if bcy is None else bcy
    u = _f64(u).copy()
    ny, nx = u.shape[-2], u.shape[-1]
    if dt is not None:
        dt = _f64(np.broadcast_to(np.asarray(dt, dtype=np.float64), (nsteps,)))
    dt_out = np.zeros(nsteps)
    lib().orc_rk3_run_2d_sw_f64(bcx, bcy, nx, ny, _ptr(u), dx, dy, cfl, nsteps, _ptr(dt),
                                C.byref(prm), gamma, _ptr(dt_out))
    return u, dt_out


def rhs_1d_char(u, dx, bc=BC_TRANSMISSIVE, alpha3=None, prm=None, gamma=GAMMA):
    """L(U) of 1D Euler with the reconstruction in local characteristic fields; returns
    (L, alpha3_used) with the three per-field LF alphas."""
    prm = prm or params()
    u = _f64(u)
    n = u.shape[-1]
    out = np.zeros_like(u)
    a_in = None if alpha3 is None else _f64(alpha3)
    a_out = np.zeros(3)
    lib().orc_rhs_1d_char_f64(bc, n, _ptr(u), _ptr(out), dx, _ptr(a_in), C.byref(prm), gamma,
                              _ptr(a_out))
    return out, a_out


def roe_eigen(UL, UR, gamma=GAMMA):
    """(R, Lc) at the Roe average of two states (3x3 arrays)."""
    R, Lc = np.zeros(9), np.zeros(9)
    lib().orc_roe_eigen_f64(_ptr(_f64(UL)), _ptr(_f64(UR)), gamma, _ptr(R), _ptr(Lc))
    return R.reshape(3, 3), Lc.reshape(3, 3)


def rk3_run_1d_char(u, dx, nsteps, cfl=0.5, bc=BC_TRANSMISSIVE, prm=None, gamma=GAMMA,
                    dt=None):
    """nsteps TVD-RK3 steps of the characteristic scheme (dt: None for the CFL step, or a
    scalar or [nsteps] of given steps); returns (u, dt[nsteps], alpha[nsteps, 3 stages,
    3 fields])."""
    prm = prm or params()
    u = _f64(u).copy()
    n = u.shape[-1]
    if dt is not None:
        dt = _f64(np.broadcast_to(np.asarray(dt, dtype=np.float64), (nsteps,)))
    dt_out = np.zeros(nsteps)
    al_out = np.zeros(nsteps * 9)
    lib().orc_rk3_run_1d_char_f64(bc, n, _ptr(u), dx, cfl, nsteps, _ptr(dt), C.byref(prm),
                                  gamma, _ptr(dt_out), _ptr(al_out))
    return u, dt_out, al_out.reshape(nsteps, 3, 3)


def num_threads():
    return int(lib().orc_num_threads())


def set_num_threads(n):
    """Thread count of the oracle's per-cell loops (results do not depend on it)."""
    lib().orc_set_num_threads(int(n))


def rhs_2d_char(u, dx, dy, bcx=BC_TRANSMISSIVE, bcy=None, alpha8=None, prm=None, gamma=GAMMA):
    """L(U) of 2D Euler [4, ny, nx] with each sweep's reconstruction in local characteristic
    fields; returns (L, alpha8_used): the per-field alphas of the x sweep, then the y sweep."""
    prm = prm or params()
    bcy = bcx if bcy is None else bcy
    u = _f64(u)
    ny, nx = u.shape[-2], u.shape[-1]
    out = np.zeros_like(u)
    a_in = None if alpha8 is None else _f64(alpha8)
    a_out = np.zeros(8)
    lib().orc_rhs_2d_char_f64(bcx, bcy, nx, ny, _ptr(u), _ptr(out), dx, dy, _ptr(a_in),
                              C.byref(prm), gamma, _ptr(a_out))
    return out, a_out


def roe_eigen_2d(UL, UR, direction, gamma=GAMMA):
    """(R, Lc) of the 2D flux Jacobian along x (direction 0) or y (1) at the Roe average of
    two states (4x4 arrays)."""
    R, Lc = np.zeros(16), np.zeros(16)
    lib().orc_roe_eigen_2d_f64(_ptr(_f64(UL)), _ptr(_f64(UR)), int(direction), gamma, _ptr(R),
                               _ptr(Lc))
    return R.reshape(4, 4), Lc.reshape(4, 4)


def rk3_run_2d_char(u, dx, dy, nsteps, cfl=0.5, bcx=BC_TRANSMISSIVE, bcy=None, dt=None,
                    prm=None, gamma=GAMMA):
    """nsteps TVD-RK3 steps of the 2D characteristic scheme; returns (u, dt[nsteps])."""
    prm = prm or params()
    bcy = bcx if bcy is None else bcy
    u = _f64(u).copy()
    ny, nx = u.shape[-2], u.shape[-1]
    if dt is not None:
        dt = _f64(np.broadcast_to(np.asarray(dt, dtype=np.float64), (nsteps,)))
    dt_out = np.zeros(nsteps)
    lib().orc_rk3_run_2d_char_f64(bcx, bcy, nx, ny, _ptr(u), dx, dy, cfl, nsteps, _ptr(dt),
                                  C.byref(prm), gamma, _ptr(dt_out))
    return u, dt_out

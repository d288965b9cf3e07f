"""PyTorch-facing binding of libwenozn: argument marshalling only.

Every function takes device tensors, checks their dtype, layout and device, and calls the
C ABI of include/wenozn.h on the current torch stream.  All arithmetic of the scheme runs in
the library's HIP kernels; PyTorch provides device memory and streams.
"""
import ctypes as C

import torch

from . import _lib
from ._lib import WznParams, check, lib

SYSTEMS = {"advection": _lib.WZN_ADVECTION, "euler": _lib.WZN_EULER}
BCS = {"periodic": _lib.WZN_PERIODIC, "transmissive": _lib.WZN_TRANSMISSIVE}
SPLITS = {"lf": _lib.WZN_SPLIT_LF, "sw": _lib.WZN_SPLIT_SW}
WEIGHTS = {"zn": _lib.WZN_WEIGHTS_ZN, "z": _lib.WZN_WEIGHTS_Z}


def params(system="euler", bc="transmissive", bc_y=None, adv_speed=1.0, gamma=1.4, A=10.0,
           eps=1e-40, lf_alpha=None, lf_alpha_y=None, dtype="fp64", split="lf", weights="zn",
           debug_nonfinite=False):
    """WENO-ZN parameters; defaults are the paper's (A = 10, eps = 1e-40, gamma = 1.4).
    split: "lf" (global Lax-Friedrichs) or "sw" (Steger-Warming, 2D only); weights: "zn"
    (the paper's) or "z" (WENO-Z, q = 1, the comparison scheme; 1D and reconstruct only);
    debug_nonfinite: scan every output for NaN / Inf and raise (synchronises; debugging only)."""
    p = WznParams()
    lib().wzn_default_params(C.byref(p), SYSTEMS[system])
    p.bc_x = BCS[bc]
    p.bc_y = BCS[bc_y or bc]
    p.adv_speed = adv_speed
    p.gamma = gamma
    p.A = A
    p.eps = eps
    p.lf_alpha_x = -1.0 if lf_alpha is None else float(lf_alpha)
    p.lf_alpha_y = -1.0 if lf_alpha_y is None else float(lf_alpha_y)
    p.dtype = {"fp64": _lib.WZN_FP64, "fp32": _lib.WZN_FP32}[dtype]
    p.flux_split = SPLITS[split]
    p.weights = WEIGHTS[weights]
    p.debug_nonfinite = 1 if debug_nonfinite else 0
    return p


_WS = {}


def workspace(device=None):
    """The per-device workspace tensor (allocated once, reused by every call)."""
    dev = torch.device(device or "cuda")
    if dev.index is None:
        dev = torch.device("cuda", torch.cuda.current_device())
    ws = _WS.get(dev.index)
    if ws is None:
        nbytes = lib().wzn_workspace_bytes(None, 1, 1)
        ws = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
        assert ws.data_ptr() % 256 == 0
        _WS[dev.index] = ws
    return ws


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _check_state(u, nv, name="u", dtype=torch.float64):
    if not isinstance(u, torch.Tensor) or not u.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if u.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, u.dtype))
    if not u.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if u.dim() != 2 or u.shape[0] != nv:
        raise ValueError("%s must have shape [%d, n], got %s" % (name, nv, tuple(u.shape)))


def _nv(p):
    return 1 if p.system == _lib.WZN_ADVECTION else 3


def _dev_f64(x, n, name, device):
    if x is None:
        return None
    if not isinstance(x, torch.Tensor):
        x = torch.as_tensor(x, dtype=torch.float64)
    elif x.dtype != torch.float64:
        # a float32 tensor would silently round the value (dt, alpha) it carries
        raise TypeError("%s must be float64, got %s" % (name, x.dtype))
    x = x.to(device=device).reshape(-1).contiguous()
    if x.numel() != n:
        raise ValueError("%s must have %d entries" % (name, n))
    return x


def reconstruct(f5, prm=None, out=None):
    """fhat[m] from the point values f5[5, m] = (f_{i-2}, ..., f_{i+2}) of m stencils."""
    prm = prm or params()
    if not isinstance(f5, torch.Tensor) or not f5.is_cuda or f5.dtype != torch.float64:
        raise TypeError("f5 must be a float64 CUDA (HIP) tensor")
    if f5.dim() != 2 or f5.shape[0] != 5 or not f5.is_contiguous():
        raise ValueError("f5 must be a contiguous [5, m] tensor")
    m = f5.shape[1]
    out = torch.empty(m, dtype=torch.float64, device=f5.device) if out is None else out
    if out.numel() != m or out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor of m elements")
    check(lib().wzn_reconstruct(C.byref(prm), _ptr(f5), _ptr(out), m, _stream()))
    return out


def rhs_1d(u, dx, prm=None, out=None):
    """L(u) for u[nvar, n] (nvar = 1 advection, 3 Euler)."""
    prm = prm or params()
    _check_state(u, _nv(prm))
    out = torch.empty_like(u) if out is None else out
    _check_state(out, _nv(prm), "out")
    check(lib().wzn_rhs_1d(C.byref(prm), _ptr(u), _ptr(out), u.shape[1], float(dx),
                           _ptr(workspace(u.device)), _stream()))
    return out


def speed_max_1d(u, prm=None, out=None):
    """Device tensor [1]: max(|u| + c) over the cells of 1D Euler u [3, n]."""
    prm = prm or params()
    _check_state(u, 3)
    out = torch.empty(1, dtype=torch.float64, device=u.device) if out is None else out
    check(lib().wzn_speed_max_1d(C.byref(prm), _ptr(u), u.shape[1], _ptr(out),
                                 _ptr(workspace(u.device)), _stream()))
    return out


def rhs_1d_slab(u, ghost_lo, ghost_hi, dx, alpha, prm=None, out=None):
    """L(u) for a slab u [3, n] of a longer 1D Euler row with ghost cells ghost_lo / ghost_hi
    [3, 3] (the three cells before / after it) and the global alpha of the whole row."""
    prm = prm or params()
    _check_state(u, 3)
    for g, name in ((ghost_lo, "ghost_lo"), (ghost_hi, "ghost_hi")):
        if (not isinstance(g, torch.Tensor) or g.dtype != torch.float64 or g.device != u.device
                or not g.is_contiguous() or tuple(g.shape) != (3, 3)):
            raise ValueError("%s must be a contiguous float64 [3, 3] tensor on u's device" % name)
    al = _dev_f64(alpha, 1, "alpha", u.device)
    out = torch.empty_like(u) if out is None else out
    _check_state(out, 3, "out")
    check(lib().wzn_rhs_1d_slab(C.byref(prm), _ptr(u), _ptr(ghost_lo), _ptr(ghost_hi),
                                _ptr(out), u.shape[1], float(dx), _ptr(al),
                                _ptr(workspace(u.device)), _stream()))
    return out


def rk3_run_1d(u, dx, nsteps, cfl=0.5, prm=None, dt=None, alpha=None, stage=None, record=False):
    """Advance u[nvar, n] in place by nsteps TVD-RK3 steps.

    dt: None (CFL from U^n) or [nsteps] step sizes; alpha: None or [nsteps, 3] frozen LF
    alphas.  With record=True returns (dt_history[nsteps], alpha_history[nsteps, 3]) as
    device tensors."""
    prm = prm or params()
    _check_state(u, _nv(prm))
    n = u.shape[1]
    if stage is None:
        stage = torch.empty((2,) + tuple(u.shape), dtype=u.dtype, device=u.device)
    if stage.numel() < 2 * u.numel() or not stage.is_contiguous() or stage.dtype != u.dtype:
        raise ValueError("stage must be a contiguous fp64 tensor of 2 * u.numel() elements")
    if dt is None:
        dt_t = None
    elif isinstance(dt, (int, float)):
        dt_t = torch.full((nsteps,), float(dt), dtype=torch.float64, device=u.device)
    else:
        dt_t = _dev_f64(dt, nsteps, "dt", u.device)
    al_t = _dev_f64(alpha, 3 * nsteps, "alpha", u.device)
    dt_o = torch.empty(nsteps, dtype=torch.float64, device=u.device) if record else None
    al_o = torch.empty(3 * nsteps, dtype=torch.float64, device=u.device) if record else None
    check(lib().wzn_rk3_run_1d(C.byref(prm), _ptr(u), _ptr(stage), n, float(dx), float(cfl),
                               int(nsteps), _ptr(dt_t), _ptr(al_t), _ptr(dt_o), _ptr(al_o),
                               _ptr(workspace(u.device)), _stream()))
    if record:
        return dt_o, al_o.view(nsteps, 3)
    return None


def rk3_step_1d(u, dx, cfl=0.5, prm=None, dt=None, stage=None):
    """One TVD-RK3 step in place; returns the dt used (device tensor of 1 element)."""
    prm = prm or params()
    _check_state(u, _nv(prm))
    if stage is None:
        stage = torch.empty((2,) + tuple(u.shape), dtype=u.dtype, device=u.device)
    dt_t = None if dt is None else torch.full((1,), float(dt), dtype=torch.float64,
                                              device=u.device)
    dt_o = torch.empty(1, dtype=torch.float64, device=u.device)
    check(lib().wzn_rk3_step_1d(C.byref(prm), _ptr(u), _ptr(stage), u.shape[1], float(dx),
                                float(cfl), _ptr(dt_t), _ptr(dt_o), _ptr(workspace(u.device)),
                                _stream()))
    return dt_o


def rhs_1d_char(u, dx, prm=None, alpha3=None, out=None):
    """L(u) for 1D Euler u[3, n] with the reconstruction in local characteristic fields.
    alpha3: None (reduced from u, or prm.lf_alpha_x for all three if >= 0) or 3 frozen
    per-field alphas."""
    prm = prm or params()
    _check_state(u, 3)
    out = torch.empty_like(u) if out is None else out
    _check_state(out, 3, "out")
    al = _dev_f64(alpha3, 3, "alpha3", u.device)
    check(lib().wzn_rhs_1d_char(C.byref(prm), _ptr(u), _ptr(out), u.shape[1], float(dx),
                                _ptr(al), _ptr(workspace(u.device)), _stream()))
    return out


def rk3_run_1d_char(u, dx, nsteps, cfl=0.5, prm=None, dt=None, alpha=None, stage=None,
                    record=False):
    """Advance 1D Euler u[3, n] in place by nsteps TVD-RK3 steps of the characteristic scheme.

    dt: None (CFL from U^n) or [nsteps]; alpha: None or [nsteps, 3, 3] frozen per-stage,
    per-field alphas.  With record=True returns (dt[nsteps], alpha[nsteps, 3, 3])."""
    prm = prm or params()
    _check_state(u, 3)
    n = u.shape[1]
    if stage is None:
        stage = torch.empty((2,) + tuple(u.shape), dtype=u.dtype, device=u.device)
    if stage.numel() < 2 * u.numel() or not stage.is_contiguous() or stage.dtype != u.dtype:
        raise ValueError("stage must be a contiguous fp64 tensor of 2 * u.numel() elements")
    if dt is None:
        dt_t = None
    elif isinstance(dt, (int, float)):
        dt_t = torch.full((nsteps,), float(dt), dtype=torch.float64, device=u.device)
    else:
        dt_t = _dev_f64(dt, nsteps, "dt", u.device)
    al_t = _dev_f64(alpha, 9 * nsteps, "alpha", u.device)
    dt_o = torch.empty(nsteps, dtype=torch.float64, device=u.device) if record else None
    al_o = torch.empty(9 * nsteps, dtype=torch.float64, device=u.device) if record else None
    check(lib().wzn_rk3_run_1d_char(C.byref(prm), _ptr(u), _ptr(stage), n, float(dx),
                                    float(cfl), int(nsteps), _ptr(dt_t), _ptr(al_t),
                                    _ptr(dt_o), _ptr(al_o), _ptr(workspace(u.device)),
                                    _stream()))
    if record:
        return dt_o, al_o.view(nsteps, 3, 3)
    return None


def _check_state_2d(u, name="u"):
    if not isinstance(u, torch.Tensor) or not u.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if u.dtype not in (torch.float64, torch.float32):
        raise TypeError("%s must be float64 or float32" % name)
    if not u.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if u.dim() != 3 or u.shape[0] != 4:
        raise ValueError("%s must have shape [4, ny, nx], got %s" % (name, tuple(u.shape)))


def _params_2d(prm, u):
    prm = prm or params("euler", eps=1e-30 if u.dtype == torch.float32 else 1e-40)
    want = _lib.WZN_FP32 if u.dtype == torch.float32 else _lib.WZN_FP64
    if prm.dtype != want:
        raise ValueError("params dtype does not match the tensor dtype")
    return prm


def rhs_2d(u, dx, dy, prm=None, out=None):
    """L(u) for u[4, ny, nx] (fp64 or fp32, with matching params dtype)."""
    _check_state_2d(u)
    prm = _params_2d(prm, u)
    out = torch.empty_like(u) if out is None else out
    _check_state_2d(out, "out")
    check(lib().wzn_rhs_2d(C.byref(prm), _ptr(u), _ptr(out), u.shape[2], u.shape[1], float(dx),
                           float(dy), _ptr(workspace(u.device)), _stream()))
    return out


def speed_max_2d(u, prm=None, out=None):
    """Device tensor [2]: max(|u| + c), max(|v| + c) over the cells of u [4, ny, nx]."""
    prm = _params_2d(prm, u)
    _check_state_2d(u)
    out = torch.empty(2, dtype=torch.float64, device=u.device) if out is None else out
    check(lib().wzn_speed_max_2d(C.byref(prm), _ptr(u), u.shape[2], u.shape[1], _ptr(out),
                                 _ptr(workspace(u.device)), _stream()))
    return out


def rhs_2d_strip(u, ghost_lo, ghost_hi, dx, dy, alpha2=None, prm=None, out=None):
    """L(u) for a strip u [4, ny, nx] of a larger grid with ghost rows ghost_lo / ghost_hi
    [4, 3, nx] (the three rows below / above it) and the global alphas alpha2 = (alpha_x,
    alpha_y) of the whole grid (device tensor or sequence; Lax-Friedrichs only)."""
    prm = _params_2d(prm, u)
    _check_state_2d(u)
    nx = u.shape[2]
    for g, name in ((ghost_lo, "ghost_lo"), (ghost_hi, "ghost_hi")):
        if (not isinstance(g, torch.Tensor) or g.dtype != u.dtype or g.device != u.device
                or not g.is_contiguous() or tuple(g.shape) != (4, 3, nx)):
            raise ValueError("%s must be a contiguous [4, 3, nx] tensor like u" % name)
    al = _dev_f64(alpha2, 2, "alpha2", u.device)
    out = torch.empty_like(u) if out is None else out
    _check_state_2d(out, "out")
    check(lib().wzn_rhs_2d_strip(C.byref(prm), _ptr(u), _ptr(ghost_lo), _ptr(ghost_hi),
                                 _ptr(out), nx, u.shape[1], float(dx), float(dy), _ptr(al),
                                 _ptr(workspace(u.device)), _stream()))
    return out


def rk3_run_2d(u, dx, dy, nsteps, cfl=0.5, prm=None, dt=None, stage=None, record=False):
    """Advance u[4, ny, nx] in place by nsteps TVD-RK3 steps; record=True returns the dt
    history (device tensor [nsteps])."""
    _check_state_2d(u)
    prm = _params_2d(prm, u)
    if stage is None:
        stage = torch.empty((2,) + tuple(u.shape), dtype=u.dtype, device=u.device)
    if stage.numel() < 2 * u.numel() or not stage.is_contiguous() or stage.dtype != u.dtype:
        raise ValueError("stage must be a contiguous tensor of 2 * u.numel() elements")
    if dt is None:
        dt_t = None
    elif isinstance(dt, (int, float)):
        dt_t = torch.full((nsteps,), float(dt), dtype=torch.float64, device=u.device)
    else:
        dt_t = _dev_f64(dt, nsteps, "dt", u.device)
    dt_o = torch.empty(nsteps, dtype=torch.float64, device=u.device) if record else None
    check(lib().wzn_rk3_run_2d(C.byref(prm), _ptr(u), _ptr(stage), u.shape[2], u.shape[1],
                               float(dx), float(dy), float(cfl), int(nsteps), _ptr(dt_t),
                               _ptr(dt_o), _ptr(workspace(u.device)), _stream()))
    return dt_o


def _char2d_work(u, work):
    need = lib().wzn_char2d_work_doubles(u.shape[2], u.shape[1])
    if work is None:
        return torch.empty(need, dtype=torch.float64, device=u.device)
    if (work.dtype != torch.float64 or work.device != u.device or not work.is_contiguous()
            or work.numel() < need):
        raise ValueError("work must be a contiguous fp64 tensor of %d elements" % need)
    return work


def rhs_2d_char(u, dx, dy, prm=None, alpha8=None, out=None, work=None):
    """L(u) for u[4, ny, nx] (fp64) with each sweep's reconstruction in local characteristic
    fields.  alpha8: None (reduced from u) or 8 frozen alphas (x sweep's four fields, then the
    y sweep's) as a float64 tensor or sequence."""
    _check_state_2d(u)
    prm = _params_2d(prm, u)
    al = _dev_f64(alpha8, 8, "alpha8", u.device)
    out = torch.empty_like(u) if out is None else out
    _check_state_2d(out, "out")
    work = _char2d_work(u, work)
    check(lib().wzn_rhs_2d_char(C.byref(prm), _ptr(u), _ptr(out), _ptr(work), u.shape[2],
                                u.shape[1], float(dx), float(dy), _ptr(al),
                                _ptr(workspace(u.device)), _stream()))
    return out


def rk3_run_2d_char(u, dx, dy, nsteps, cfl=0.5, prm=None, dt=None, stage=None, work=None,
                    record=False):
    """Advance u[4, ny, nx] (fp64) in place by nsteps TVD-RK3 steps of the characteristic
    scheme; record=True returns the dt history (device tensor [nsteps])."""
    _check_state_2d(u)
    prm = _params_2d(prm, u)
    if stage is None:
        stage = torch.empty((2,) + tuple(u.shape), dtype=u.dtype, device=u.device)
    if stage.numel() < 2 * u.numel() or not stage.is_contiguous() or stage.dtype != u.dtype:
        raise ValueError("stage must be a contiguous tensor of 2 * u.numel() elements")
    work = _char2d_work(u, work)
    if dt is None:
        dt_t = None
    elif isinstance(dt, (int, float)):
        dt_t = torch.full((nsteps,), float(dt), dtype=torch.float64, device=u.device)
    else:
        dt_t = _dev_f64(dt, nsteps, "dt", u.device)
    dt_o = torch.empty(nsteps, dtype=torch.float64, device=u.device) if record else None
    check(lib().wzn_rk3_run_2d_char(C.byref(prm), _ptr(u), _ptr(stage), _ptr(work), u.shape[2],
                                    u.shape[1], float(dx), float(dy), float(cfl), int(nsteps),
                                    _ptr(dt_t), _ptr(dt_o), _ptr(workspace(u.device)),
                                    _stream()))
    return dt_o


def batch_tuning(nt=128, k=2, blocks_per_cu=0, layout=0):
    return _lib.WznBatchTuning(int(nt), int(k), int(blocks_per_cu), int(layout))


def lpt_order(lengths, device="cuda"):
    """Longest-first processing order of the instances (balances the persistent launch)."""
    lengths = torch.as_tensor(lengths).cpu()
    order = torch.argsort(lengths, descending=True, stable=True).to(torch.int32)
    return order.to(device)


def batched_rk3_run_1d(u, offsets, dx, nsteps, cfl=0.5, prm=None, order=None, tuning=None,
                       stage=None, record=False):
    """Advance every instance of the concatenated state u[3, total] by nsteps TVD-RK3 steps
    in one persistent launch.  offsets: device int64 [batch + 1]; dx: device fp64 [batch];
    order: device int32 [batch] or None.  record=True returns dt history [batch, nsteps]."""
    prm = prm or params("euler", bc="transmissive")
    _check_state(u, 3)
    total = u.shape[1]
    if offsets.dtype != torch.int64 or not offsets.is_cuda or not offsets.is_contiguous():
        raise TypeError("offsets must be a contiguous CUDA int64 tensor")
    batch = offsets.numel() - 1
    if dx.dtype != torch.float64 or not dx.is_cuda or dx.numel() != batch:
        raise TypeError("dx must be a CUDA float64 tensor of batch entries")
    if order is not None and (order.dtype != torch.int32 or not order.is_cuda or
                              order.numel() != batch):
        raise TypeError("order must be a CUDA int32 tensor of batch entries")
    if not torch.cuda.is_current_stream_capturing():
        # overlapping instances or a repeated order entry would make two workgroups race on
        # the same cells; the kernel only skips entries that are out of range.  (Under graph
        # capture the check, which reads back to the host, is left to the caller.)
        if batch > 0 and (int(offsets[0]) < 0 or int(offsets[-1]) != total or
                          bool((offsets[1:] < offsets[:-1]).any())):
            raise ValueError("offsets must be non-decreasing from >= 0 to u.shape[1]")
        if order is not None and not torch.equal(
                torch.sort(order.long())[0], torch.arange(batch, device=order.device)):
            raise ValueError("order must be a permutation of 0 .. batch-1")
    if stage is None:
        stage = torch.empty((2, 3, total), dtype=torch.float64, device=u.device)
    if stage.numel() < 2 * u.numel() or not stage.is_contiguous():
        raise ValueError("stage must be a contiguous fp64 tensor of 2 * u.numel() elements")
    dt_o = torch.empty((batch, nsteps), dtype=torch.float64, device=u.device) if record else None
    tn = tuning if tuning is not None else None
    check(lib().wzn_batched_rk3_run_1d(C.byref(prm), _ptr(u), _ptr(stage), total, _ptr(offsets),
                                       _ptr(dx), _ptr(order), int(batch), int(nsteps),
                                       float(cfl), C.byref(tn) if tn is not None else None,
                                       _ptr(dt_o), _ptr(workspace(u.device)), _stream()))
    return dt_o


def rhs_1d_vjp(u, mu, dx, prm=None, out=None):
    """J(u)^T mu for the 1D Euler right-hand side, alpha frozen (prm.lf_alpha_x if >= 0, else
    max(|u| + c) of u held constant)."""
    prm = prm or params("euler")
    _check_state(u, 3)
    _check_state(mu, 3, "mu")
    out = torch.empty_like(u) if out is None else out
    check(lib().wzn_rhs_1d_vjp(C.byref(prm), _ptr(u), _ptr(mu), _ptr(out), u.shape[1], float(dx),
                               _ptr(workspace(u.device)), _stream()))
    return out


def rk3_step_1d_vjp(stages, lam_next, dt, alpha3, dx, prm=None, out=None, scratch=None):
    """(dU^{n+1}/dU^n)^T lam_next for one TVD-RK3 step with frozen dt and stage alphas.
    stages: [3, 3, n] (U^n, U1, U2); dt: device tensor (1 element); alpha3: device [3]."""
    prm = prm or params("euler")
    if stages.dim() != 3 or stages.shape[0] != 3 or not stages.is_contiguous():
        raise ValueError("stages must be a contiguous [3, 3, n] tensor")
    _check_state(lam_next, 3, "lam_next")
    n = lam_next.shape[1]
    out = torch.empty_like(lam_next) if out is None else out
    scratch = torch.empty((3, 3, n), dtype=torch.float64, device=lam_next.device) \
        if scratch is None else scratch
    check(lib().wzn_rk3_step_1d_vjp(C.byref(prm), _ptr(stages), _ptr(lam_next), _ptr(out),
                                    _ptr(scratch), n, float(dx), _ptr(dt), _ptr(alpha3),
                                    _ptr(workspace(lam_next.device)), _stream()))
    return out

"""Discrete adjoint of a 1D Euler WENO-ZN TVD-RK3 run with checkpointed recomputation.

The forward pass runs the fused stage kernels, records the dt of every step and the
Lax-Friedrichs alpha of every stage, and keeps the state every `ckpt_every` steps.  The
backward pass walks the segments in reverse: it recomputes the stage states of a segment from
its checkpoint with the recorded (frozen) schedule, then applies the hand-written
vector-Jacobian kernels of the TVD-RK3 step in reverse order.  The gradient is that of the
forward map with dt and alphas held at their recorded values.
"""
import torch

from . import api


def forward_checkpointed(U0, dx, nsteps, cfl=0.5, prm=None, ckpt_every=20):
    """Returns (U_T, dt[nsteps], alpha[nsteps, 3], checkpoints).  checkpoints[k] is the state
    after k * ckpt_every steps (k = 0 .. number of segments - 1)."""
    prm = prm or api.params("euler", bc="periodic")
    U = U0.clone()
    stage = torch.empty((2,) + tuple(U.shape), dtype=U.dtype, device=U.device)
    dts = torch.empty(nsteps, dtype=torch.float64, device=U.device)
    als = torch.empty((nsteps, 3), dtype=torch.float64, device=U.device)
    ckpts = []
    t = 0
    while t < nsteps:
        steps = min(ckpt_every, nsteps - t)
        ckpts.append(U.clone())
        d, a = api.rk3_run_1d(U, dx, steps, cfl=cfl, prm=prm, stage=stage, record=True)
        dts[t:t + steps].copy_(d)
        als[t:t + steps].copy_(a)
        t += steps
    return U, dts, als, ckpts


def run_frozen(U0, dx, dts, als, prm=None):
    """Forward run with a recorded schedule (for finite-difference checks)."""
    prm = prm or api.params("euler", bc="periodic")
    U = U0.clone()
    api.rk3_run_1d(U, dx, dts.numel(), dt=dts, alpha=als, prm=prm)
    return U


def backward_checkpointed(lamT, dx, dts, als, ckpts, ckpt_every=20, prm=None, work=None):
    """lam_0 = (dU_T/dU_0)^T lam_T with the frozen schedule: one library call that enqueues
    the recomputation of every segment and the step adjoints in reverse."""
    import ctypes as C
    from ._lib import check, lib
    prm = prm or api.params("euler", bc="periodic")
    nsteps = dts.numel()
    n = lamT.shape[1]
    ck = ckpts if isinstance(ckpts, torch.Tensor) else torch.stack(list(ckpts))
    ck = ck.contiguous()
    lam = lamT.clone().contiguous()
    need = lib().wzn_rk3_adjoint_1d_work_doubles(n, ckpt_every)
    if work is None or work.numel() < need:
        work = torch.empty(need, dtype=torch.float64, device=lamT.device)
    check(lib().wzn_rk3_adjoint_1d(C.byref(prm), api._ptr(ck), int(nsteps), int(ckpt_every),
                                   api._ptr(dts.contiguous()), api._ptr(als.contiguous()),
                                   api._ptr(lam), api._ptr(work), n, float(dx),
                                   api._ptr(api.workspace(lamT.device)), api._stream()))
    return lam


class CapturedAdjoint:
    """The checkpointed forward run and the adjoint pass of one problem shape, each captured
    once in a HIP graph and replayed per evaluation, so that a gradient costs the GPU work
    only, not one host launch per kernel (at N = 65536 a stage kernel runs for about as long
    as its launch takes).  Inputs are copied into the captured buffers:

        cap = CapturedAdjoint(U0, dx, nsteps)
        UT = cap.forward(U0_new)      # U_T; cap.dts, cap.als hold the recorded schedule
        lam0 = cap.backward(lamT)     # dJ/dU_0 for dJ/dU_T = lamT, with that schedule

    The returned tensors are the graphs' own buffers and are overwritten by the next replay.
    """

    def __init__(self, U0, dx, nsteps, cfl=0.5, prm=None, ckpt_every=20):
        prm = prm or api.params("euler", bc="periodic")
        self.U0 = U0.detach().clone().contiguous()
        self.lamT = torch.zeros_like(self.U0)
        # an eager pass first: it allocates the library workspace outside the graphs
        UT, dts, als, ckpts = forward_checkpointed(self.U0, dx, nsteps, cfl, prm, ckpt_every)
        backward_checkpointed(self.lamT, dx, dts, als, ckpts, ckpt_every, prm)
        torch.cuda.synchronize()
        self.g_fwd = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.g_fwd):
            self.UT, self.dts, self.als, ck = forward_checkpointed(self.U0, dx, nsteps, cfl,
                                                                   prm, ckpt_every)
            self.ckpts = torch.stack(ck)
        self.g_bwd = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.g_bwd):
            self.lam0 = backward_checkpointed(self.lamT, dx, self.dts, self.als, self.ckpts,
                                              ckpt_every, prm)

    def forward(self, U0=None):
        if U0 is not None:
            self.U0.copy_(U0)
        self.g_fwd.replay()
        return self.UT

    def backward(self, lamT):
        self.lamT.copy_(lamT)
        self.g_bwd.replay()
        return self.lam0


class WenoZNRK3(torch.autograd.Function):
    """U_T = RK3^nsteps(U_0) with WENO-ZN right-hand sides; backward = discrete adjoint with
    checkpointed recomputation (dt and alphas frozen at the forward's values)."""

    @staticmethod
    def forward(ctx, U0, dx, nsteps, cfl, ckpt_every, bc):
        prm = api.params("euler", bc=bc)
        UT, dts, als, ckpts = forward_checkpointed(U0.detach().contiguous(), dx, nsteps, cfl,
                                                   prm, ckpt_every)
        ctx.save_for_backward(dts, als, *ckpts)
        ctx.cfg = (dx, ckpt_every, bc)
        return UT

    @staticmethod
    def backward(ctx, gUT):
        dts, als, *ckpts = ctx.saved_tensors
        dx, ckpt_every, bc = ctx.cfg
        lam0 = backward_checkpointed(gUT.contiguous(), dx, dts, als, ckpts, ckpt_every,
                                     api.params("euler", bc=bc))
        return lam0, None, None, None, None, None

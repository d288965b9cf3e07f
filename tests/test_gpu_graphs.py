"""Runs captured in a HIP graph (torch.cuda.CUDAGraph), as the benchmark launches them: every
replay, with the program's own eager work and synchronisations between the replays, equals
the eager run bit for bit.  The library clears its reduction slots and queue counter with a
kernel, never with a memset node."""
import numpy as np
import pytest

from paper_2004_07954_amd import inputs as I

pytestmark = pytest.mark.gpu

REPLAYS = 3


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2004_07954_amd import api
    return api


def note(*args):
    print("[gpu-case]", *args, flush=True)


def _replays_match(run, u, u0, ref, side):
    """Capture run(u) once, then replay it REPLAYS times from u0; every replay must equal
    `ref`.  `side` is eager work run between the replays."""
    import torch
    g = torch.cuda.CUDAGraph()
    u.copy_(u0)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        run(u)
    for r in range(REPLAYS):
        u.copy_(u0)
        side()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(u, ref), "replay %d differs from the eager run" % r
    del g


def test_graph_rk3_run_1d(api):
    import torch
    note("graph: rk3_run_1d, n = 4099, 20 steps")
    u0, dx = I.shu_osher_like(4099)
    u0 = torch.tensor(u0, dtype=torch.float64, device="cuda")
    stage = torch.empty((2,) + tuple(u0.shape), dtype=torch.float64, device="cuda")
    u = u0.clone()
    api.rk3_run_1d(u, dx, 20, cfl=0.5, stage=stage)
    ref = u.clone()
    other = torch.tensor(I.random_smooth_1d(1000, seed=3), dtype=torch.float64, device="cuda")
    _replays_match(lambda t: api.rk3_run_1d(t, dx, 20, cfl=0.5, stage=stage), u, u0, ref,
                   lambda: api.rhs_1d(other, 0.01))


def test_graph_rk3_run_2d(api):
    import torch
    for split in ("lf", "sw"):
        note("graph: rk3_run_2d, 200 x 130, 5 steps,", split)
        u0, dx, dy = I.riemann_2d(2, 200)
        u0 = torch.tensor(u0[:, :130, :], dtype=torch.float64, device="cuda").contiguous()
        prm = api.params("euler", split=split)
        stage = torch.empty((2,) + tuple(u0.shape), dtype=torch.float64, device="cuda")
        u = u0.clone()
        api.rk3_run_2d(u, dx, dy, 5, prm=prm, stage=stage)
        ref = u.clone()
        other = torch.tensor(I.random_smooth_1d(500, seed=4), dtype=torch.float64,
                             device="cuda")
        _replays_match(lambda t: api.rk3_run_2d(t, dx, dy, 5, prm=prm, stage=stage), u, u0,
                       ref, lambda: api.rk3_run_1d(other, 0.01, 1))


def test_graph_rk3_run_2d_char(api):
    import torch
    note("graph: rk3_run_2d_char, 150 x 110, 5 steps")
    u0, dx, dy = I.riemann_2d(2, 150)
    u0 = torch.tensor(u0[:, :110, :], dtype=torch.float64, device="cuda").contiguous()
    stage = torch.empty((2,) + tuple(u0.shape), dtype=torch.float64, device="cuda")
    work = torch.empty(12 * u0[0].numel(), dtype=torch.float64, device="cuda")
    u = u0.clone()
    api.rk3_run_2d_char(u, dx, dy, 5, stage=stage, work=work)
    ref = u.clone()
    other = torch.tensor(I.random_smooth_2d(40, 30, seed=5), dtype=torch.float64, device="cuda")
    _replays_match(lambda t: api.rk3_run_2d_char(t, dx, dy, 5, stage=stage, work=work), u, u0,
                   ref, lambda: api.rhs_2d_char(other, 0.01, 0.01))


def test_graph_batched(api):
    import torch
    note("graph: batched_rk3_run_1d, 96 instances, 10 steps")
    U, offs, dx = I.shock_tube_batch(96, seed=12, nmin=256, nmax=3000)
    U0 = torch.tensor(U, dtype=torch.float64, device="cuda")
    offg = torch.tensor(offs, dtype=torch.int64, device="cuda")
    dxg = torch.tensor(dx, dtype=torch.float64, device="cuda")
    order = api.lpt_order(np.diff(offs))
    stage = torch.empty((2, 3, U.shape[1]), dtype=torch.float64, device="cuda")
    for tn in (api.batch_tuning(128, 2, 0, 0), api.batch_tuning(256, 2, 0, 1)):
        u = U0.clone()
        api.batched_rk3_run_1d(u, offg, dxg, 10, order=order, tuning=tn, stage=stage)
        ref = u.clone()
        assert torch.isfinite(ref).all()
        _replays_match(lambda t: api.batched_rk3_run_1d(t, offg, dxg, 10, order=order,
                                                        tuning=tn, stage=stage),
                       u, U0, ref, lambda: torch.cuda.synchronize())


def test_graph_adjoint(api):
    """The captured checkpointed forward and adjoint pass equal the eager ones bit for bit, on
    replays with new initial states and new cotangents."""
    import torch
    from paper_2004_07954_amd import adjoint
    note("graph: checkpointed forward + adjoint, n = 4096, 40 steps, checkpoints every 10")
    n, nsteps, ck = 4096, 40, 10
    u0, _, dx = I.adjoint_case(n=n, seed=5)
    U0 = torch.tensor(u0, dtype=torch.float64, device="cuda")
    prm = api.params("euler", bc="periodic")
    cap = adjoint.CapturedAdjoint(U0, dx, nsteps, 0.5, prm, ck)
    gen = torch.Generator(device="cuda").manual_seed(0)
    for r in range(REPLAYS):
        Ur = U0 * (1.0 + 0.01 * r)
        lamT = torch.randn(U0.shape, generator=gen, dtype=torch.float64, device="cuda")
        UT, dts, als, ckpts = adjoint.forward_checkpointed(Ur, dx, nsteps, 0.5, prm, ck)
        lam0 = adjoint.backward_checkpointed(lamT, dx, dts, als, ckpts, ck, prm)
        torch.cuda.synchronize()
        assert torch.equal(cap.forward(Ur), UT), r
        assert torch.equal(cap.dts, dts) and torch.equal(cap.als, als), r
        assert torch.equal(cap.backward(lamT), lam0), r
        torch.cuda.synchronize()

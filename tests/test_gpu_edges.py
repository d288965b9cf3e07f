"""Empty and degenerate inputs through the C ABI on the GPU.

A run of zero steps leaves the state untouched bit for bit on every run entry point; an empty
reconstruction (m = 0) enqueues nothing; the batched launch leaves instances shorter than six
cells (and empty ones) untouched, as include/wenozn.h states, while every other instance of
the same launch advances exactly as its one-instance run does."""
import numpy as np
import pytest

from paper_2004_07954_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2004_07954_amd import api
    return api


def note(*args):
    print("[gpu-case]", *args, flush=True)


def dev(a, dtype=None):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device="cuda")


def test_zero_step_runs_leave_state_unchanged(api):
    import torch
    note("zero-step runs")
    u0, dx = I.shu_osher_like(1000)
    u = dev(u0)
    dts, als = api.rk3_run_1d(u, dx, 0, record=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u.cpu().numpy(), u0)
    assert dts.numel() == 0 and als.numel() == 0

    a0, adx = I.advection_smooth(200)[:2]
    ua = dev(np.asarray(a0).reshape(1, -1))
    api.rk3_run_1d(ua, adx, 0, prm=api.params("advection", bc="periodic"))
    np.testing.assert_array_equal(ua.cpu().numpy().ravel(), np.asarray(a0).ravel())

    u = dev(u0)
    api.rk3_run_1d_char(u, dx, 0)
    np.testing.assert_array_equal(u.cpu().numpy(), u0)

    v0, dx2, dy2 = I.riemann_2d(2, 64)
    v = dev(v0)
    api.rk3_run_2d(v, dx2, dy2, 0)
    np.testing.assert_array_equal(v.cpu().numpy(), v0)
    v = dev(v0)
    api.rk3_run_2d_char(v, dx2, dy2, 0)
    np.testing.assert_array_equal(v.cpu().numpy(), v0)


def test_empty_reconstruction(api):
    import torch
    note("empty reconstruction")
    f5 = torch.empty((5, 0), dtype=torch.float64, device="cuda")
    out = api.reconstruct(f5)
    torch.cuda.synchronize()
    assert out.numel() == 0


def test_batched_skips_short_and_empty_instances(api):
    import torch
    note("batched with empty and short instances")
    lens = np.array([0, 3, 5, 6, 300, 0, 1000, 7], dtype=np.int64)
    offs = np.zeros(len(lens) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(lens)
    rng = np.random.default_rng(77)
    U = np.empty((3, offs[-1]))
    for b, n in enumerate(lens):
        if n == 0:
            continue
        rl, ul, pl, rr, ur, pr = (rng.uniform(0.125, 5.0), rng.uniform(-1, 1), rng.uniform(0.1, 10),
                                  rng.uniform(0.125, 5.0), rng.uniform(-1, 1), rng.uniform(0.1, 10))
        x = (np.arange(n) + 0.5) / n
        left = x < 0.5
        U[:, offs[b]:offs[b + 1]] = I.prim_to_cons_1d(np.where(left, rl, rr),
                                                      np.where(left, ul, ur),
                                                      np.where(left, pl, pr))
    dx = 1.0 / np.maximum(lens, 1).astype(np.float64)
    nsteps = 6
    Ug = dev(U)
    api.batched_rk3_run_1d(Ug, dev(offs, torch.int64), dev(dx), nsteps)
    Ub = Ug.cpu().numpy()
    for b, n in enumerate(lens):
        sl = slice(offs[b], offs[b + 1])
        if n < 6:
            np.testing.assert_array_equal(Ub[:, sl], U[:, sl])
            continue
        u1 = dev(U[:, sl])
        api.rk3_run_1d(u1, dx[b], nsteps, cfl=0.5)
        np.testing.assert_array_equal(Ub[:, sl], u1.cpu().numpy())

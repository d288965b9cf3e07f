"""GPU parity of the 2D dimension-by-dimension HIP path against the CPU oracle.

fp64: normwise per component <= 1e-12 per RHS and <= 1e-10 after a run (the same reading as
1D).  fp32: compared with the fp64 oracle at the same eps (1e-30); the bound follows from
fp32 rounding: flux values carry relative errors of a few u32 = 6e-8, and their difference
over dx is compared with max|L| ~ |jump| / dx, so the normwise error is a small multiple of
u32 per RHS; the tests use 2e-5 per RHS and 1e-4 after 20 steps.
"""
import numpy as np
import pytest

from paper_2004_07954_amd import inputs as I

pytestmark = pytest.mark.gpu

RHS_TOL, RUN_TOL = 1e-12, 1e-10
RHS_TOL32, RUN_TOL32 = 2e-5, 1e-4


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2004_07954_amd import api
    return api


def note(*args):
    print("[gpu-case]", *args, flush=True)


def normwise(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    out = []
    for c in range(ref.shape[0]):
        scale = np.abs(ref[c]).max()
        out.append(np.abs(gpu[c] - ref[c]).max() / (scale if scale > 0 else 1.0))
    return max(out)


def to_dev(x, dtype=None):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype or torch.float64, device="cuda")


BC = {"transmissive": 1, "periodic": 0}


@pytest.mark.parametrize("nx,ny", [(6, 6), (37, 29), (130, 67), (1100, 70), (64, 300)])
@pytest.mark.parametrize("bcx,bcy", [("transmissive", "transmissive"), ("periodic", "transmissive"),
                                     ("transmissive", "periodic")])
def test_rhs_2d_random(api, orc, nx, ny, bcx, bcy):
    note("rhs_2d random", nx, ny, bcx, bcy)
    u = I.random_smooth_2d(nx, ny, seed=nx * 1000 + ny)
    g = api.rhs_2d(to_dev(u), 0.01, 0.02, api.params("euler", bc=bcx, bc_y=bcy)).cpu().numpy()
    r, _ = orc.rhs_2d(u, 0.01, 0.02, bcx=BC[bcx], bcy=BC[bcy])
    assert normwise(g, r) <= RHS_TOL


def test_rhs_2d_four_quadrant(api, orc):
    note("rhs_2d four quadrant 200x160")
    u, dx, dy = I.four_quadrant_random(200, 160, seed=3)
    g = api.rhs_2d(to_dev(u), dx, dy).cpu().numpy()
    r, _ = orc.rhs_2d(u, dx, dy)
    assert normwise(g, r) <= RHS_TOL


def test_rhs_2d_frozen_alphas(api, orc):
    note("rhs_2d frozen alphas")
    u = I.random_smooth_2d(50, 40, seed=5)
    prm = api.params("euler", lf_alpha=2.5, lf_alpha_y=3.0)
    g = api.rhs_2d(to_dev(u), 0.01, 0.01, prm).cpu().numpy()
    r, al = orc.rhs_2d(u, 0.01, 0.01, alpha_x=2.5, alpha_y=3.0)
    assert al == (2.5, 3.0)
    assert normwise(g, r) <= RHS_TOL


def test_run_2d_four_quadrant(api, orc):
    """128 x 96 four-quadrant data, 20 steps at CFL 0.5: states and dt history."""
    note("run_2d four quadrant 128x96 x20")
    u0, dx, dy = I.four_quadrant_random(128, 96, seed=3)
    ug = to_dev(u0)
    dtg = api.rk3_run_2d(ug, dx, dy, 20, cfl=0.5, record=True)
    ur, dtr = orc.rk3_run_2d(u0, dx, dy, 20, cfl=0.5)
    np.testing.assert_allclose(dtg.cpu().numpy(), dtr, rtol=1e-12)
    assert normwise(ug.cpu().numpy(), ur) <= RUN_TOL


def test_run_2d_periodic_conservation(api):
    """Periodic in both directions: sum_ij U_ij is conserved to rounding (telescoping of
    eq:2d) over 50 steps at 512 x 384."""
    import torch
    note("run_2d periodic conservation 512x384 x50")
    u0, dx, dy = I.four_quadrant_random(512, 384, seed=3)
    ug = to_dev(u0)
    api.rk3_run_2d(ug, dx, dy, 50, cfl=0.5, prm=api.params("euler", bc="periodic"))
    torch.cuda.synchronize()
    u = ug.cpu().numpy()
    s0 = u0.reshape(4, -1).sum(axis=1)
    s1 = u.reshape(4, -1).sum(axis=1)
    scale = np.abs(u0).reshape(4, -1).sum(axis=1)
    assert np.all(np.abs(s1 - s0) <= 1e-12 * scale)
    assert np.isfinite(u).all() and u[0].min() > 0


def test_full_size_rhs_2d(api, orc):
    """4096 x 4096 (the benchmark grid): one RHS against the oracle on every cell."""
    note("rhs_2d full size 4096^2")
    u, dx, dy = I.four_quadrant_random(4096, 4096, seed=3)
    g = api.rhs_2d(to_dev(u), dx, dy).cpu().numpy()
    r, _ = orc.rhs_2d(u, dx, dy)
    assert normwise(g, r) <= RHS_TOL


def test_full_size_steps_2d(api, orc):
    """4096 x 4096: two RK3 steps against the oracle."""
    note("run_2d full size 4096^2 x2")
    u0, dx, dy = I.four_quadrant_random(4096, 4096, seed=3)
    ug = to_dev(u0)
    api.rk3_run_2d(ug, dx, dy, 2, cfl=0.5)
    ur, _ = orc.rk3_run_2d(u0, dx, dy, 2, cfl=0.5)
    assert normwise(ug.cpu().numpy(), ur) <= RUN_TOL


# ---------------------------------------------------------------- fp32
def test_rhs_2d_fp32(api, orc):
    import torch
    note("rhs_2d fp32 four quadrant 300x200")
    u, dx, dy = I.four_quadrant_random(300, 200, seed=3)
    prm = api.params("euler", dtype="fp32", eps=1e-30)
    g = api.rhs_2d(to_dev(u, torch.float32), dx, dy, prm).cpu().numpy()
    r, _ = orc.rhs_2d(u.astype(np.float32).astype(np.float64), dx, dy, prm=orc.params(eps=1e-30))
    err = normwise(g, r)
    print("fp32 rhs normwise error %.3e" % err)
    assert err <= RHS_TOL32


def test_rhs_2d_fp32_degenerate(api, orc):
    """Plateaus, steps and symmetric peaks (IS_k = 0, tau5 = 0, tau8 = 0): the fp32 weights
    must stay finite and agree with the fp64 oracle."""
    import torch
    note("rhs_2d fp32 degenerate stencils")
    nx, ny = 64, 48
    i = np.arange(nx)[None, :] * np.ones((ny, 1))
    rho = 1.0 + (np.abs(i - 30) <= 1) + 2.0 * (i >= 45)
    U = I.prim_to_cons_2d(rho, 0.2, -0.1, 1.0 + 0.5 * (i >= 40))
    prm = api.params("euler", dtype="fp32", eps=1e-30)
    g = api.rhs_2d(to_dev(U, torch.float32), 0.05, 0.05, prm).cpu().numpy()
    r, _ = orc.rhs_2d(U.astype(np.float32).astype(np.float64), 0.05, 0.05,
                      prm=orc.params(eps=1e-30))
    assert np.isfinite(g).all()
    assert normwise(g, r) <= RHS_TOL32


def test_run_2d_fp32(api, orc):
    import torch
    note("run_2d fp32 128x96 x20")
    u0, dx, dy = I.four_quadrant_random(128, 96, seed=3)
    prm = api.params("euler", dtype="fp32", eps=1e-30)
    ug = to_dev(u0, torch.float32)
    api.rk3_run_2d(ug, dx, dy, 20, cfl=0.5, prm=prm)
    ur, _ = orc.rk3_run_2d(u0.astype(np.float32).astype(np.float64), dx, dy, 20, cfl=0.5,
                           prm=orc.params(eps=1e-30))
    err = normwise(ug.cpu().numpy(), ur)
    print("fp32 20-step normwise error %.3e" % err)
    assert err <= RUN_TOL32


def test_full_size_rhs_2d_fp32(api, orc):
    import torch
    note("rhs_2d fp32 full size 4096^2")
    u, dx, dy = I.four_quadrant_random(4096, 4096, seed=3)
    prm = api.params("euler", dtype="fp32", eps=1e-30)
    g = api.rhs_2d(to_dev(u, torch.float32), dx, dy, prm).cpu().numpy()
    r, _ = orc.rhs_2d(u.astype(np.float32).astype(np.float64), dx, dy, prm=orc.params(eps=1e-30))
    err = normwise(g, r)
    print("fp32 full-size rhs normwise error %.3e" % err)
    assert err <= RHS_TOL32

"""GPU parity of the 2D Steger-Warming path (the paper's 2D setup, Sec. 4.4) against the CPU
oracle, through the C ABI.  Same tolerances as the Lax-Friedrichs 2D path: fp64 normwise
per component 1e-12 per RHS and 1e-10 after a run; fp32 against the fp64 oracle at
eps = 1e-30, 2e-5 per RHS and 1e-4 after a run."""
import numpy as np
import pytest

from paper_2004_07954_amd import inputs as I

pytestmark = pytest.mark.gpu

RHS_TOL, RUN_TOL = 1e-12, 1e-10
RHS_TOL32, RUN_TOL32 = 2e-5, 1e-4
BC = {"transmissive": 1, "periodic": 0}


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


def sw(api, bc="transmissive", bc_y=None, **kw):
    return api.params("euler", bc=bc, bc_y=bc_y, split="sw", **kw)


@pytest.mark.parametrize("nx,ny", [(6, 6), (37, 29), (130, 67), (1100, 70), (64, 300)])
@pytest.mark.parametrize("bcx,bcy", [("transmissive", "transmissive"), ("periodic", "transmissive"),
                                     ("transmissive", "periodic")])
def test_rhs_random(api, orc, nx, ny, bcx, bcy):
    note("rhs_2d sw random", nx, ny, bcx, bcy)
    u = I.random_smooth_2d(nx, ny, seed=nx * 7 + ny)
    g = api.rhs_2d(to_dev(u), 0.01, 0.02, sw(api, bcx, bcy)).cpu().numpy()
    r = orc.rhs_2d_sw(u, 0.01, 0.02, bcx=BC[bcx], bcy=BC[bcy])
    assert normwise(g, r) <= RHS_TOL, normwise(g, r)


def test_rhs_supersonic_and_sonic_states(api, orc):
    """States with |u|, |v| around and above c, so every eigenvalue changes sign somewhere:
    both branches of every split."""
    note("rhs_2d sw sonic")
    rng = np.random.default_rng(61)
    ny, nx = 40, 70
    rho = rng.uniform(0.5, 1.5, (ny, nx))
    p = rng.uniform(0.5, 1.5, (ny, nx))
    c = np.sqrt(1.4 * p / rho)
    u = rng.uniform(-2.0, 2.0, (ny, nx)) * c
    v = rng.uniform(-2.0, 2.0, (ny, nx)) * c
    U = I.prim_to_cons_2d(rho, u, v, p)
    g = api.rhs_2d(to_dev(U), 0.02, 0.02, sw(api)).cpu().numpy()
    r = orc.rhs_2d_sw(U, 0.02, 0.02)
    assert normwise(g, r) <= RHS_TOL, normwise(g, r)


@pytest.mark.parametrize("case,n", [(1, 400), (2, 300)])
def test_rhs_riemann_cases(api, orc, case, n):
    note("rhs_2d sw riemann", case, n)
    u, dx, dy = I.riemann_2d(case, n)
    g = api.rhs_2d(to_dev(u), dx, dy, sw(api)).cpu().numpy()
    r = orc.rhs_2d_sw(u, dx, dy)
    assert normwise(g, r) <= RHS_TOL, normwise(g, r)


@pytest.mark.parametrize("case,n", [(1, 128), (2, 160)])
def test_run_riemann_cases(api, orc, case, n):
    """10 steps (through the initial discontinuities), with the dt history."""
    note("rk3_run_2d sw riemann", case, n)
    u0, dx, dy = I.riemann_2d(case, n)
    ug = to_dev(u0)
    dtg = api.rk3_run_2d(ug, dx, dy, 10, cfl=0.5, prm=sw(api), record=True)
    ur, dtr = orc.rk3_run_2d_sw(u0, dx, dy, 10, cfl=0.5)
    assert np.allclose(dtg.cpu().numpy(), dtr, rtol=1e-13, atol=0)
    assert normwise(ug.cpu().numpy(), ur) <= RUN_TOL, normwise(ug.cpu().numpy(), ur)


def test_run_periodic_conservation(api):
    note("rk3_run_2d sw periodic conservation")
    u0 = I.random_smooth_2d(96, 80, seed=62)
    ug = to_dev(u0)
    api.rk3_run_2d(ug, 0.01, 0.01, 30, cfl=0.4, prm=sw(api, "periodic"))
    g = ug.cpu().numpy()
    assert np.abs(g.sum(axis=(1, 2)) - u0.sum(axis=(1, 2))).max() <= 1e-11 * np.abs(u0).sum()


def test_full_size_rhs(api, orc):
    """The paper's finest grid, 2400^2, case 2: every cell against the oracle."""
    note("rhs_2d sw riemann 2 at 2400^2")
    u, dx, dy = I.riemann_2d(2, 2400)
    g = api.rhs_2d(to_dev(u), dx, dy, sw(api)).cpu().numpy()
    r = orc.rhs_2d_sw(u, dx, dy)
    assert normwise(g, r) <= RHS_TOL, normwise(g, r)


def test_rhs_fp32(api, orc):
    import torch
    note("rhs_2d sw fp32")
    u, dx, dy = I.riemann_2d(1, 200)
    g = api.rhs_2d(to_dev(u, torch.float32), dx, dy, sw(api, dtype="fp32", eps=1e-30)).cpu().numpy()
    r = orc.rhs_2d_sw(u.astype(np.float32).astype(np.float64), dx, dy, prm=orc.params(eps=1e-30))
    assert normwise(g, r) <= RHS_TOL32, normwise(g, r)


def test_run_fp32(api, orc):
    import torch
    note("rk3_run_2d sw fp32")
    u0, dx, dy = I.riemann_2d(2, 128)
    ug = to_dev(u0, torch.float32)
    api.rk3_run_2d(ug, dx, dy, 20, cfl=0.5, prm=sw(api, dtype="fp32", eps=1e-30))
    ur, _ = orc.rk3_run_2d_sw(u0.astype(np.float32).astype(np.float64), dx, dy, 20, cfl=0.5,
                              prm=orc.params(eps=1e-30))
    assert normwise(ug.cpu().numpy(), ur) <= RUN_TOL32, normwise(ug.cpu().numpy(), ur)


def test_split_bits_do_not_depend_on_row_shape(api):
    """The x sweep's launch shapes (tile and split layouts) give the same bits under the
    Steger-Warming split."""
    from paper_2004_07954_amd import autotune
    note("rhs_2d sw row shapes")
    u, dx, dy = I.riemann_2d(2, 333)
    ud = to_dev(u)
    outs = []
    try:
        for nt, k, lay in [(256, 2, 0), (256, 4, 0), (128, 4, 0), (256, 2, 1), (256, 4, 1)]:
            autotune.set_row_tuning(nt, k, lay)
            outs.append(api.rhs_2d(ud, dx, dy, sw(api)).cpu().numpy())
    finally:
        autotune.set_row_tuning(0, 0)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_sw_rejected_by_1d_entry_points(api):
    from paper_2004_07954_amd import _lib
    note("sw in 1D rejected")
    u = to_dev(I.random_smooth_1d(64, seed=2))
    prm = api.params("euler", split="sw")
    with pytest.raises(_lib.WznError) as e:
        api.rhs_1d(u, 0.1, prm)
    assert e.value.code == _lib.WZN_ERR_UNSUPPORTED

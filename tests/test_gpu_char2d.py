"""2D Euler with each sweep's reconstruction in local characteristic fields on the GPU
(wzn_rhs_2d_char, wzn_rk3_run_2d_char) against the oracle: right-hand sides at ragged sizes
with both boundary conditions and on the paper's Riemann data, frozen alphas, runs with their
dt history, the x/y exchange (bit for bit: the column kernel's y sweep evaluates the x
sweep's faces on the state with its momenta exchanged), the reduction to the 1D
characteristic scheme, conservation and the argument checks."""
import numpy as np
import pytest

from paper_2004_07954_amd import inputs as I

pytestmark = pytest.mark.gpu

RHS_TOL, RUN_TOL = 1e-12, 1e-10


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2004_07954_amd import api
    return api


def note(*args):
    print("[gpu-case]", *args, flush=True)


def to_dev(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def normwise(gpu, ref):
    out = []
    for c in range(ref.shape[0]):
        scale = np.abs(ref[c]).max()
        out.append(np.abs(gpu[c] - ref[c]).max() / (scale if scale > 0 else 1.0))
    return max(out)


BC = {"transmissive": 1, "periodic": 0}


@pytest.mark.parametrize("nx,ny", [(6, 6), (37, 23), (260, 70), (300, 257)])
@pytest.mark.parametrize("bcx,bcy", [("transmissive", "periodic"), ("periodic", "transmissive")])
def test_rhs_random(api, orc, nx, ny, bcx, bcy):
    note("rhs_2d_char random", nx, ny, bcx, bcy)
    U = I.random_smooth_2d(nx, ny, seed=700 + nx + ny)
    prm = api.params("euler", bc=bcx, bc_y=bcy)
    g = api.rhs_2d_char(to_dev(U), 0.02, 0.03, prm).cpu().numpy()
    r, _ = orc.rhs_2d_char(U, 0.02, 0.03, bcx=BC[bcx], bcy=BC[bcy])
    assert normwise(g, r) <= RHS_TOL, normwise(g, r)


@pytest.mark.parametrize("case", [1, 2])
def test_rhs_riemann_and_frozen_alphas(api, orc, case):
    note("rhs_2d_char riemann", case)
    U, dx, dy = I.riemann_2d(case, 200)
    r, a8 = orc.rhs_2d_char(U, dx, dy)
    g = api.rhs_2d_char(to_dev(U), dx, dy).cpu().numpy()
    assert normwise(g, r) <= RHS_TOL, normwise(g, r)
    # the same alphas passed in: the frozen path
    gf = api.rhs_2d_char(to_dev(U), dx, dy, alpha8=to_dev(a8)).cpu().numpy()
    assert normwise(gf, r) <= RHS_TOL
    # other frozen alphas: the oracle with the same ones
    a2 = a8 * 1.25
    r2, _ = orc.rhs_2d_char(U, dx, dy, alpha8=a2)
    g2 = api.rhs_2d_char(to_dev(U), dx, dy, alpha8=to_dev(a2)).cpu().numpy()
    assert normwise(g2, r2) <= RHS_TOL


def test_full_size_riemann_case_2(api, orc):
    """The paper's 1200^2 grid of its second Riemann case: every cell against the oracle."""
    note("rhs_2d_char riemann case 2 at 1200^2")
    U, dx, dy = I.riemann_2d(2, 1200)
    r, _ = orc.rhs_2d_char(U, dx, dy)
    g = api.rhs_2d_char(to_dev(U), dx, dy).cpu().numpy()
    assert normwise(g, r) <= RHS_TOL, normwise(g, r)


@pytest.mark.parametrize("case,n", [(1, 96), (2, 128)])
def test_runs(api, orc, case, n):
    import torch
    note("rk3_run_2d_char riemann", case, n)
    U, dx, dy = I.riemann_2d(case, n)
    ug = to_dev(U)
    dtg = api.rk3_run_2d_char(ug, dx, dy, 10, cfl=0.5, record=True)
    r, dtr = orc.rk3_run_2d_char(U, dx, dy, 10, cfl=0.5)
    assert np.allclose(dtg.cpu().numpy(), dtr, rtol=1e-13, atol=0)
    assert normwise(ug.cpu().numpy(), r) <= RUN_TOL
    # a frozen dt schedule reproduces the same run
    ug2 = to_dev(U)
    api.rk3_run_2d_char(ug2, dx, dy, 10, dt=dtg)
    assert torch.equal(ug2, ug)


def test_exchange_of_x_and_y_is_bitwise(api):
    import torch
    note("rhs_2d_char x/y exchange")
    U = I.random_smooth_2d(70, 45, seed=720)
    prm = api.params("euler", bc="transmissive", bc_y="periodic")
    L = api.rhs_2d_char(to_dev(U), 0.02, 0.035, prm)
    T = np.ascontiguousarray(U[[0, 2, 1, 3]].transpose(0, 2, 1))
    prm_t = api.params("euler", bc="periodic", bc_y="transmissive")
    Lt = api.rhs_2d_char(to_dev(T), 0.035, 0.02, prm_t)
    want = L[[0, 2, 1, 3]].transpose(1, 2).contiguous()
    assert torch.equal(Lt, want)


def test_reduces_to_the_1d_characteristic_path(api):
    note("rhs_2d_char y-uniform state against rhs_1d_char")
    u1, dx = I.shu_osher_like(700)
    U = np.zeros((4, 9, 700))
    U[0], U[1], U[3] = u1[0], u1[1], u1[2]
    L = api.rhs_2d_char(to_dev(U), dx, 0.37, api.params("euler", bc="transmissive",
                                                        bc_y="periodic")).cpu().numpy()
    r = api.rhs_1d_char(to_dev(u1), dx).cpu().numpy()
    assert np.all(L[2] == 0.0)
    for j in range(9):
        for c2, c1 in ((0, 0), (1, 1), (3, 2)):
            assert np.abs(L[c2, j] - r[c1]).max() <= 1e-13 * np.abs(r[c1]).max()


def test_periodic_conservation(api):
    note("rhs_2d_char periodic conservation")
    U = I.random_smooth_2d(300, 200, seed=721)
    L = api.rhs_2d_char(to_dev(U), 0.01, 0.01, api.params("euler", bc="periodic")).cpu().numpy()
    assert np.abs(L.sum(axis=(1, 2))).max() <= 1e-12 * np.abs(L).sum(axis=(1, 2)).max()


def test_argument_checks(api):
    import torch
    from paper_2004_07954_amd import _lib
    note("rhs_2d_char argument checks")
    U = to_dev(I.random_smooth_2d(16, 12, seed=722))
    for kw, code in ((dict(split="sw"), _lib.WZN_ERR_UNSUPPORTED),
                     (dict(weights="z"), _lib.WZN_ERR_UNSUPPORTED)):
        with pytest.raises(_lib.WznError) as e:
            api.rhs_2d_char(U, 0.1, 0.1, api.params("euler", **kw))
        assert e.value.code == code
    with pytest.raises(_lib.WznError) as e:
        api.rhs_2d_char(U.float(), 0.1, 0.1, api.params("euler", dtype="fp32", eps=1e-30))
    assert e.value.code == _lib.WZN_ERR_DTYPE
    with pytest.raises(_lib.WznError) as e:  # one direction frozen, the other reduced
        api.rhs_2d_char(U, 0.1, 0.1, api.params("euler", lf_alpha=2.0))
    assert e.value.code == _lib.WZN_ERR_UNSUPPORTED
    with pytest.raises(ValueError):
        api.rhs_2d_char(U, 0.1, 0.1, work=torch.empty(10, dtype=torch.float64, device="cuda"))

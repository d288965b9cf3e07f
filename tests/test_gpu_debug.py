"""The debug_nonfinite mode: with it set, an entry point scans its output, synchronises and
returns WZN_ERR_NONFINITE for NaN / Inf; without it nothing is checked."""
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


def to_dev(x, dtype=None):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype or torch.float64, device="cuda")


def test_nonfinite_reported_only_in_debug_mode(api):
    from paper_2004_07954_amd import _lib
    print("[gpu-case] debug_nonfinite 1d", flush=True)
    u = I.random_smooth_1d(500, seed=3)
    u[0, 17] = np.nan
    L = api.rhs_1d(to_dev(u), 0.01).cpu().numpy()  # no scan: returns, with NaNs in L
    assert not np.isfinite(L).all()
    with pytest.raises(_lib.WznError) as e:
        api.rhs_1d(to_dev(u), 0.01, api.params("euler", debug_nonfinite=True))
    assert e.value.code == _lib.WZN_ERR_NONFINITE and "non-finite" in str(e.value)
    good = to_dev(I.random_smooth_1d(500, seed=3))
    api.rhs_1d(good, 0.01, api.params("euler", debug_nonfinite=True))
    api.rk3_run_1d(good, 0.01, 3, prm=api.params("euler", debug_nonfinite=True))


def test_nonfinite_2d_fp32_and_runs(api):
    import torch
    from paper_2004_07954_amd import _lib
    print("[gpu-case] debug_nonfinite 2d", flush=True)
    U, dx, dy = I.riemann_2d(1, 64)
    prm = api.params("euler", dtype="fp32", eps=1e-30, debug_nonfinite=True)
    api.rk3_run_2d(to_dev(U, torch.float32), dx, dy, 2, prm=prm)
    bad = U.copy()
    bad[3, 10, 20] = np.inf
    with pytest.raises(_lib.WznError) as e:
        api.rhs_2d(to_dev(bad, torch.float32), dx, dy, prm)
    assert e.value.code == _lib.WZN_ERR_NONFINITE
    # a run whose step is far beyond the CFL limit blows up: the scan reports it
    u = to_dev(I.shu_osher_like(400)[0])
    with pytest.raises(_lib.WznError) as e:
        api.rk3_run_1d(u, 0.025, 50, dt=5.0, prm=api.params("euler", debug_nonfinite=True))
    assert e.value.code == _lib.WZN_ERR_NONFINITE

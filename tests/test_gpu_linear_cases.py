"""The paper's linear advection cases (Sec. 4.2; N = 200, T = 6, periodic, dt = T / ceil(T /
(0.5 dx))) on the GPU: the full runs against the oracle, self-similarity of case 1 under the
reference value A, and the non-oscillation bound, for the paper's weights and for the WENO-Z
comparison weights."""
import numpy as np
import pytest

from paper_2004_07954_amd import inputs as I

pytestmark = pytest.mark.gpu

N, T = 200, 6.0
RUN_TOL = 1e-10
JUMP = {1: 1.0, 2: 1.0, 3: 2.0}


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2004_07954_amd import api
    return api


def note(*args):
    print("[gpu-case]", *args, flush=True)


def _schedule(dx):
    nsteps = int(np.ceil(T / (0.5 * dx) - 1e-12))
    return nsteps, T / nsteps


def _gpu_run(api, u0, dx, weights="zn"):
    import torch
    nsteps, dt = _schedule(dx)
    u = torch.tensor(u0, dtype=torch.float64, device="cuda")
    api.rk3_run_1d(u, dx, nsteps, dt=dt,
                   prm=api.params("advection", bc="periodic", weights=weights))
    return u.cpu().numpy()[0]


@pytest.mark.parametrize("case", [1, 2, 3])
@pytest.mark.parametrize("weights,scheme", [("zn", 0), ("z", 1)])
def test_runs_against_oracle(api, orc, case, weights, scheme):
    note("linear case", case, weights)
    u0, dx = I.linear_case(case, N)
    g = _gpu_run(api, u0, dx, weights)
    nsteps, dt = _schedule(dx)
    r, _, _ = orc.rk3_run_1d(u0, dx, nsteps, dt=dt, sys=orc.SYS_ADV, bc=orc.BC_PERIODIC,
                             prm=orc.params(scheme=scheme, q=1))
    assert np.abs(g - r[0]).max() <= RUN_TOL * np.abs(r[0]).max()


@pytest.mark.parametrize("weights", ["zn", "z"])
def test_self_similarity(api, weights):
    note("linear case 1 self-similarity", weights)
    u1, dx = I.linear_case(1, N, 1.0)
    g1 = _gpu_run(api, u1, dx, weights)
    for A in (100.0, 0.01):
        uA, _ = I.linear_case(1, N, A)
        gA = _gpu_run(api, uA, dx, weights)
        assert np.abs(A * gA - g1).max() <= 1e-12


@pytest.mark.parametrize("case", [1, 2, 3])
def test_non_oscillatory(api, case):
    note("linear case non-oscillatory", case)
    u0, dx = I.linear_case(case, N)
    g = _gpu_run(api, u0, dx)
    assert g.max() - u0.max() <= 0.01 * JUMP[case]
    assert u0.min() - g.min() <= 0.01 * JUMP[case]

"""GPU checks that every launch shape of the 1D row kernel gives the same bits.

The LDS-tile layout (one workgroup tile staged in LDS) and its split variant (the two signs of
the split flux staged one after the other) evaluate the same arithmetic in the same order, so a right-hand side and a short TVD-RK3 run must agree bit for bit across all
shapes, and with the CPU oracle to the parity tolerances, on ragged sizes (runs and tiles
that end inside the row, rows shorter than one run) and both boundary conditions.
"""
import numpy as np
import pytest

from paper_2004_07954_amd import inputs as I

pytestmark = pytest.mark.gpu

RHS_TOL = 1e-12
RUN_TOL = 1e-10
SHAPES = [(256, 4, 0), (256, 2, 0), (256, 1, 0), (128, 4, 0), (128, 8, 0), (64, 8, 0),
          (64, 4, 0), (64, 2, 0), (64, 1, 0), (256, 4, 1), (256, 2, 1), (128, 4, 1), (64, 4, 1)]


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2004_07954_amd import api, autotune
    yield api
    autotune.set_row_tuning(0, 0)


def note(*args):
    print("[gpu-case]", *args, flush=True)


def normwise(gpu, ref):
    out = []
    for c in range(ref.shape[0]):
        scale = np.abs(ref[c]).max()
        out.append(np.abs(gpu[c] - ref[c]).max() / (scale if scale > 0 else 1.0))
    return max(out)


def to_dev(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("n", [6, 7, 130, 255, 256, 257, 1000, 5000, 20011])
@pytest.mark.parametrize("bc", ["transmissive", "periodic"])
def test_euler_shapes_agree(api, orc, n, bc):
    from paper_2004_07954_amd import autotune
    note("row shapes euler", n, bc)
    u0 = I.random_smooth_1d(n, seed=300 + n)
    if bc == "transmissive":
        u0[:, n // 3:] *= 1.5  # a jump inside the row
    dx = 1.0 / n
    bcc = orc.BC_TRANSMISSIVE if bc == "transmissive" else orc.BC_PERIODIC
    r, _ = orc.rhs_1d(u0, dx, bc=bcc)
    ur, _, _ = orc.rk3_run_1d(u0, dx, 4, cfl=0.5, bc=bcc)
    prm = api.params("euler", bc=bc)
    ref_rhs = ref_run = None
    for shape in SHAPES:
        autotune.set_row_tuning(*shape)
        g = api.rhs_1d(to_dev(u0), dx, prm).cpu().numpy()
        ug = to_dev(u0)
        api.rk3_run_1d(ug, dx, 4, cfl=0.5, prm=prm)
        ug = ug.cpu().numpy()
        if ref_rhs is None:
            ref_rhs, ref_run = g, ug
            assert normwise(g, r) <= RHS_TOL
            assert normwise(ug, ur) <= RUN_TOL
        else:
            np.testing.assert_array_equal(g, ref_rhs, err_msg=str(shape))
            np.testing.assert_array_equal(ug, ref_run, err_msg=str(shape))
    autotune.set_row_tuning(0, 0)

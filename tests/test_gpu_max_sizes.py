"""The largest sizes the entry points accept, where element offsets pass 2^31.

A row of 2^30 cells (the 1D limit) and a 65536 x 32768 fp32 grid (a plane of 2^31 elements)
are built by tiling a small pattern.  Away from the ends of the big row (the edges of the
big grid), every cell then sees the same stencil values as the small pattern with periodic
boundaries.  The global maxima are the same too, because the big array holds the same
multiset of cells.  So the big right-hand side must equal the small periodic one bit for bit
on every interior copy.  The small periodic right-hand side is checked against the oracle in
the other tests; the cells next to the big row's ends are checked against the oracle here,
on a window with the same alpha."""
import numpy as np
import pytest

from paper_2004_07954_amd import inputs as I

pytestmark = pytest.mark.gpu

RHS_TOL = 1e-12


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2004_07954_amd import api
    return api


def note(*args):
    print("[gpu-case]", *args, flush=True)


def normwise(gpu, ref, scale):
    """max_i |gpu - ref| / scale per component (the scale of the whole row: a window of a
    smooth region holds only rounding-level values of L, which a norm over the window would
    magnify)."""
    return max(np.abs(gpu[c] - ref[c]).max() / scale[c] for c in range(ref.shape[0]))


def _free():
    import torch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_row_of_2_30_cells(api, orc):
    import torch
    M, R = 1 << 20, 1 << 10
    n = M * R
    note("rhs_1d and one RK3 step at n = 2^30 (a 2^20 pattern tiled 1024 times)")
    u0, dx = I.shu_osher_like(M)
    small = torch.tensor(u0, dtype=torch.float64, device="cuda")
    Ls = api.rhs_1d(small, dx, api.params("euler", bc="periodic"))
    alpha = api.speed_max_1d(small).item()

    big = small.repeat(1, R)
    assert big.shape == (3, n)
    assert api.speed_max_1d(big).item() == alpha
    Lb = api.rhs_1d(big, dx, api.params("euler"))
    for r in range(1, R - 1):
        assert torch.equal(Lb[:, r * M:(r + 1) * M], Ls), r
    assert torch.equal(Lb[:, 3:M], Ls[:, 3:])
    assert torch.equal(Lb[:, n - M:n - 3], Ls[:, :M - 3])
    # the cells next to the two ends (transmissive there) against the oracle, same alpha
    W = 64
    lo = Lb[:, :W].cpu().numpy()
    hi = Lb[:, n - W:].cpu().numpy()
    rlo, _ = orc.rhs_1d(u0[:, :W], dx, alpha=alpha)
    rhi, _ = orc.rhs_1d(u0[:, M - W:], dx, alpha=alpha)
    scale = Ls.abs().amax(dim=1).cpu().numpy()
    assert normwise(lo[:, :W - 3], rlo[:, :W - 3], scale) <= RHS_TOL
    assert normwise(hi[:, 3:], rhi[:, 3:], scale) <= RHS_TOL
    del Lb
    _free()

    # one TVD-RK3 step with a frozen schedule (the same dt and per-stage alphas for both)
    us = small.clone()
    dts, als = api.rk3_run_1d(us, dx, 1, cfl=0.5, prm=api.params("euler", bc="periodic"),
                              record=True)
    api.rk3_run_1d(big, dx, 1, dt=dts, alpha=als, prm=api.params("euler"))
    for r in range(1, R - 1):
        assert torch.equal(big[:, r * M:(r + 1) * M], us), r
    assert torch.isfinite(big[:, :M]).all() and torch.isfinite(big[:, n - M:]).all()
    del big, us, small
    _free()


def test_grid_with_a_2_31_element_plane(api):
    import torch
    P, BY, BX = 256, 128, 256
    ny, nx = P * BY, P * BX
    note("rhs_2d fp32 at %d x %d (plane of 2^31 elements, a 256^2 pattern tiled)" % (nx, ny))
    u0, dx, dy = I.four_quadrant_random(P, P, seed=3)
    prm_p = api.params("euler", dtype="fp32", eps=1e-30, bc="periodic")
    prm_t = api.params("euler", dtype="fp32", eps=1e-30)
    small = torch.tensor(u0, dtype=torch.float32, device="cuda")
    Ls = api.rhs_2d(small, dx, dy, prm_p)
    big = small.repeat(1, BY, BX)
    assert big.shape == (4, ny, nx) and ny * nx == 1 << 31
    assert torch.equal(api.speed_max_2d(big, prm_t), api.speed_max_2d(small, prm_t))
    Lb = api.rhs_2d(big, dx, dy, prm_t)
    Lv = Lb.view(4, BY, P, BX, P)
    for by in range(1, BY - 1):
        blk = Lv[:, by, :, 1:BX - 1, :]
        assert torch.equal(blk, Ls[:, :, None, :].expand_as(blk)), by
    assert torch.isfinite(Lb[:, :3]).all() and torch.isfinite(Lb[:, -3:]).all()
    del Lb, Lv, big, small
    _free()


def test_batched_launch_at_its_2_30_cell_limit(api):
    """1024 instances of 2^20 cells in one batched launch: the concatenated state holds the
    2^30 cells the launch accepts at most, so the third component starts at element 2^31.
    Every instance starts from the same state, so every one must come out bit for bit equal
    to the one-instance run of that state (same tile, exact maxima)."""
    import torch
    M, B = 1 << 20, 1024
    note("batched run of %d instances of 2^20 cells (%d cells, the third component at 2^31)"
         % (B, B * M))
    u0, dx = I.shu_osher_like(M)
    one = torch.tensor(u0, dtype=torch.float64, device="cuda")
    big = one.repeat(1, B)
    assert 2 * B * M == (1 << 31)
    offs = torch.arange(0, B + 1, dtype=torch.int64, device="cuda") * M
    dxs = torch.full((B,), dx, dtype=torch.float64, device="cuda")
    api.batched_rk3_run_1d(big, offs, dxs, 1)
    api.rk3_run_1d(one, dx, 1, cfl=0.5)
    assert bool((big.view(3, B, M) == one[:, None, :]).all())
    del big, one, offs, dxs
    _free()

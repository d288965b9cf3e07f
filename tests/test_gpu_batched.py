"""GPU checks of the persistent batched launch (many 1D Euler shock tubes of uneven length).

The batched kernel runs the same row tile as the one-instance path, and maxima are exact, so
each instance must come out bit for bit equal to a one-instance run of the same state; both
are checked against the CPU oracle (normwise 1e-10 after a short run through the shock).
"""
import numpy as np
import pytest

from paper_2004_07954_amd import inputs as I

pytestmark = pytest.mark.gpu
RUN_TOL = 1e-10


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2004_07954_amd import api
    return api


def note(*args):
    print("[gpu-case]", *args, flush=True)


def normwise(gpu, ref):
    out = []
    for c in range(ref.shape[0]):
        scale = np.abs(ref[c]).max()
        out.append(np.abs(gpu[c] - ref[c]).max() / (scale if scale > 0 else 1.0))
    return max(out)


def make_batch(lens, seed):
    """Shock tubes with the given lengths (state draws as in the batched workload)."""
    import torch
    rng = np.random.default_rng(seed)
    lens = np.asarray(lens, dtype=np.int64)
    offs = np.zeros(len(lens) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(lens)
    U = np.empty((3, offs[-1]))
    for b, n in enumerate(lens):
        rl, ul, pl, rr, ur, pr = (rng.uniform(0.125, 5.0), rng.uniform(-1, 1), rng.uniform(0.1, 10),
                                  rng.uniform(0.125, 5.0), rng.uniform(-1, 1), rng.uniform(0.1, 10))
        x, _ = I.cell_centres(0.0, 1.0, int(n))
        left = x < 0.5
        U[:, offs[b]:offs[b + 1]] = I.prim_to_cons_1d(np.where(left, rl, rr), np.where(left, ul, ur),
                                                      np.where(left, pl, pr))
    dx = 1.0 / lens.astype(np.float64)
    dev = lambda a, dt: torch.tensor(a, dtype=dt, device="cuda")
    return U, offs, dx, dev(U, torch.float64), dev(offs, torch.int64), dev(dx, torch.float64)


LENS = [6, 7, 100, 255, 256, 257, 511, 1024, 1025, 3000, 40, 777]


@pytest.mark.parametrize("nt,k,lay", [(64, 2, 0), (64, 4, 0), (128, 2, 0), (128, 4, 0), (256, 1, 0),
                                      (256, 2, 0), (256, 4, 0), (128, 4, 1), (256, 2, 1),
                                      (256, 4, 1)])
def test_batched_matches_single_and_oracle(api, orc, nt, k, lay):
    import torch
    note("batched vs single vs oracle", nt, k, lay)
    U, offs, dx, Ug, offg, dxg = make_batch(LENS, seed=41)
    nsteps = 12
    order = api.lpt_order(np.diff(offs))
    dtb = api.batched_rk3_run_1d(Ug, offg, dxg, nsteps, order=order,
                                 tuning=api.batch_tuning(nt, k, 0, lay), record=True)
    torch.cuda.synchronize()
    Ub = Ug.cpu().numpy()
    dtb = dtb.cpu().numpy()
    for b in range(len(LENS)):
        sl = slice(offs[b], offs[b + 1])
        u1 = torch.tensor(np.ascontiguousarray(U[:, sl]), dtype=torch.float64, device="cuda")
        dts, _ = api.rk3_run_1d(u1, dx[b], nsteps, cfl=0.5, record=True)
        np.testing.assert_array_equal(Ub[:, sl], u1.cpu().numpy())
        np.testing.assert_array_equal(dtb[b], dts.cpu().numpy())
        ur, dtr, _ = orc.rk3_run_1d(U[:, sl], dx[b], nsteps, cfl=0.5)
        assert normwise(Ub[:, sl], ur) <= RUN_TOL, b
        np.testing.assert_allclose(dtb[b], dtr, rtol=RUN_TOL)


def test_batched_order_and_blocks_invariance(api):
    """The processing order and the number of resident workgroups do not change results."""
    note("batched order/blocks invariance")
    U, offs, dx, Ug, offg, dxg = make_batch(LENS * 3, seed=42)
    a = Ug.clone()
    api.batched_rk3_run_1d(a, offg, dxg, 8, tuning=api.batch_tuning(128, 2, 1))
    b = Ug.clone()
    api.batched_rk3_run_1d(b, offg, dxg, 8, order=api.lpt_order(np.diff(offs)),
                           tuning=api.batch_tuning(128, 2, 0))
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())


# Instance 1767 of the seed-4 batch (N = 12399; left rho 4.09, u 0.61, p 0.13; right rho 0.23,
# u -0.52, p 1.99) loses positivity after ~200 steps: the CPU oracle run of that instance
# alone reaches rho < 0 at step ~220 and NaN by step ~275.  Component-wise Lax-Friedrichs
# WENO-ZN carries no positivity limiter; the instances are independent, so the NaNs stay in
# that instance.
UNSTABLE = {1767}


def test_batched_full_workload_sampled(api):
    """The benchmark workload (4096 instances, N_i in [256, 16384], seed 4) for 500 steps in
    the launch configuration the benchmark times (autotuned): a sample of instances is re-run
    one by one through the single-instance path and must match bit for bit (including the
    unstable instance's NaNs); every other instance stays finite with rho, p > 0."""
    import torch
    from paper_2004_07954_amd import autotune
    note("batched full workload 4096 x 500")
    U, offs, dx = I.shock_tube_batch(4096, seed=4)
    Ug = torch.tensor(U, dtype=torch.float64, device="cuda")
    offg = torch.tensor(offs, dtype=torch.int64, device="cuda")
    dxg = torch.tensor(dx, dtype=torch.float64, device="cuda")
    order = api.lpt_order(np.diff(offs))
    tn, _ = autotune.tune_batched(Ug, offg, dxg, order=order)
    api.batched_rk3_run_1d(Ug, offg, dxg, 500, order=order, tuning=tn)
    torch.cuda.synchronize()
    Ub = Ug.cpu().numpy()
    rho, m, E = Ub
    with np.errstate(invalid="ignore", divide="ignore"):
        p = 0.4 * (E - 0.5 * m * m / rho)
    bad = ~np.isfinite(Ub).all(axis=0) | (rho <= 0) | (p <= 0)
    bad_inst = set(np.unique(np.searchsorted(offs, np.nonzero(bad)[0], side="right") - 1).tolist())
    assert bad_inst == UNSTABLE, bad_inst
    sample = list(np.random.default_rng(7).choice(4096, 12, replace=False)) + sorted(UNSTABLE)
    for b in sample:
        sl = slice(offs[b], offs[b + 1])
        u1 = torch.tensor(np.ascontiguousarray(U[:, sl]), dtype=torch.float64, device="cuda")
        api.rk3_run_1d(u1, dx[b], 500, cfl=0.5)
        np.testing.assert_array_equal(Ub[:, sl], u1.cpu().numpy())


def test_batched_bad_arguments(api):
    import torch
    from paper_2004_07954_amd._lib import WznError
    U, offs, dx, Ug, offg, dxg = make_batch([10, 20], seed=1)
    with pytest.raises(WznError):
        api.batched_rk3_run_1d(Ug, offg, dxg, 2, tuning=api.batch_tuning(96, 2))
    with pytest.raises(WznError):
        api.batched_rk3_run_1d(Ug, offg, dxg, 2, tuning=api.batch_tuning(64, 2, 0, 1))
    with pytest.raises(WznError):
        api.batched_rk3_run_1d(Ug, offg, dxg, 2, prm=api.params("euler", lf_alpha=1.0))

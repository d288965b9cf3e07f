"""The allocation-free right-hand side (wzn_rhs_1d_noalloc) through the C ABI: its scratch is
the library's own device array, so the caller passes only the input and the output.  Two calls
in a row, the second with a smaller grid, each equal bit for bit to wzn_rhs_1d with a caller
workspace (the same kernels) and within the right-hand-side tolerance of the oracle."""
import ctypes as C

import numpy as np
import pytest

from paper_2004_07954_amd import inputs as I

pytestmark = pytest.mark.gpu


def _noalloc(L):
    return L.wzn_rhs_1d_noalloc


@pytest.mark.parametrize("system", ["euler", "advection"])
def test_rhs_1d_noalloc_matches_workspace_entry_point(orc, system):
    import torch
    from paper_2004_07954_amd import _lib, api
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    print("[gpu-case] wzn_rhs_1d_noalloc", system, flush=True)
    L = _lib.lib()
    f = _noalloc(L)
    prm = api.params(system, bc="transmissive" if system == "euler" else "periodic")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    # the second call smaller than the first; smooth advection stays at sizes where the
    # right-hand side's ulp-level flux differences over dx stay below 1e-12 of its scale
    for n in ((300000, 4099) if system == "euler" else (5000, 1000)):
        if system == "euler":
            u0, dx = I.shu_osher_like(n)
        else:
            u0, dx = I.advection_smooth(n)
        u = torch.tensor(u0, dtype=torch.float64, device="cuda")
        out = torch.full_like(u, float("nan"))
        _lib.check(f(C.byref(prm), C.c_void_p(u.data_ptr()), C.c_void_p(out.data_ptr()), n,
                     float(dx), stream))
        ref = api.rhs_1d(u, dx, prm)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        np.testing.assert_array_equal(a, b)
        r, _ = orc.rhs_1d(u0, dx, sys=orc.SYS_EULER1 if system == "euler" else orc.SYS_ADV,
                          bc=orc.BC_TRANSMISSIVE if system == "euler" else orc.BC_PERIODIC)
        err = max(np.abs(a[c] - r[c]).max() / np.abs(r[c]).max() for c in range(r.shape[0]))
        assert err <= 1e-12, err


def test_rhs_1d_noalloc_rejects_bad_sizes():
    from paper_2004_07954_amd import _lib, api
    L = _lib.lib()
    f = _noalloc(L)
    prm = api.params("euler")
    assert f(C.byref(prm), C.c_void_p(256), C.c_void_p(512), 5, 0.1, None) == _lib.WZN_ERR_SIZE
    assert f(C.byref(prm), C.c_void_p(256), C.c_void_p(512), (1 << 30) + 1, 0.1, None) == \
        _lib.WZN_ERR_SIZE

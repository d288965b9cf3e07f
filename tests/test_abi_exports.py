"""The C ABI library loads and exports every symbol include/wenozn.h declares (no GPU
needed: nothing here launches a kernel)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "wenozn.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(wzn_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    for s in ("wzn_rhs_1d", "wzn_rk3_run_1d", "wzn_rk3_step_1d", "wzn_workspace_bytes"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2004_07954_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libwenozn.so not built; run __graft_entry__.build()")
    L = _lib.lib()
    for s in declared_symbols():
        assert hasattr(L, s), s
    names = {name for name, _, _ in _lib.SIGNATURES}
    assert set(declared_symbols()) == names


def test_host_only_calls():
    """Entry points that touch no device memory: defaults, status strings, workspace size,
    and argument validation (rejected before any launch)."""
    import ctypes as C
    from paper_2004_07954_amd import _lib
    L = _lib.lib()
    p = _lib.WznParams()
    L.wzn_default_params(C.byref(p), _lib.WZN_EULER)
    assert p.abi_version == _lib.WZN_ABI_VERSION and p.A == 10.0 and p.eps == 1e-40
    assert p.p_C == 2 and p.q == 1 and p.gamma == 1.4
    assert L.wzn_status_string(0) == b"ok"
    assert L.wzn_status_string(_lib.WZN_ERR_NONFINITE) == b"non-finite output"
    assert L.wzn_workspace_bytes(C.byref(p), 1 << 20, 1) >= 256
    # n < 6 is rejected before anything is enqueued
    rc = L.wzn_rhs_1d(C.byref(p), C.c_void_p(256), C.c_void_p(512), 5, 0.1, C.c_void_p(1024),
                      None)
    assert rc == _lib.WZN_ERR_SIZE and b"n = 5" in L.wzn_last_error()
    p.q = 2
    rc = L.wzn_rhs_1d(C.byref(p), C.c_void_p(256), C.c_void_p(512), 100, 0.1,
                      C.c_void_p(1024), None)
    assert rc == _lib.WZN_ERR_UNSUPPORTED
    p.q = 1
    rc = L.wzn_rhs_1d(C.byref(p), C.c_void_p(256), C.c_void_p(512), 100, 0.1,
                      C.c_void_p(1000), None)
    assert rc == _lib.WZN_ERR_ARG  # unaligned workspace
    p.debug_nonfinite = 2
    rc = L.wzn_rhs_1d(C.byref(p), C.c_void_p(256), C.c_void_p(512), 100, 0.1,
                      C.c_void_p(1024), None)
    assert rc == _lib.WZN_ERR_ARG and b"debug_nonfinite" in L.wzn_last_error()
    p.debug_nonfinite = 0


@pytest.mark.parametrize("dtype,eps,ok", [
    (0, 1e-60, True), (0, 1e50, True), (0, 1e-40, True),
    (0, 1e-61, False), (0, 1e-64, False), (0, 1e51, False), (0, 0.0, False),
    (0, float("nan"), False), (0, float("inf"), False),
    (1, 1e-36, True), (1, 1e-30, True), (1, 1e30, True),
    (1, 1e-37, False), (1, 1e-40, False), (1, 1e31, False)])
def test_eps_range_rejected_before_launch(dtype, eps, ok):
    """The weights' product form needs (16 eps)^5 to stay a normal double in fp64 (and 16 eps
    a normal float in fp32): eps outside [1e-60, 1e50] (fp64) or [1e-36, 1e30] (fp32) is
    rejected with WZN_ERR_ARG before anything is enqueued.  An accepted eps fails later, on the
    grid size (n = 5), so no call here launches a kernel."""
    import ctypes as C
    from paper_2004_07954_amd import _lib
    L = _lib.lib()
    p = _lib.WznParams()
    L.wzn_default_params(C.byref(p), _lib.WZN_EULER)
    p.eps = eps
    p.dtype = dtype
    if dtype == _lib.WZN_FP64:
        rc = L.wzn_rhs_1d(C.byref(p), C.c_void_p(256), C.c_void_p(512), 5, 0.1,
                          C.c_void_p(1024), None)
    else:
        rc = L.wzn_rhs_2d(C.byref(p), C.c_void_p(256), C.c_void_p(512), 5, 5, 0.1, 0.1,
                          C.c_void_p(1024), None)
    if ok:
        assert rc == _lib.WZN_ERR_SIZE, L.wzn_last_error()
    else:
        assert rc == _lib.WZN_ERR_ARG and b"eps" in L.wzn_last_error(), L.wzn_last_error()


def test_row_tuning_host_calls():
    """Launch-shape override: valid shapes are accepted and reported back, unknown ones are
    rejected, (0, 0) restores the size-based choice; over-long rows are rejected."""
    import ctypes as C
    from paper_2004_07954_amd import _lib, autotune
    from paper_2004_07954_amd._lib import WznError
    try:
        autotune.set_row_tuning(0, 0)
        assert autotune.get_row_tuning(3, 1 << 20) == (256, 4, 1)
        assert autotune.get_row_tuning(3, 65536) == (256, 2, 0)
        assert autotune.get_row_tuning(3, 1 << 18) == (256, 2, 1)
        assert autotune.get_row_tuning(3, 1000) == (256, 1, 0)
        assert autotune.get_row_tuning(1, 200) == (64, 4, 0)
        for shape in autotune.ROW_SHAPES:
            autotune.set_row_tuning(*shape)
            assert autotune.get_row_tuning(3, 12345) == shape
        for shape in [(96, 4, 0), (256, 8, 1), (128, 8, 1), (64, 2, 1), (256, 4, 2)]:
            with pytest.raises(WznError):
                autotune.set_row_tuning(*shape)
        with pytest.raises(WznError):
            autotune.get_row_tuning(2, 100)
    finally:
        autotune.set_row_tuning(0, 0)
    L = _lib.lib()
    p = _lib.WznParams()
    L.wzn_default_params(C.byref(p), _lib.WZN_EULER)
    rc = L.wzn_rhs_1d(C.byref(p), C.c_void_p(256), C.c_void_p(512), (1 << 30) + 1, 0.1,
                      C.c_void_p(1024), None)
    assert rc == _lib.WZN_ERR_SIZE

"""Argument checks of every compute entry point of the C ABI (include/wenozn.h): each invalid
call below is rejected with its documented status before anything is enqueued, so these run
without a GPU.  The pointers are never dereferenced: the checks fail first."""
import ctypes as C

import pytest

from paper_2004_07954_amd import _lib

P, Q, R, WS = C.c_void_p(1 << 20), C.c_void_p(2 << 20), C.c_void_p(3 << 20), C.c_void_p(4 << 20)
NULL = None


def _params(**kw):
    p = _lib.WznParams()
    _lib.lib().wzn_default_params(C.byref(p), kw.pop("system", _lib.WZN_EULER))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _call(name, p, *args):
    L = _lib.lib()
    return getattr(L, name)(C.byref(p) if p is not None else None, *args)


E = _lib
CASES = [
    # (id, entry point, params overrides, arguments after params, expected status)
    ("rhs1d-null-params", "wzn_rhs_1d", None, (P, Q, 100, 0.1, WS, NULL), E.WZN_ERR_ARG),
    ("rhs1d-abi-version", "wzn_rhs_1d", {"abi_version": 1}, (P, Q, 100, 0.1, WS, NULL),
     E.WZN_ERR_ARG),
    ("rhs1d-system", "wzn_rhs_1d", {"system": 7}, (P, Q, 100, 0.1, WS, NULL), E.WZN_ERR_ARG),
    ("rhs1d-fp32", "wzn_rhs_1d", {"dtype": E.WZN_FP32}, (P, Q, 100, 0.1, WS, NULL),
     E.WZN_ERR_DTYPE),
    ("rhs1d-bc", "wzn_rhs_1d", {"bc_x": 5}, (P, Q, 100, 0.1, WS, NULL), E.WZN_ERR_ARG),
    ("rhs1d-gamma", "wzn_rhs_1d", {"gamma": 1.0}, (P, Q, 100, 0.1, WS, NULL), E.WZN_ERR_ARG),
    ("rhs1d-A", "wzn_rhs_1d", {"A": 0.0}, (P, Q, 100, 0.1, WS, NULL), E.WZN_ERR_ARG),
    ("rhs1d-pC", "wzn_rhs_1d", {"p_C": 1}, (P, Q, 100, 0.1, WS, NULL), E.WZN_ERR_UNSUPPORTED),
    ("rhs1d-split-sw", "wzn_rhs_1d", {"flux_split": E.WZN_SPLIT_SW},
     (P, Q, 100, 0.1, WS, NULL), E.WZN_ERR_UNSUPPORTED),
    ("rhs1d-split-unknown", "wzn_rhs_1d", {"flux_split": 9}, (P, Q, 100, 0.1, WS, NULL),
     E.WZN_ERR_ARG),
    ("rhs1d-weights-unknown", "wzn_rhs_1d", {"weights": 9}, (P, Q, 100, 0.1, WS, NULL),
     E.WZN_ERR_ARG),
    ("rhs1d-n-too-big", "wzn_rhs_1d", {}, (P, Q, (1 << 30) + 1, 0.1, WS, NULL), E.WZN_ERR_SIZE),
    ("rhs1d-dx-zero", "wzn_rhs_1d", {}, (P, Q, 100, 0.0, WS, NULL), E.WZN_ERR_ARG),
    ("rhs1d-dx-nan", "wzn_rhs_1d", {}, (P, Q, 100, float("nan"), WS, NULL), E.WZN_ERR_ARG),
    ("rhs1d-ws-null", "wzn_rhs_1d", {}, (P, Q, 100, 0.1, NULL, NULL), E.WZN_ERR_ARG),
    ("rhs1d-u-null", "wzn_rhs_1d", {}, (NULL, Q, 100, 0.1, WS, NULL), E.WZN_ERR_ARG),
    ("rhs1d-alias", "wzn_rhs_1d", {}, (P, P, 100, 0.1, WS, NULL), E.WZN_ERR_ARG),
    ("rhs1d-advection-speed", "wzn_rhs_1d", {"system": E.WZN_ADVECTION, "adv_speed": 0.0},
     (P, Q, 100, 0.1, WS, NULL), E.WZN_ERR_ARG),
    ("reconstruct-m-negative", "wzn_reconstruct", {}, (P, Q, -1, NULL), E.WZN_ERR_SIZE),
    ("reconstruct-null", "wzn_reconstruct", {}, (NULL, Q, 10, NULL), E.WZN_ERR_ARG),
    ("speed1d-advection", "wzn_speed_max_1d", {"system": E.WZN_ADVECTION},
     (P, 100, Q, WS, NULL), E.WZN_ERR_ARG),
    ("run1d-nsteps", "wzn_rk3_run_1d", {}, (P, Q, 100, 0.1, 0.5, -1, NULL, NULL, NULL, NULL, WS,
                                            NULL), E.WZN_ERR_ARG),
    ("run1d-cfl", "wzn_rk3_run_1d", {}, (P, Q, 100, 0.1, 0.0, 3, NULL, NULL, NULL, NULL, WS,
                                         NULL), E.WZN_ERR_ARG),
    ("run1d-stage-null", "wzn_rk3_run_1d", {}, (P, NULL, 100, 0.1, 0.5, 3, NULL, NULL, NULL,
                                                NULL, WS, NULL), E.WZN_ERR_ARG),
    ("rhs1d-char-advection", "wzn_rhs_1d_char", {"system": E.WZN_ADVECTION},
     (P, Q, 100, 0.1, NULL, WS, NULL), E.WZN_ERR_ARG),
    ("run1d-char-nsteps", "wzn_rk3_run_1d_char", {}, (P, Q, 100, 0.1, 0.5, -2, NULL, NULL, NULL,
                                                      NULL, WS, NULL), E.WZN_ERR_ARG),
    ("rhs2d-nx-small", "wzn_rhs_2d", {}, (P, Q, 5, 100, 0.1, 0.1, WS, NULL), E.WZN_ERR_SIZE),
    ("rhs2d-ny-small", "wzn_rhs_2d", {}, (P, Q, 100, 5, 0.1, 0.1, WS, NULL), E.WZN_ERR_SIZE),
    ("rhs2d-nx-big", "wzn_rhs_2d", {}, (P, Q, (1 << 24) + 1, 6, 0.1, 0.1, WS, NULL),
     E.WZN_ERR_SIZE),
    ("rhs2d-cells-big", "wzn_rhs_2d", {}, (P, Q, 1 << 19, 1 << 18, 0.1, 0.1, WS, NULL),
     E.WZN_ERR_SIZE),
    ("rhs2d-advection", "wzn_rhs_2d", {"system": E.WZN_ADVECTION}, (P, Q, 100, 100, 0.1, 0.1,
                                                                    WS, NULL), E.WZN_ERR_ARG),
    ("rhs2d-dy", "wzn_rhs_2d", {}, (P, Q, 100, 100, 0.1, -0.1, WS, NULL), E.WZN_ERR_ARG),
    ("rhs2d-bc-y", "wzn_rhs_2d", {"bc_y": 3}, (P, Q, 100, 100, 0.1, 0.1, WS, NULL),
     E.WZN_ERR_ARG),
    ("rhs2d-weights-z", "wzn_rhs_2d", {"weights": E.WZN_WEIGHTS_Z},
     (P, Q, 100, 100, 0.1, 0.1, WS, NULL), E.WZN_ERR_UNSUPPORTED),
    ("strip-lf-needs-alphas", "wzn_rhs_2d_strip", {}, (P, Q, R, WS, 100, 100, 0.1, 0.1, NULL,
                                                       WS, NULL), E.WZN_ERR_ARG),
    ("run2d-nsteps", "wzn_rk3_run_2d", {}, (P, Q, 100, 100, 0.1, 0.1, 0.5, -1, NULL, NULL, WS,
                                            NULL), E.WZN_ERR_ARG),
    ("rhs2d-char-fp32", "wzn_rhs_2d_char", {"dtype": E.WZN_FP32, "eps": 1e-30},
     (P, Q, R, 100, 100, 0.1, 0.1, NULL, WS, NULL), E.WZN_ERR_DTYPE),
    ("rhs2d-char-sw", "wzn_rhs_2d_char", {"flux_split": E.WZN_SPLIT_SW},
     (P, Q, R, 100, 100, 0.1, 0.1, NULL, WS, NULL), E.WZN_ERR_UNSUPPORTED),
    ("rhs2d-char-work-null", "wzn_rhs_2d_char", {}, (P, Q, NULL, 100, 100, 0.1, 0.1, NULL, WS,
                                                     NULL), E.WZN_ERR_ARG),
    ("run2d-char-alias", "wzn_rk3_run_2d_char", {}, (P, Q, Q, 100, 100, 0.1, 0.1, 0.5, 2, NULL,
                                                     NULL, WS, NULL), E.WZN_ERR_ARG),
    ("batched-batch-zero", "wzn_batched_rk3_run_1d", {},
     (P, Q, 1000, R, WS, NULL, 0, 5, 0.5, NULL, NULL, WS, NULL), E.WZN_ERR_ARG),
    ("batched-frozen-alpha", "wzn_batched_rk3_run_1d", {"lf_alpha_x": 2.0},
     (P, Q, 1000, R, WS, NULL, 4, 5, 0.5, NULL, NULL, WS, NULL), E.WZN_ERR_UNSUPPORTED),
    ("batched-cfl", "wzn_batched_rk3_run_1d", {},
     (P, Q, 1000, R, WS, NULL, 4, 5, 0.0, NULL, NULL, WS, NULL), E.WZN_ERR_ARG),
    ("vjp-alias", "wzn_rhs_1d_vjp", {}, (P, Q, P, 100, 0.1, WS, NULL), E.WZN_ERR_ARG),
    ("vjp-advection", "wzn_rhs_1d_vjp", {"system": E.WZN_ADVECTION},
     (P, Q, R, 100, 0.1, WS, NULL), E.WZN_ERR_ARG),
    ("adjoint-ckpt-every", "wzn_rk3_adjoint_1d", {}, (P, 10, 0, Q, R, WS, P, 100, 0.1, WS,
                                                      NULL), E.WZN_ERR_ARG),
]


@pytest.mark.parametrize("name,entry,over,args,status", CASES, ids=[c[0] for c in CASES])
def test_rejected_before_launch(name, entry, over, args, status):
    L = _lib.lib()
    p = None if over is None else _params(**over)
    rc = _call(entry, p, *args)
    assert rc == status, (rc, L.wzn_last_error())
    assert L.wzn_last_error(), "no error message"

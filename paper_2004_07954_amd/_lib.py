"""ctypes loader of libwenozn.so: argument types of every exported entry point.

The library is built in-tree by ``paper_2004_07954_amd/build.py`` (``__graft_entry__.build``).
There is no fallback: if the shared library is missing, importing the binding raises.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwenozn.so")

WZN_ABI_VERSION = 2
WZN_OK, WZN_ERR_ARG, WZN_ERR_SIZE, WZN_ERR_DTYPE, WZN_ERR_HIP = 0, 1, 2, 3, 4
WZN_ERR_NONFINITE = 5
WZN_ERR_UNSUPPORTED = 6
WZN_ERR_NONPHYSICAL = 7
WZN_ERR_RANGE = 8
WZN_ADVECTION, WZN_EULER = 0, 1
WZN_FP64, WZN_FP32 = 0, 1
WZN_PERIODIC, WZN_TRANSMISSIVE = 0, 1
WZN_SPLIT_LF, WZN_SPLIT_SW = 0, 1
WZN_WEIGHTS_ZN, WZN_WEIGHTS_Z = 0, 1


class WznParams(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("system", C.c_int32), ("dtype", C.c_int32),
                ("bc_x", C.c_int32), ("bc_y", C.c_int32), ("p_C", C.c_int32), ("q", C.c_int32),
                ("flux_split", C.c_int32), ("adv_speed", C.c_double), ("gamma", C.c_double),
                ("A", C.c_double), ("eps", C.c_double), ("lf_alpha_x", C.c_double),
                ("lf_alpha_y", C.c_double), ("weights", C.c_int32), ("debug_nonfinite", C.c_int32)]


class WznBatchTuning(C.Structure):
    _fields_ = [("nt", C.c_int32), ("k", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("layout", C.c_int32)]


# (name, restype, argtypes) of every symbol include/wenozn.h declares
_P, _D, _I32, _I64, _SZ = C.c_void_p, C.c_double, C.c_int32, C.c_int64, C.c_size_t
_PP = C.POINTER(WznParams)
SIGNATURES = [
    ("wzn_default_params", None, [_PP, _I32]),
    ("wzn_abi_version", _I32, []),
    ("wzn_status_string", C.c_char_p, [_I32]),
    ("wzn_last_error", C.c_char_p, []),
    ("wzn_set_row_tuning", _I32, [_I32, _I32, _I32]),
    ("wzn_get_row_tuning", _I32, [_I32, _I64, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int32)]),
    ("wzn_workspace_bytes", _SZ, [_PP, _I64, _I64]),
    ("wzn_reconstruct", _I32, [_PP, _P, _P, _I64, _P]),
    ("wzn_rhs_1d", _I32, [_PP, _P, _P, _I64, _D, _P, _P]),
    ("wzn_rhs_1d_noalloc", _I32, [_PP, _P, _P, _I64, _D, _P]),
    ("wzn_speed_max_1d", _I32, [_PP, _P, _I64, _P, _P, _P]),
    ("wzn_rhs_1d_slab", _I32, [_PP, _P, _P, _P, _P, _I64, _D, _P, _P, _P]),
    ("wzn_rk3_run_1d", _I32, [_PP, _P, _P, _I64, _D, _D, _I32, _P, _P, _P, _P, _P, _P]),
    ("wzn_rk3_step_1d", _I32, [_PP, _P, _P, _I64, _D, _D, _P, _P, _P, _P]),
    ("wzn_rhs_1d_char", _I32, [_PP, _P, _P, _I64, _D, _P, _P, _P]),
    ("wzn_rk3_run_1d_char", _I32, [_PP, _P, _P, _I64, _D, _D, _I32, _P, _P, _P, _P, _P, _P]),
    ("wzn_char2d_work_doubles", _I64, [_I64, _I64]),
    ("wzn_rhs_2d_char", _I32, [_PP, _P, _P, _P, _I64, _I64, _D, _D, _P, _P, _P]),
    ("wzn_rk3_run_2d_char", _I32, [_PP, _P, _P, _P, _I64, _I64, _D, _D, _D, _I32, _P, _P, _P,
                                   _P]),
    ("wzn_rhs_2d", _I32, [_PP, _P, _P, _I64, _I64, _D, _D, _P, _P]),
    ("wzn_speed_max_2d", _I32, [_PP, _P, _I64, _I64, _P, _P, _P]),
    ("wzn_rhs_2d_strip", _I32, [_PP, _P, _P, _P, _P, _I64, _I64, _D, _D, _P, _P, _P]),
    ("wzn_rk3_run_2d", _I32, [_PP, _P, _P, _I64, _I64, _D, _D, _D, _I32, _P, _P, _P, _P]),
    ("wzn_rk3_step_2d", _I32, [_PP, _P, _P, _I64, _I64, _D, _D, _D, _P, _P, _P, _P]),
    ("wzn_batched_rk3_run_1d", _I32, [_PP, _P, _P, _I64, _P, _P, _P, _I32, _I32, _D,
                                      C.POINTER(WznBatchTuning), _P, _P, _P]),
    ("wzn_rhs_1d_vjp", _I32, [_PP, _P, _P, _P, _I64, _D, _P, _P]),
    ("wzn_rk3_step_1d_vjp", _I32, [_PP, _P, _P, _P, _P, _I64, _D, _P, _P, _P, _P]),
    ("wzn_rk3_adjoint_1d_work_doubles", _I64, [_I64, _I32]),
    ("wzn_rk3_adjoint_1d", _I32, [_PP, _P, _I32, _I32, _P, _P, _P, _P, _I64, _D, _P, _P]),
]

_LIB = None


class WznError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libwenozn status %d (%s)" % (code, msg))
        self.code = code


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libwenozn.so is not built: run __graft_entry__.build() "
                              "(expected at %s)" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        if L.wzn_abi_version() != WZN_ABI_VERSION:
            raise ImportError("libwenozn ABI version mismatch")
        _LIB = L
    return _LIB


def check(code):
    if code != WZN_OK:
        L = lib()
        msg = L.wzn_last_error().decode() or L.wzn_status_string(code).decode()
        raise WznError(code, msg)

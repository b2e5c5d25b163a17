"""ctypes declarations of the C-ABI in ``include/mpk.h`` (argument marshalling only).

The library is loaded from this package directory.  If it is missing the
import fails loudly: there is no CPU fallback anywhere in the package.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libmpk.so")

MPK_MAX_POWER = 32
MPK_MAX_NRHS = 32
MPK_SYNC_NODE = 0
MPK_SYNC_WAVEFRONT = 1
MPK_NUM_FEATURES = 24

STATUS = {0: "MPK_OK", -1: "MPK_ERR_ARG", -2: "MPK_ERR_CSR", -3: "MPK_ERR_OOM", -4: "MPK_ERR_HIP",
          -5: "MPK_ERR_TIMEOUT", -6: "MPK_ERR_UNSUPPORTED", -7: "MPK_ERR_STATE"}
DTYPES = {"f64": 0, "f32": 1, "bf16": 2}


class MpkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class mpk_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.POINTER(ctypes.c_int64)),
                ("col", ctypes.POINTER(ctypes.c_int32)),
                ("val", ctypes.POINTER(ctypes.c_double))]


class mpk_options(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("safety_factor", ctypes.c_double),
                ("root_mode", ctypes.c_int32), ("val_dtype", ctypes.c_int32),
                ("nrhs", ctypes.c_int32), ("workgroups", ctypes.c_int32),
                ("tile_nnz", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("watchdog_spins", ctypes.c_int64), ("budget_vectors", ctypes.c_int32),
                ("skew", ctypes.c_int32), ("xcd_streams", ctypes.c_int32),
                ("plan_on_device", ctypes.c_int32), ("force_acquire", ctypes.c_int32),
                ("recursion_stages", ctypes.c_int32), ("accum_f64", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class mpk_plan_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("p", ctypes.c_int32),
                ("nrhs", ctypes.c_int32), ("n_levels", ctypes.c_int64), ("n_groups", ctypes.c_int64),
                ("n_tiles", ctypes.c_int64), ("n_tickets", ctypes.c_int64), ("root", ctypes.c_int64),
                ("max_level_rows", ctypes.c_int64), ("max_group_nnz", ctypes.c_int64),
                ("violating_groups", ctypes.c_int64), ("device_bytes", ctypes.c_uint64),
                ("workgroups", ctypes.c_int32), ("n_chunks", ctypes.c_int32),
                ("tile_nnz", ctypes.c_int32), ("val_dtype", ctypes.c_int32),
                ("plan_seconds", ctypes.c_double), ("phase_seconds", ctypes.c_double * 4),
                ("line_closed_deps", ctypes.c_int32), ("last_run_fenced", ctypes.c_int32),
                ("recursive", ctypes.c_int32), ("max_stage", ctypes.c_int32),
                ("n_units", ctypes.c_int64), ("n_dep_ranges", ctypes.c_int64)]


class mpk_recurrence(ctypes.Structure):
    _fields_ = [("alpha", ctypes.POINTER(ctypes.c_double)), ("beta", ctypes.POINTER(ctypes.c_double)),
                ("gamma", ctypes.POINTER(ctypes.c_double)), ("coef", ctypes.POINTER(ctypes.c_double)),
                ("complex_pairs", ctypes.c_int32), ("y_prev", ctypes.c_void_p),
                ("acc", ctypes.c_void_p), ("coef0", ctypes.POINTER(ctypes.c_double))]


_P = ctypes.c_void_p
_I32P = ctypes.POINTER(ctypes.c_int32)
_I64P = ctypes.POINTER(ctypes.c_int64)
_F64P = ctypes.POINTER(ctypes.c_double)

# name -> (restype, argtypes); every symbol declared in include/mpk.h
SIGNATURES = {
    "mpk_options_default": (None, [ctypes.POINTER(mpk_options)]),
    "mpk_plan_create": (ctypes.c_int32, [ctypes.POINTER(mpk_csr), ctypes.c_int32, ctypes.c_uint64,
                                         ctypes.POINTER(mpk_options), ctypes.POINTER(_P)]),
    "mpk_plan_create_device": (ctypes.c_int32, [ctypes.POINTER(mpk_csr), ctypes.c_int32, ctypes.c_uint64,
                                         ctypes.POINTER(mpk_options), ctypes.POINTER(_P)]),
    "mpk_plan_retune": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_uint64, ctypes.POINTER(mpk_options)]),
    "mpk_plan_query": (ctypes.c_int32, [_P, ctypes.POINTER(mpk_plan_info)]),
    "mpk_plan_arrays": (ctypes.c_int32, [_P, _I32P, _I32P, _I32P, _I32P]),
    "mpk_plan_matrix": (ctypes.c_int32, [_P, _I64P, _I32P, _F64P]),
    "mpk_plan_tiles": (ctypes.c_int32, [_P, _I32P, _I32P, _I32P, _I32P]),
    "mpk_plan_tile_deps": (ctypes.c_int32, [_P, _I32P, ctypes.c_int32]),
    "mpk_plan_units": (ctypes.c_int32, [_P, _I32P, _I32P, _I32P, _I32P]),
    "mpk_plan_features": (ctypes.c_int32, [_P, _F64P]),
    "mpk_plan_upload": (ctypes.c_int32, [_P]),
    "mpk_permute": (ctypes.c_int32, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P]),
    "mpk_run": (ctypes.c_int32, [_P, _P, _P, ctypes.POINTER(mpk_recurrence), _P]),
    "mpk_run_baseline": (ctypes.c_int32, [_P, _P, _P, ctypes.POINTER(mpk_recurrence), _P]),
    "mpk_run_first": (ctypes.c_int32, [_P, ctypes.c_int32, _P, _P, ctypes.POINTER(mpk_recurrence), _P]),
    "mpk_run_baseline_first": (ctypes.c_int32, [_P, ctypes.c_int32, _P, _P, ctypes.POINTER(mpk_recurrence), _P]),
    "mpk_run_sync": (ctypes.c_int32, [_P, _P, _P, ctypes.c_int32, _P]),
    "mpk_plan_status": (ctypes.c_int32, [_P, _P]),
    "mpk_plan_destroy": (None, [_P]),
    "spmv_create": (ctypes.c_int32, [ctypes.POINTER(mpk_csr), ctypes.POINTER(mpk_options),
                                     ctypes.POINTER(_P)]),
    "spmv_run": (ctypes.c_int32, [_P, _P, _P, _P]),
    "spmv_powers_run": (ctypes.c_int32, [_P, ctypes.c_int32, _P, _P, _P]),
    "spmv_destroy": (None, [_P]),
    "mpk_bw_probe": (ctypes.c_int32, [_P, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, _P, _P]),
    "mpk_bw_probe_ex": (ctypes.c_int32, [_P, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, _P, _P]),
    "mpk_xcd_ids": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int64, _P]),
    "mpk_hop_probe": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _P,
                                       _I32P, _P]),
    "mpk_mlp_param_count": (ctypes.c_int64, [ctypes.c_int32, ctypes.c_int32]),
    "mpk_mlp_forward": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int32, _P, _P, _P]),
    "mpk_mlp_backward": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, _P, _P, ctypes.c_int32, _P, _P, _P,
                                          _P, _P, _P]),
    "mpk_mlp_backward_noalloc": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, _P, _P, ctypes.c_int32, _P,
                                                  _P, _P, _P, _P]),
    "mpk_mlp_adam": (ctypes.c_int32, [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_float, ctypes.c_int32, _P]),
    "mpk_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "mpk_last_error": (ctypes.c_char_p, []),
    "mpk_version": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError(f"{LIBPATH} not found: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIBPATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != 0:
        msg = lib().mpk_last_error()
        raise MpkError(status, msg.decode() if msg else "")


def default_options(**kw) -> mpk_options:
    o = mpk_options()
    lib().mpk_options_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "val_dtype" and isinstance(v, str):
            v = DTYPES[v]
        setattr(o, k, v)
    return o

"""ctypes loader for ``libldbp.so`` (the in-tree gfx950 HIP library).

The library must have been built (``python -m paper_2010_14258_amd.build`` or
``__graft_entry__.build()``); there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libldbp.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "ldbp.h")

c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_size_t = ctypes.c_size_t
c_void_p = ctypes.c_void_p
c_uint64 = ctypes.c_uint64
c_double = ctypes.c_double
P_i32 = ctypes.POINTER(ctypes.c_int32)
P_i64 = ctypes.POINTER(ctypes.c_int64)
P_f64 = ctypes.POINTER(ctypes.c_double)
P_size = ctypes.POINTER(ctypes.c_size_t)

LDBP_OK, LDBP_EINVAL, LDBP_EWORKSPACE, LDBP_EUNSUPPORTED, LDBP_EHIP, LDBP_ENONFINITE = 0, -1, -2, -3, -4, -5
LDBP_C64, LDBP_C128 = 0, 1
LDBP_NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024


class LdbpPlan(ctypes.Structure):
    _fields_ = [("steps_per_pass", c_int32), ("chunks", c_int32), ("outputs_per_thread", c_int32),
                ("flags", c_int32)]


LDBP_PLAN_SYMMETRIC = 1
LDBP_PLAN_ONE_STREAM = 2
LDBP_PLAN_GUARD = 4
LDBP_EDGE_ZERO = 1
LDBP_EDGE_VALID = 2


P_plan = ctypes.POINTER(LdbpPlan)


class SsmLink(ctypes.Structure):
    _fields_ = [("fs", c_double), ("alpha", c_double), ("beta2", c_double), ("gamma", c_double),
                ("span_len", c_double), ("kerr_scale", c_double), ("ase_var", c_double),
                ("nspan", c_int32), ("nstep", c_int32), ("step_len", P_f64), ("edfa_gain", c_int32),
                ("reserved", c_int32)]


P_link = ctypes.POINTER(SsmLink)

# name -> (restype, argtypes)
SIGNATURES = {
    "ldbp_version": (ctypes.c_char_p, []),
    "ldbp_status_string": (ctypes.c_char_p, [c_int32]),
    "ldbp_last_error": (ctypes.c_char_p, []),
    "ldbp_forward_workspace_size": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_int32, P_i32, c_void_p,
                                              c_int32, P_plan, P_size]),
    "ldbp_forward": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_int32, P_i32, c_void_p, c_void_p,
                               c_void_p, c_void_p, c_void_p, c_int32, P_plan, c_void_p, c_size_t, c_void_p]),
    "ldbp_forward_noalloc": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_int32, P_i32, c_void_p, c_void_p,
                                       c_void_p, c_void_p, c_void_p, c_int32, P_plan, c_void_p]),
    "ldbp_forward_plan_query": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_int32, P_i32, c_int32, P_plan,
                                          P_i32, P_i32, P_i32]),
    "essm_forward_workspace_size": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_int32, P_i32, P_i32, c_void_p,
                                              c_int32, P_plan, P_size]),
    "essm_forward": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_int32, P_i32, P_i32, c_void_p, c_void_p,
                               c_void_p, c_void_p, c_void_p, c_void_p, c_int32, P_plan, c_void_p, c_size_t,
                               c_void_p]),
    "ldbp_forward_aperiodic_workspace_size": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_int32, P_i32, P_i32,
                                                        c_int32, P_plan, P_size]),
    "ldbp_forward_aperiodic": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_int32, P_i32, P_i32, c_void_p,
                                         c_void_p, c_void_p, c_void_p, c_void_p, c_int32, P_plan, c_void_p, c_size_t,
                                         c_void_p]),
    "essm_forward_plan_query": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_int32, P_i32, P_i32, c_int32,
                                          P_plan, P_i32, P_i32, P_i32]),
    "essm_backward_workspace_size": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_int32, P_i32, P_i32,
                                               c_void_p, c_int32, P_size]),
    "essm_backward": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_int32, P_i32, P_i32, c_void_p, c_void_p,
                                c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                c_void_p, P_plan, c_void_p, c_size_t, c_void_p]),
    "ldbp_backward_workspace_size": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_int32, P_i32, c_void_p,
                                               c_int32, P_size]),
    "ldbp_backward": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_int32, P_i32, c_void_p, c_void_p, c_void_p,
                                c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, P_plan, c_void_p,
                                c_size_t, c_void_p]),
    "ldbp_batch_plan_create": (c_int32, [c_int32, c_int32, c_int32, P_i64, P_i32, P_i32, P_plan,
                                         ctypes.POINTER(c_void_p)]),
    "ldbp_batch_plan_destroy": (c_int32, [c_void_p]),
    "ldbp_batch_plan_info": (c_int32, [c_void_p, P_i64, P_i64, P_i64, P_i64, P_i32, P_i32]),
    "ldbp_batch_forward": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ldbp_batch_forward_graph": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ssm_workspace_size": (c_int32, [c_int32, c_int32, c_int64, c_int64, P_link, P_size]),
    "ssm_channel": (c_int32, [c_int32, c_int32, c_int64, c_int64, P_link, c_void_p, c_void_p, c_void_p, c_void_p,
                              c_size_t, c_void_p]),
    "ssm_batch_plan_create": (c_int32, [c_int32, c_int32, c_int32, P_i64, P_i32, P_link, c_int32,
                                        ctypes.POINTER(c_void_p)]),
    "ssm_batch_plan_destroy": (c_int32, [c_void_p]),
    "ssm_batch_plan_info": (c_int32, [c_void_p, P_i64, P_i64, P_i32, P_i32]),
    "ssm_batch_run": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "fft_dbp": (c_int32, [c_int32, c_int32, c_int64, c_int64, P_link, c_void_p, c_void_p, c_void_p, c_size_t,
                          c_void_p]),
    "ldbp_fft_workspace_size": (c_int32, [c_int32, c_int32, c_int64, c_int64, P_size]),
    "ldbp_fft": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_void_p, c_void_p, c_int32, c_void_p, c_size_t,
                           c_void_p]),
    "tx_shape_workspace_size": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_int32, P_size]),
    "tx_shape": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_int32, c_double, c_double, c_void_p, c_void_p,
                           c_void_p, c_void_p, c_size_t, c_void_p]),
    "tx_shape_symbols": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_int32, c_double, c_double, c_void_p,
                                   c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "rx_lpf_decimate_workspace_size": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_int64, P_size]),
    "rx_lpf_decimate": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_int64, c_void_p, c_void_p, c_void_p,
                                  c_size_t, c_void_p]),
    "rx_mse_workspace_size": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_int32, P_size]),
    "rx_mse": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_int32, c_double, c_double, c_void_p, c_void_p,
                         c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "qam16_symbols": (c_int32, [c_int32, c_int64, c_void_p, c_void_p, c_void_p]),
    "ldbp_randbits": (c_int32, [c_void_p, c_int64, c_uint64, c_uint64, c_void_p]),
    "ldbp_randn": (c_int32, [c_int32, c_void_p, c_int64, c_uint64, c_uint64, c_void_p]),
    "ldbp_sum_rows": (c_int32, [c_int32, c_void_p, c_void_p, c_int64, c_int64, c_void_p]),
    "ldbp_adam": (c_int32, [c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_int32,
                            c_double, c_double, c_double, c_double, c_int64, c_void_p]),
}

_lib = None


class LdbpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ldbp status {status}: {msg}")
        self.status = status


def load():
    """Loads the library once; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(python -m paper_2010_14258_amd.build); there is no CPU fallback")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int):
    if status != LDBP_OK:
        msg = load().ldbp_last_error().decode(errors="replace")
        raise LdbpError(status, msg)


def i32_array(values):
    arr = (c_int32 * len(values))(*[int(v) for v in values])
    return arr

"""ctypes loader for libsystec.so (the C ABI declared in include/systec.h).

The library must have been built in-tree (``python -m
paper_2406_09266_amd.build``). There is no fallback: if it is missing or
fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsystec.so")

STATUS = {0: "SYSTEC_OK", 1: "SYSTEC_EINVAL", 2: "SYSTEC_ENONCANON", 3: "SYSTEC_ENOMEM",
          4: "SYSTEC_EBUDGET", 5: "SYSTEC_EBUSY", 6: "SYSTEC_ETIMEOUT", 7: "SYSTEC_ENOTFOUND",
          8: "SYSTEC_EDEVICE"}
SYSTEC_F32, SYSTEC_BF16 = 0, 1

P = ctypes.c_void_p
I32 = ctypes.c_int
I64 = ctypes.c_int64
PP = ctypes.POINTER(ctypes.c_void_p)
PI64 = ctypes.POINTER(ctypes.c_int64)
PD = ctypes.POINTER(ctypes.c_double)

# name -> argtypes; every function returns int (systec_status) unless listed
# in _RESTYPE.
SIGNATURES = {
    "systec_last_error": [],
    "systec_version": [],
    "systec_ssymv": [I64, I64, P, P, P, P, I32, P, P],
    "systec_syprd": [I64, I64, P, P, P, P, I32, P, P],
    "systec_syprd_noalloc": [I64, I64, P, P, P, P, I32, P, P],
    "systec_bellman_ford": [I64, I64, P, P, P, P, P, P],
    "systec_bellman_ford_t": [P, P, P, P],
    "systec_cp_step": [P, P, I32, I64, P, P, P, P, P],
    "systec_ttm": [I64, I64, PP, P, P, I32, I64, P, I32, P],
    "systec_mttkrp_partial": [I32, I32, P, I64, I64, PP, P, PP, I32, I64, P, P],
    "systec_mttkrp": [I32, I64, I64, PP, P, P, I32, I64, P, P],
    "systec_mttkrp_choose": [I64, I32, I64, I32, P],
    "systec_mttkrp_ex": [I32, I64, I64, PP, P, P, I32, I64, P, I32, P],
    "systec_spmv_csr": [I64, I64, P, P, P, P, I32, P, P],
    "systec_mttkrp_full": [I32, I64, I64, PP, P, P, I32, I64, P, P],
    "systec_expand_csr_size": [I64, I64, P, P, PI64, P],
    "systec_expand_csr": [I64, I64, P, P, P, P, P, P, P],
    "systec_expand_coo_size": [I32, I64, I64, PP, PI64, P],
    "systec_expand_coo": [I32, I64, I64, PP, P, PP, P, P],
    "systec_expansion_stats": [I32, I64, I64, PP, PI64, PI64, P],
    "systec_validate_csr_upper": [I64, I64, P, P, P],
    "systec_validate_coo": [I32, I64, I64, PP, P],
    "systec_canonicalize_coo": [I32, I64, PP, P, PI64],
    "systec_quantize_bf16": [P, P, I64, P],
    "systec_tensor_create_csr": [I64, I64, P, P, P, P, PP],
    "systec_tensor_create_csr_ex": [I64, I64, P, P, P, I32, P, PP],
    "systec_tensor_create_coo": [I32, I64, I64, PP, P, P, PP],
    "systec_tensor_info": [P, ctypes.POINTER(ctypes.c_int), PI64, PI64, PI64,
                           ctypes.POINTER(ctypes.c_uint64)],
    "systec_tensor_vertex_order": [P, ctypes.POINTER(ctypes.c_int), P, P],
    "systec_tensor_bytes": [P, ctypes.POINTER(ctypes.c_uint64)],
    "systec_syprd_t": [P, P, I32, P, P],
    "systec_ssymv_t_ex": [P, P, I32, P, I32, P],
    "systec_syprd_t_ex": [P, P, I32, P, I32, P],
    "systec_tensor_destroy": [P],
    "systec_ssymv_t": [P, P, I32, P, P],
    "systec_mttkrp_t": [P, P, I32, I64, P, P],
    "systec_mttkrp_t_ex": [P, P, I32, I64, P, I32, P],
    "systec_kernel_timing": [I32],
    "systec_kernel_timing_read": [PD, PI64],
}


class ServeConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_int32),
                ("step_work_nnz", ctypes.c_int64), ("device", ctypes.c_int32),
                ("max_queue", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("streams", ctypes.c_int32), ("min_step_work_nnz", ctypes.c_int64)]


class ServeStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "failed", "rejected",
                                             "steps", "queued", "running")] + \
               [(n, ctypes.c_double) for n in ("p50_us", "p99_us", "mean_us", "max_us",
                                              "req_per_s", "eff_nnz_per_s")] + \
               [("bytes_in_use", ctypes.c_uint64)]


SIGNATURES.update({
    "systec_serve_create": [ctypes.POINTER(ServeConfig), PP],
    "systec_serve_register": [P, P, PI64],
    "systec_serve_unregister": [P, I64],
    "systec_serve_submit": [P, I64, P, I32, I64, P, I64, PI64],
    "systec_serve_submit_after": [P, I64, P, I32, I64, P, I64, P, PI64],
    "systec_serve_poll": [P, I64, ctypes.POINTER(ctypes.c_int)],
    "systec_serve_wait": [P, I64, I64],
    "systec_serve_get_stats": [P, ctypes.POINTER(ServeStats)],
    "systec_serve_reset_stats": [P],
    "systec_serve_now_ns": [],
    "systec_serve_destroy": [P],
})
_RESTYPE = {"systec_last_error": ctypes.c_char_p, "systec_version": ctypes.c_char_p,
            "systec_serve_now_ns": ctypes.c_int64}

_lib = None


class SystecError(RuntimeError):
    def __init__(self, fn, status, message):
        self.status = status
        self.status_name = STATUS.get(status, str(status))
        super().__init__(f"{fn}: {self.status_name}: {message}")


def lib():
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} not found: build it with `python -m paper_2406_09266_amd.build`")
        h = ctypes.CDLL(LIB_PATH)
        for name, argtypes in SIGNATURES.items():
            f = getattr(h, name)
            f.argtypes = argtypes
            f.restype = _RESTYPE.get(name, ctypes.c_int)
        _lib = h
    return _lib


def call(name, *args):
    """Calls `name`; raises SystecError on a nonzero status."""
    rc = getattr(lib(), name)(*args)
    if rc != 0:
        msg = lib().systec_last_error().decode(errors="replace")
        raise SystecError(name, rc, msg)
    return rc


def ptr_array(ptrs):
    """A C array of device pointers (for the `const int32_t* const* idx` arguments)."""
    arr = (ctypes.c_void_p * len(ptrs))(*[ctypes.c_void_p(p) for p in ptrs])
    return ctypes.cast(arr, PP), arr  # keep `arr` alive while the pointer is used

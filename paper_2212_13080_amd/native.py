"""ctypes binding of libeqfmm.so (the C ABI in include/eqfmm.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  torch is imported first so that the library binds to the HIP
runtime torch already loaded (same soname), and torch tensors supply the
device memory and the stream.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must be loaded before the library)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeqfmm.so")

FREE, FREE_CONTINUOUS, PERIODIC, PERIODIC_CONTINUOUS = 0, 1, 2, 3
FP64, FP32, FP32_BF16FAR = 0, 1, 2
STAGES = ("bin", "p2m", "m2m", "m2l", "l2l", "leaf", "gather", "adjoint")

_ERR = {0: "EQFMM_OK", -1: "EQFMM_EINVAL", -2: "EQFMM_EBOX", -3: "EQFMM_ENEUTRAL",
        -4: "EQFMM_ENONFINITE", -5: "EQFMM_EWORKSPACE", -6: "EQFMM_EHIP", -7: "EQFMM_ESTATE"}

EXPORTS = ("eqfmm_plan_create", "eqfmm_plan_device_bytes", "eqfmm_plan_upload",
           "eqfmm_workspace_bytes", "eqfmm_forward", "eqfmm_forward_async", "eqfmm_backward",
           "eqfmm_plan_destroy", "eqfmm_strerror", "eqfmm_profile_enable", "eqfmm_profile_read",
           "eqfmm_version")


class EqfmmError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        self.name = _ERR.get(code, str(code))
        msg = lib().eqfmm_strerror(code).decode() if _lib is not None else ""
        super().__init__(f"{where}: {self.name} ({msg})")


class Params(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("order", ctypes.c_int32),
                ("boundary", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("origin", ctypes.c_double * 3), ("box", ctypes.c_double),
                ("split_d", ctypes.c_double), ("node_shrink", ctypes.c_double),
                ("max_fragments", ctypes.c_int64)]


_lib = None
_VP = ctypes.c_void_p


def lib():
    """Load libeqfmm.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        L.eqfmm_plan_create.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(_VP)]
        L.eqfmm_plan_device_bytes.argtypes = [_VP, ctypes.POINTER(ctypes.c_size_t)]
        L.eqfmm_plan_upload.argtypes = [_VP, _VP, ctypes.c_size_t, _VP]
        L.eqfmm_workspace_bytes.argtypes = [_VP, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]
        L.eqfmm_forward.argtypes = [_VP, ctypes.c_int64, _VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP]
        L.eqfmm_forward_async.argtypes = [_VP, ctypes.c_int64, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                          ctypes.c_size_t, _VP]
        L.eqfmm_backward.argtypes = [_VP, ctypes.c_int64, _VP, _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP]
        L.eqfmm_plan_destroy.argtypes = [_VP]
        L.eqfmm_strerror.argtypes = [ctypes.c_int]
        L.eqfmm_strerror.restype = ctypes.c_char_p
        L.eqfmm_profile_enable.argtypes = [_VP, ctypes.c_int]
        L.eqfmm_profile_read.argtypes = [_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]
        L.eqfmm_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def check(rc, where):
    if rc != 0:
        raise EqfmmError(rc, where)


# ----------------------------------------------------------- same-name calls

def eqfmm_plan_create(params: Params):
    h = _VP()
    check(lib().eqfmm_plan_create(ctypes.byref(params), ctypes.byref(h)), "eqfmm_plan_create")
    return h


def eqfmm_plan_device_bytes(plan) -> int:
    b = ctypes.c_size_t()
    check(lib().eqfmm_plan_device_bytes(plan, ctypes.byref(b)), "eqfmm_plan_device_bytes")
    return b.value


def eqfmm_plan_upload(plan, dev_ptr: int, nbytes: int, stream: int):
    check(lib().eqfmm_plan_upload(plan, dev_ptr, nbytes, stream), "eqfmm_plan_upload")


def eqfmm_workspace_bytes(plan, n: int) -> int:
    b = ctypes.c_size_t()
    check(lib().eqfmm_workspace_bytes(plan, n, ctypes.byref(b)), "eqfmm_workspace_bytes")
    return b.value


def eqfmm_forward(plan, n, pos_ptr, q_ptr, phi_ptr, field_ptr, energy_ptr, ws_ptr, ws_bytes, stream):
    check(lib().eqfmm_forward(plan, n, pos_ptr, q_ptr, phi_ptr, field_ptr, energy_ptr, ws_ptr,
                              ws_bytes, stream), "eqfmm_forward")


def eqfmm_forward_async(plan, n, pos_ptr, q_ptr, phi_ptr, field_ptr, energy_ptr, status_ptr, ws_ptr, ws_bytes,
                        stream):
    check(lib().eqfmm_forward_async(plan, n, pos_ptr, q_ptr, phi_ptr, field_ptr, energy_ptr, status_ptr, ws_ptr,
                                    ws_bytes, stream), "eqfmm_forward_async")


def eqfmm_backward(plan, n, q_ptr, grad_ptr, dEdx_ptr, dEdq_ptr, ws_ptr, ws_bytes, stream):
    check(lib().eqfmm_backward(plan, n, q_ptr, grad_ptr, dEdx_ptr, dEdq_ptr, ws_ptr, ws_bytes, stream),
          "eqfmm_backward")


def eqfmm_plan_destroy(plan):
    check(lib().eqfmm_plan_destroy(plan), "eqfmm_plan_destroy")


def eqfmm_profile_enable(plan, stages: int):
    check(lib().eqfmm_profile_enable(plan, int(stages)), "eqfmm_profile_enable")


def eqfmm_profile_read(plan, stage: int):
    ms, cnt = ctypes.c_double(), ctypes.c_int64()
    fl, by = ctypes.c_double(), ctypes.c_double()
    check(lib().eqfmm_profile_read(plan, stage, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(fl),
                                   ctypes.byref(by)), "eqfmm_profile_read")
    return dict(ms=ms.value, launches=cnt.value, flops=fl.value, bytes=by.value)


def eqfmm_version() -> str:
    return lib().eqfmm_version().decode()

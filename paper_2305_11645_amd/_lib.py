"""ctypes prototypes for libqmcred.so (the C ABI declared in include/qmcred.h).

Loading fails loudly when the library has not been built: there is no
fallback of any kind behind these entry points.
"""
from __future__ import annotations

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqmcred.so")

# every symbol include/qmcred.h declares
EXPORTS = [
    "qmc_points_init", "qmc_points_free", "qmc_points_info", "qmc_points_grad_split", "qmc_point_values",
    "qmc_point_matrix", "qmc_workspace_size", "qmc_reduced_matvec", "qmc_estimate",
    "qmc_estimate_static",
    "qmc_estimate_grad", "qmc_status_string", "qmc_last_error", "qmc_timing_enable",
    "qmc_timing_reset", "qmc_timing_read", "qmc_probe_valu", "qmc_probe_mfma",
]

STATUS = {0: "QMC_OK", 1: "QMC_EINVAL", 2: "QMC_EUNSUPPORTED", 3: "QMC_ENOMEM", 4: "QMC_EDEVICE"}


class PointSpec(ct.Structure):
    _fields_ = [("b", ct.c_int32), ("m", ct.c_int32), ("s", ct.c_int32), ("kind", ct.c_int32),
                ("w", ct.POINTER(ct.c_int32)), ("gen", ct.POINTER(ct.c_uint64)),
                ("rand", ct.c_int32), ("R", ct.c_int32),
                ("shift", ct.POINTER(ct.c_double)), ("dshift", ct.POINTER(ct.c_uint64)),
                ("map", ct.c_int32), ("samples", ct.POINTER(ct.c_double))]


class Integrand(ct.Structure):
    _fields_ = [("g", ct.c_int32), ("c", ct.c_double), ("h", ct.c_int32), ("K", ct.c_double)]


_lib = None


def load() -> ct.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libqmcred.so is not built ({LIB_PATH}); run "
                           "`python -m paper_2305_11645_amd.build` first")
    # PyTorch's wheel carries its own HIP runtime under the same soname as the
    # system one.  Importing torch first makes the dynamic linker resolve this
    # library's HIP dependency to the copy torch already loaded, so the process
    # runs one HIP runtime and torch's device pointers and streams are valid
    # here; loaded the other way round, two runtimes would compete for the GPU.
    import torch  # noqa: F401
    L = ct.CDLL(LIB_PATH)
    vp, i32, i64, sz = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_size_t
    L.qmc_points_init.argtypes = [ct.POINTER(vp), ct.POINTER(PointSpec)]
    L.qmc_points_free.argtypes = [vp]
    L.qmc_points_info.argtypes = [vp, ct.POINTER(i64), ct.POINTER(i32), ct.POINTER(i32),
                                  ct.POINTER(i32), ct.POINTER(i64)]
    L.qmc_points_grad_split.argtypes = [vp, ct.POINTER(i32)]
    L.qmc_point_values.argtypes = [vp, i32, i32, vp, vp]
    L.qmc_point_matrix.argtypes = [vp, i32, vp, i64, vp]
    L.qmc_workspace_size.argtypes = [vp, i32, i32, ct.POINTER(Integrand), i32, ct.POINTER(sz)]
    L.qmc_reduced_matvec.argtypes = [vp, i32, vp, i32, i64, i32, vp, i64, vp, sz, vp]
    L.qmc_estimate.argtypes = [vp, vp, i32, i64, ct.POINTER(Integrand), i32, vp, vp, sz, vp]
    L.qmc_estimate_static.argtypes = [vp, vp, i32, i64, ct.POINTER(Integrand), i32, vp, vp]
    L.qmc_estimate_grad.argtypes = [vp, vp, i32, i64, ct.POINTER(Integrand), i32, vp, vp, vp, sz, vp]
    L.qmc_status_string.argtypes = [i32]
    L.qmc_status_string.restype = ct.c_char_p
    L.qmc_last_error.restype = ct.c_char_p
    L.qmc_timing_enable.argtypes = [i32]
    L.qmc_timing_read.argtypes = [ct.c_char_p, ct.POINTER(ct.c_double), ct.POINTER(i64)]
    L.qmc_probe_valu.argtypes = [ct.POINTER(ct.c_double)] * 3 + [vp]
    L.qmc_probe_mfma.argtypes = [ct.POINTER(ct.c_double)] * 3 + [vp]
    for name in EXPORTS:
        if name not in ("qmc_status_string", "qmc_last_error"):
            getattr(L, name).restype = ct.c_int32
    _lib = L
    return L


class QMCError(RuntimeError):
    """A libqmcred call returned a non-zero status."""

    def __init__(self, status: int, detail: str):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {detail}")


class QMCInvalid(QMCError, ValueError):
    pass


class QMCUnsupported(QMCError, NotImplementedError):
    pass


class QMCNoMemory(QMCError, MemoryError):
    pass


class QMCDeviceError(QMCError):
    pass


_EXC = {1: QMCInvalid, 2: QMCUnsupported, 3: QMCNoMemory, 4: QMCDeviceError}


def check(status: int) -> None:
    if status != 0:
        detail = load().qmc_last_error().decode(errors="replace")
        raise _EXC.get(status, QMCError)(status, detail)

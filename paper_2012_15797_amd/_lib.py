"""ctypes binding of libgfc.so (include/gfc.h).  Argument marshalling only:
every step of the render runs in the library's HIP kernels.

The HIP runtime that torch loads and the one libgfc.so links share one soname
(libamdhip64.so.7), so torch is imported first and the library then binds to
the same runtime: torch's device pointers and streams are valid in it.
"""

from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (load torch's HIP runtime before libgfc.so)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgfc.so")

GFC_KMAX = 16
GFC_FORCE_FOURIER = 1
GFC_FORCE_REAL = 2
GFC_RAMP_LINEAR = 4
GFC_SHIFT_LANCZOS3 = 8
GFC_ACCUMULATE = 16
GFC_NOALLOC_MAX_GALAXIES = 262144

STATUS = {
    0: "GFC_OK", -1: "GFC_EINVAL", -2: "GFC_EUNSUPPORTED", -3: "GFC_ENOMEM",
    -4: "GFC_EDEVICE", -5: "GFC_EBUSY", -6: "GFC_EREJECTED", -7: "GFC_ETIMEOUT",
}


class GfcError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where} -> {STATUS.get(status, status)}: {message}")


class gfc_galaxies(ctypes.Structure):
    _fields_ = [
        ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("flux", ctypes.c_void_p),
        ("r_e", ctypes.c_void_p), ("e1", ctypes.c_void_p), ("e2", ctypes.c_void_p),
        ("mix_id", ctypes.c_void_p), ("cd", ctypes.POINTER(ctypes.c_float)),
        ("psf_x", ctypes.c_void_p), ("psf_y", ctypes.c_void_p), ("mix_amp", ctypes.c_void_p),
    ]


class gfc_request(ctypes.Structure):
    _fields_ = [
        ("psf", ctypes.c_void_p), ("mix", ctypes.c_void_p), ("W", ctypes.c_int),
        ("n", ctypes.c_int), ("flags", ctypes.c_uint),
        ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("flux", ctypes.c_void_p),
        ("r_e", ctypes.c_void_p), ("e1", ctypes.c_void_p), ("e2", ctypes.c_void_p),
        ("mix_id", ctypes.c_void_p),
    ]


P = ctypes.c_void_p
PP = ctypes.POINTER(ctypes.c_void_p)
I32, U32, I64, U64 = ctypes.c_int, ctypes.c_uint, ctypes.c_int64, ctypes.c_uint64
D = ctypes.c_double

# name -> (restype, argtypes); every entry point of include/gfc.h
PROTOTYPES = {
    "gfc_status_str": (ctypes.c_char_p, [I32]),
    "gfc_last_error": (ctypes.c_char_p, []),
    "gfc_stamp_size_supported": (I32, [I32]),
    "gfc_ctx_create": (I32, [I32, PP]),
    "gfc_ctx_destroy": (I32, [P]),
    "gfc_ctx_invalid_count": (I32, [P, ctypes.POINTER(U64)]),
    "gfc_psf_create": (I32, [P, ctypes.POINTER(ctypes.c_float), I32, I32, ctypes.POINTER(D), PP]),
    "gfc_psf_create_f64": (I32, [P, ctypes.POINTER(D), I32, I32, ctypes.POINTER(D), PP]),
    "gfc_psf_create_eigen": (I32, [P, ctypes.POINTER(ctypes.c_float), I32, I32, I32, I32, ctypes.POINTER(D),
                                   ctypes.POINTER(D), PP]),
    "gfc_psf_gauss": (I32, [P, ctypes.POINTER(D)]),
    "gfc_psf_prepare": (I32, [P, I32, P]),
    "gfc_psf_spectrum": (I32, [P, I32, P, P]),
    "gfc_psf_destroy": (I32, [P]),
    "gfc_mix_create": (I32, [P, I32, ctypes.POINTER(I32), ctypes.POINTER(ctypes.c_float),
                             ctypes.POINTER(ctypes.c_float), PP]),
    "gfc_mix_device_tables": (I32, [P, PP, PP]),
    "gfc_mix_set_amp": (I32, [P, P, P]),
    "gfc_mix_destroy": (I32, [P]),
    "gfc_render_stamps": (I32, [P, P, P, ctypes.POINTER(gfc_galaxies), I64, I32, U32, P, P]),
    "gfc_sersic_create": (I32, [P, I32, ctypes.POINTER(ctypes.c_float), I32, ctypes.POINTER(ctypes.c_float),
                                ctypes.POINTER(ctypes.c_float), PP]),
    "gfc_sersic_destroy": (I32, [P]),
    "gfc_render_stamps_sersic": (I32, [P, P, P, ctypes.POINTER(gfc_galaxies), P, I64, I32, U32, P, P]),
    "gfc_render_stamps_composite": (I32, [P, P, P, I32, I32, ctypes.POINTER(gfc_galaxies), P, P, I64, I32, U32,
                                          P, P]),
    "gfc_backward_workspace_bytes": (ctypes.c_size_t, [I64]),
    "gfc_render_stamps_backward": (I32, [P, P, P, ctypes.POINTER(gfc_galaxies), I64, I32, U32,
                                         P, P, P, P, P]),
    "gfc_render_stamps_backward_noalloc": (I32, [P, P, P, ctypes.POINTER(gfc_galaxies), I64, I32, U32,
                                                 P, P, P, P]),
    "gfc_server_create": (I32, [P, ctypes.c_size_t, I32, I64, PP]),
    "gfc_server_submit": (I32, [P, ctypes.POINTER(gfc_request), ctypes.POINTER(U64)]),
    "gfc_server_poll": (I32, [P, U64, ctypes.POINTER(I32), PP, ctypes.POINTER(I32)]),
    "gfc_server_wait": (I32, [P, U64, I32, PP]),
    "gfc_server_copy": (I32, [P, U64, P, P]),
    "gfc_server_release": (I32, [P, U64]),
    "gfc_server_stats": (I32, [P, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D),
                               ctypes.POINTER(D), ctypes.POINTER(U64), ctypes.POINTER(U64)]),
    "gfc_server_replay": (I32, [P, ctypes.POINTER(gfc_request), ctypes.POINTER(D), I64, ctypes.POINTER(P),
                                ctypes.POINTER(D), ctypes.POINTER(D)]),
    "gfc_server_destroy": (I32, [P]),
    "gfc_sched_create": (I32, [ctypes.c_void_p, ctypes.c_size_t, I32, I64, PP]),
    "gfc_sched_submit": (I32, [P, U64, I64, ctypes.c_size_t, ctypes.POINTER(U64)]),
    "gfc_sched_step": (I32, [P]),
    "gfc_sched_query": (I32, [P, U64, ctypes.POINTER(I32), ctypes.POINTER(U64)]),
    "gfc_sched_release": (I32, [P, U64]),
    "gfc_sched_usage": (I32, [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(U64)]),
    "gfc_sched_stats": (I32, [P, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D),
                              ctypes.POINTER(D), ctypes.POINTER(U64), ctypes.POINTER(U64)]),
    "gfc_sched_destroy": (I32, [P]),
}

# gfc_sched_executor callbacks
SCHED_NOW = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.c_void_p)
SCHED_LAUNCH = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                ctypes.POINTER(ctypes.c_uint64), ctypes.c_int64)
SCHED_POLL = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64)
SCHED_RELEASE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_uint64)


class gfc_sched_executor(ctypes.Structure):
    _fields_ = [("user", ctypes.c_void_p), ("now", SCHED_NOW), ("launch", SCHED_LAUNCH),
                ("poll", SCHED_POLL), ("release", SCHED_RELEASE)]

_lib = None


def lib():
    """Loads libgfc.so once.  Raises loudly when it has not been built: there
    is no fallback implementation."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2012_15797_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(status: int, where: str) -> None:
    if status != 0:
        msg = lib().gfc_last_error().decode(errors="replace")
        raise GfcError(status, where, msg)


def call(name: str, *args):
    """Calls a status-returning entry point and raises GfcError on failure."""
    st = getattr(lib(), name)(*args)
    check(st, name)
    return st

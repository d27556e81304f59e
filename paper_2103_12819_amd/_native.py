"""ctypes mirror of include/mm.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmm.so")

MM_OK, MM_EINVAL, MM_ENOMEM, MM_EDEVICE, MM_ENOCONV, MM_ENONFINITE, MM_ESTATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "MM_OK", -1: "MM_EINVAL", -2: "MM_ENOMEM", -3: "MM_EDEVICE",
                -4: "MM_ENOCONV", -5: "MM_ENONFINITE", -6: "MM_ESTATE"}
MM_BC_PEC, MM_BC_PERIODIC = 0, 1
MM_FP64, MM_FP32 = 0, 1

EXPORTED = ["mm_init", "mm_step", "mm_step_noalloc", "mm_add_probe", "mm_add_hard_source", "mm_add_surface_current",
            "mm_probe", "mm_get_field", "mm_set_field", "mm_get_field_device", "mm_set_field_device",
            "mm_stats", "mm_sync", "mm_info", "mm_layout", "mm_adjoint_enable", "mm_adjoint", "mm_profile",
            "mm_profile_read", "mm_last_error", "mm_destroy"]

_dptr = C.POINTER(C.c_double)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class mm_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("bc", C.c_int32 * 3), ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double)]


class mm_materials(C.Structure):
    _fields_ = [("eps_r", _dptr), ("sigma", _dptr), ("mu_r", _dptr), ("Ms", _dptr),
                ("alpha", _dptr), ("gamma", _dptr), ("m0_dir", _dptr)]


class mm_bias(C.Structure):
    _fields_ = [("H0", C.c_double * 3)]


class mm_source(C.Structure):
    _fields_ = [("comp", C.c_int32), ("profile", _dptr), ("f0", C.c_double),
                ("Tp", C.c_double), ("t0", C.c_double)]


class mm_hard_source(C.Structure):
    _fields_ = [("field", C.c_int32), ("profile", _dptr), ("f0", C.c_double),
                ("Tp", C.c_double), ("t0", C.c_double)]


class mm_surface_current(C.Structure):
    _fields_ = [("axis", C.c_int32), ("side", C.c_int32), ("comp", C.c_int32), ("profile", _dptr),
                ("f0", C.c_double), ("Tp", C.c_double), ("t0", C.c_double)]


MM_MAX_HARD = 8


class mm_pml(C.Structure):
    _fields_ = [("cells", C.c_int32 * 6), ("R0", C.c_double), ("order", C.c_double)]


class mm_options(C.Structure):
    _fields_ = [("prec", C.c_int32), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("fixed_iter", C.c_int32), ("hip_stream", C.c_void_p),
                ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN), ("alloc_ctx", C.c_void_p),
                ("scheme", C.c_int32), ("pml", C.POINTER(mm_pml)), ("fused", C.c_int32)]


class mm_probe_desc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("field", C.c_int32), ("i", C.c_int32),
                ("j", C.c_int32), ("k", C.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libmm.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP library {path} is missing; run `python -m paper_2103_12819_amd.build`")
    # torch ships its own HIP runtime; load it first so that libmm.so binds to
    # that one (its libamdhip64.so.7 dependency is then already loaded) and
    # the process holds a single HIP runtime, whatever the caller imported
    # first.  Loading libmm.so first would pull in a second runtime.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.mm_init.argtypes = [C.POINTER(P), C.POINTER(mm_grid), C.c_double, C.POINTER(mm_materials),
                            C.POINTER(mm_bias), C.POINTER(mm_source), C.POINTER(mm_options)]
    lib.mm_init.restype = C.c_int
    lib.mm_step.argtypes = [P, C.c_int64]
    lib.mm_step.restype = C.c_int
    lib.mm_step_noalloc.argtypes = [P, C.c_int64]
    lib.mm_step_noalloc.restype = C.c_int
    lib.mm_add_probe.argtypes = [P, C.POINTER(mm_probe_desc), C.POINTER(C.c_int32)]
    lib.mm_add_probe.restype = C.c_int
    lib.mm_add_hard_source.argtypes = [P, C.POINTER(mm_hard_source)]
    lib.mm_add_hard_source.restype = C.c_int
    lib.mm_add_surface_current.argtypes = [P, C.POINTER(mm_surface_current)]
    lib.mm_add_surface_current.restype = C.c_int
    lib.mm_probe.argtypes = [P, C.c_int32, _dptr, C.c_size_t, C.POINTER(C.c_size_t), _dptr]
    lib.mm_probe.restype = C.c_int
    lib.mm_get_field.argtypes = [P, C.c_int32, _dptr]
    lib.mm_get_field.restype = C.c_int
    lib.mm_set_field.argtypes = [P, C.c_int32, _dptr]
    lib.mm_get_field_device.argtypes = [P, C.c_int32, C.c_void_p]
    lib.mm_get_field_device.restype = C.c_int
    lib.mm_set_field_device.argtypes = [P, C.c_int32, C.c_void_p]
    lib.mm_set_field_device.restype = C.c_int
    lib.mm_set_field.restype = C.c_int
    lib.mm_stats.argtypes = [P, C.POINTER(C.c_int32), C.c_size_t, C.POINTER(C.c_size_t)]
    lib.mm_stats.restype = C.c_int
    lib.mm_sync.argtypes = [P]
    lib.mm_sync.restype = C.c_int
    lib.mm_info.argtypes = [P, C.POINTER(C.c_int64)]
    lib.mm_info.restype = C.c_int
    lib.mm_layout.argtypes = [P, C.POINTER(C.c_int64)]
    lib.mm_layout.restype = C.c_int
    lib.mm_adjoint_enable.argtypes = [P, C.c_int32, C.c_int32]
    lib.mm_adjoint_enable.restype = C.c_int
    lib.mm_adjoint.argtypes = [P, C.c_int32, _dptr, _dptr]
    lib.mm_adjoint.restype = C.c_int
    lib.mm_profile.argtypes = [P, C.c_int32]
    lib.mm_profile.restype = C.c_int
    lib.mm_profile_read.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.mm_profile_read.restype = C.c_int
    lib.mm_last_error.argtypes = [P]
    lib.mm_last_error.restype = C.c_char_p
    lib.mm_destroy.argtypes = [P]
    lib.mm_destroy.restype = None
    _lib = lib
    return lib

"""ctypes binding of libskei_ct.so (include/skei_ct.h): argument marshalling only.

The binding never computes anything itself; every operator runs in the HIP
kernels of the library.  Loading fails loudly when the library has not been
built -- there is no CPU fallback.

torch is imported before the library is opened so that the process uses the
HIP runtime torch ships (one runtime per process; torch's streams are valid
handles for the library's calls).
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must precede loading the HIP library)

from . import build as _build

LIB_PATH = _build.LIB

_lib = None

c_int, c_float, c_size_t, c_void_p, c_double = ctypes.c_int, ctypes.c_float, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_double
c_char_p = ctypes.c_char_p


class EiProblem(ctypes.Structure):
    """skei_ei_problem (include/skei_ct.h); pointers are device addresses."""
    _fields_ = [
        ("geom", c_void_p), ("batch", c_int), ("x", c_void_p), ("y", c_void_p),
        ("mc_idx", c_void_p), ("m_mc", c_int), ("angle_idx", c_void_p), ("m", c_int),
        ("copies", c_int), ("cos_sin", c_void_p), ("lam", c_float), ("loss", c_void_p), ("grad", c_void_p),
        ("step", c_float), ("work", c_void_p), ("work_bytes", c_size_t),
    ]


_PROB = ctypes.POINTER(EiProblem)

# name -> (restype, argtypes); every pointer is passed as void*.
_SIGS = {
    "skei_version": (c_char_p, []),
    "skei_strerror": (c_char_p, [c_int]),
    "skei_geom_create": (c_int, [c_int, c_int, c_int, ctypes.POINTER(c_void_p)]),
    "skei_geom_destroy": (c_int, [c_void_p]),
    "skei_geom_set_tuning": (c_int, [c_void_p, c_int, c_int, c_int, c_int]),
    "skei_geom_info": (c_int, [c_void_p, ctypes.POINTER(c_int), ctypes.POINTER(c_int), ctypes.POINTER(c_int)]),
    "skei_radon_fwd": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_int, c_void_p, c_void_p]),
    "skei_radon_adj": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_int, c_void_p, c_void_p]),
    "skei_radon_resid": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_int, c_void_p, c_void_p]),
    "skei_sketch_rows": (c_int, [c_void_p, c_int, c_int, c_void_p, c_int, c_int, c_void_p, c_void_p]),
    "skei_sketch_rows_T": (c_int, [c_void_p, c_int, c_int, c_void_p, c_int, c_int, c_void_p, c_void_p]),
    # multicoil MRI (include/skei_mri.h)
    "skei_mri_fwd": (c_int, [c_void_p, c_int, c_int, c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "skei_mri_adj": (c_int, [c_void_p, c_int, c_int, c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                             c_void_p]),
    "skei_mri_work_bytes": (c_size_t, [c_int, c_int, c_int]),
    "skei_coil_weights": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p]),
    "skei_coil_mix": (c_int, [c_void_p, c_int, c_int, c_void_p, c_int, ctypes.c_longlong, c_void_p, c_void_p]),
    "skei_coil_covariance": (c_int, [c_void_p, c_int, ctypes.c_longlong, c_void_p, c_void_p]),
    "skei_coil_pca": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p]),
    "skei_ramp": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_void_p]),
    "skei_backproject": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_int, c_void_p, c_void_p]),
    "skei_backproject_T": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_int, c_void_p, c_void_p]),
    "skei_fbp_workspace_bytes": (c_size_t, [c_void_p, c_int, c_int]),
    "skei_fbp": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_int, c_void_p, c_void_p, c_size_t, c_void_p]),
    "skei_fbp_adj": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_int, c_void_p, c_void_p, c_size_t, c_void_p]),
    "skei_rotate": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p]),
    "skei_rotate_adj": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p]),
    "skei_sumsq_workspace_bytes": (c_size_t, [c_size_t]),
    "skei_sumsq_diff": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_void_p, c_size_t, c_void_p]),
    "skei_ei_workspace_bytes": (c_size_t, [c_void_p, c_int, c_int, c_int, c_int]),
    "skei_probe_set": (c_int, [c_int, c_void_p, c_void_p]),
    "skei_ei_loss_grad": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_int, c_void_p, c_int,
                                  c_int, c_void_p, c_float, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "skei_lds_read_bounds": (c_int, [c_int, c_int, ctypes.POINTER(ctypes.c_longlong)]),
    "skei_ei_noalloc_scratch_bytes": (c_size_t, []),
    "skei_ei_loss_grad_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_int, c_void_p, c_int,
                                          c_int, c_void_p, c_float, c_void_p, c_void_p, c_void_p]),
    "skei_ei_plan_workspace_bytes": (c_size_t, [_PROB, c_int]),
    "skei_ei_problem_workspace_bytes": (c_size_t, [_PROB]),
    "skei_ei_plan_create": (c_int, [_PROB, c_int, c_void_p, c_size_t, ctypes.POINTER(c_void_p)]),
    "skei_ei_plan_destroy": (c_int, [c_void_p]),
    "skei_ei_plan_run": (c_int, [c_void_p, c_void_p]),
    "skei_ei_plan_configure": (c_int, [c_void_p, c_int, c_int, c_int]),
    "skei_ei_plan_get_config": (c_int, [c_void_p, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]),
    "skei_ei_plan_autotune": (c_int, [c_void_p, c_void_p, c_int, c_char_p]),
}


class SkeiError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn} failed: {strerror(code)} (code {code})")
        self.code = code


# Stages of one EI step in launch order (SKEI_STAGE_*).
STAGES = ["rotate", "fwd", "ramp", "bp_resid", "reduce", "bp_T", "ramp_T", "adj", "rotate_adj"]
DISPATCH_PERSISTENT, DISPATCH_STATIC = 0, 1


def exported_symbols() -> list[str]:
    return sorted(_SIGS)


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built ({LIB_PATH}); run __graft_entry__.build() first")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def strerror(code: int) -> str:
    return lib().skei_strerror(int(code)).decode()


def version() -> str:
    return lib().skei_version().decode()


def call(name: str, *args) -> int:
    """Call an int-returning entry point and raise SkeiError on failure."""
    rc = getattr(lib(), name)(*args)
    if rc != 0:
        raise SkeiError(name, rc)
    return rc


def query(name: str, *args):
    return getattr(lib(), name)(*args)

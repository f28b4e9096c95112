"""ctypes binding of libpm.so (the C ABI declared in include/pm.h).

Argument marshalling only: every step of the PM path runs in the HIP
kernels of the library.  Importing this module without a built library
raises ImportError; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpm.so")

PM_OK, PM_EINVAL, PM_ENOMEM, PM_EHIP, PM_ESTATE, PM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "PM_OK", -1: "PM_EINVAL", -2: "PM_ENOMEM", -3: "PM_EHIP", -4: "PM_ESTATE",
                -5: "PM_EUNSUPPORTED"}
KERNEL_CLASSES = ["fill", "deposit", "fft_rows", "fft_cols", "gather_kick", "adj_kick", "dipole",
                  "adj_drift", "misc", "bin"]
PM_FORCE_PM, PM_FORCE_NUFFT = 0, 1
PM_SPEC_POWERLAW, PM_SPEC_BBKS = 0, 1


class pm_config(C.Structure):
    _fields_ = [
        ("n_p", C.c_int32), ("n_g", C.c_int32),
        ("box", C.c_double),
        ("omega_m", C.c_double), ("h", C.c_double), ("n_s", C.c_double), ("sigma8", C.c_double),
        ("spectrum", C.c_int32),
        ("pl_rms_cells", C.c_double),
        ("a_start", C.c_double), ("a_end", C.c_double),
        ("n_steps", C.c_int32),
        ("force", C.c_int32), ("mak", C.c_int32), ("deconvolve", C.c_int32),
        ("grad_order", C.c_int32), ("lap_order", C.c_int32),
        ("es_width", C.c_int32),
        ("es_beta", C.c_double),
        ("batch", C.c_int32),
        ("lpt_order", C.c_int32), ("stepper", C.c_int32), ("time_var", C.c_int32), ("antialias", C.c_int32),
    ]


EXPORTS = {
    "pm_create": (C.c_int, [C.POINTER(pm_config), C.POINTER(C.c_void_p)]),
    "pm_workspace_bytes": (C.c_size_t, [C.c_void_p, C.c_int32]),
    "pm_bind": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32, C.c_void_p]),
    "pm_destroy": (C.c_int, [C.c_void_p]),
    "pm_schedule": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "pm_describe": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pm_last_error": (C.c_char_p, [C.c_void_p]),
    "pm_profile": (C.c_int, [C.c_void_p, C.c_int32]),
    "pm_use_graphs": (C.c_int, [C.c_void_p, C.c_int32]),
    "pm_set_active": (C.c_int, [C.c_void_p, C.c_uint64]),
    "pm_kernel_times": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pm_set_slot_params": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pm_init_ics": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pm_power_spectrum_mesh_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_int32,
                                                 C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pm_step": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pm_set_step_index": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pm_step_device": (C.c_int, [C.c_void_p]),
    "pm_get_step_index": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pm_run": (C.c_int, [C.c_void_p]),
    "pm_adjoint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pm_adjoint_full": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pm_power_spectrum": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pm_jvp": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pm_get_tangent": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pm_power_spectrum_jvp": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p]),
    "pm_density": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pm_get_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pm_set_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pm_deposit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "pm_force": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]),
    "pm_force_vjp": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_int32, C.c_void_p]),
    "pm_fft": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
}

_lib = None


def load():
    """Load libpm.so once; raise ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2510_05206_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PMError(RuntimeError):
    pass


def check(status, ctx=None, what=""):
    if status != PM_OK:
        msg = ""
        if ctx:
            raw = load().pm_last_error(ctx)
            msg = raw.decode() if raw else ""
        raise PMError(f"{what}: {STATUS_NAMES.get(status, status)} {msg}".strip())

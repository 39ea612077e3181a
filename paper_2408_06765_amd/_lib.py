"""ctypes declarations of the librsi C ABI (include/rsi.h).

Loading fails loudly: there is no fallback path.  Build the library first with
``python -m paper_2408_06765_amd.build`` (``__graft_entry__.build()`` does it).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "librsi.so")

_dp = C.POINTER(C.c_double)


class rsi_points(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("n", C.c_int64)]


class rsi_medium(C.Structure):
    _fields_ = [("c", C.c_double), ("rho", C.c_double)]


class rsi_transducer(C.Structure):
    _fields_ = [("pts", rsi_points), ("w", C.c_void_p), ("v0", C.c_double),
                ("centre", C.c_double * 3), ("axis", C.c_double * 3)]


class rsi_interface(C.Structure):
    _fields_ = [("pts", rsi_points), ("w", C.c_void_p), ("z", C.c_double)]


class rsi_instance(C.Structure):
    _fields_ = [("src", rsi_points), ("w", C.c_void_p), ("vel", C.c_void_p), ("v0", C.c_double),
                ("normal", C.c_double * 3), ("tgt", rsi_points), ("medium", rsi_medium),
                ("freq", C.c_double), ("kind", C.c_int), ("out", C.c_void_p)]


# every function the header declares, with its ctypes signature
SIGNATURES = {
    "rsi_status_string": ([C.c_int], C.c_char_p),
    "rsi_last_error": ([], C.c_char_p),
    "rsi_version": ([], C.c_int),
    "rsi_set_check_finite": ([C.c_int], C.c_int),
    "rsi_sobol2d": ([C.c_uint32, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p], C.c_int),
    "rsi_sample_disc": ([C.c_uint32, C.c_int64, C.c_double, _dp, C.c_double, C.c_void_p,
                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "rsi_sample_square": ([C.c_uint32, C.c_int64, C.c_double, C.c_double, C.c_double, C.c_double,
                           C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "rsi_halton2d": ([C.c_int64, C.c_int64, C.c_void_p, C.c_void_p], C.c_int),
    "rsi_sample_disc_ex": ([C.c_int, C.c_uint32, C.c_int64, C.c_double, _dp, C.c_double, C.c_void_p,
                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "rsi_sample_square_ex": ([C.c_int, C.c_uint32, C.c_int64, C.c_double, C.c_double, C.c_double,
                              C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
                             C.c_int),
    "rsi_sample_cap": ([C.c_int, C.c_uint32, C.c_int64, C.c_double, C.c_double, _dp, C.c_double,
                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "rsi_apodise": ([C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, _dp, _dp, C.c_double, C.c_void_p,
                     C.c_void_p], C.c_int),
    "rsi_transmission": ([C.c_int, C.c_int, _dp, C.POINTER(rsi_medium), _dp, _dp, C.c_int64,
                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "rsi_propagate": ([C.POINTER(rsi_points), C.c_void_p, C.c_void_p, _dp, C.POINTER(rsi_points),
                       rsi_medium, C.c_double, C.c_int, C.c_int, C.c_void_p, C.c_void_p], C.c_int),
    "rsi_propagate_ex": ([C.POINTER(rsi_points), C.c_void_p, C.c_void_p, _dp, C.POINTER(rsi_points),
                          rsi_medium, C.c_double, C.c_int, C.c_int, C.c_uint32, C.c_void_p,
                          C.c_void_p], C.c_int),
    "rsi_propagate_multifreq": ([C.POINTER(rsi_points), C.c_void_p, C.c_void_p, _dp,
                                 C.POINTER(rsi_points), rsi_medium, _dp, C.c_int, C.c_int, C.c_int,
                                 C.c_uint32, C.c_void_p, C.c_void_p], C.c_int),
    "rsi_propagate_noalloc": ([C.POINTER(rsi_points), C.c_void_p, C.c_void_p, _dp,
                               C.POINTER(rsi_points), rsi_medium, C.c_double, C.c_int, C.c_int,
                               C.c_uint32, C.c_void_p, C.c_void_p], C.c_int),
    "rsi_chain": ([C.POINTER(rsi_transducer), C.POINTER(rsi_interface), C.c_int,
                   C.POINTER(rsi_medium), C.POINTER(rsi_points), _dp, C.c_int, C.c_int, C.c_int,
                   C.c_void_p, C.c_void_p], C.c_int),
    "rsi_chain_ex": ([C.POINTER(rsi_transducer), C.POINTER(rsi_interface), C.c_int,
                      C.POINTER(rsi_medium), C.POINTER(rsi_points), _dp, C.c_int, C.c_int, C.c_int,
                      C.c_uint32, C.c_void_p, C.c_void_p], C.c_int),
    "rsi_reflection": ([C.c_int, C.c_int, _dp, C.POINTER(rsi_medium), _dp, _dp, C.c_int64,
                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "rsi_ray_field": ([C.POINTER(rsi_transducer), _dp, C.c_int, C.POINTER(rsi_medium),
                       C.POINTER(rsi_points), _dp, C.c_int, C.c_int, C.c_void_p, C.c_void_p], C.c_int),
    "rsi_propagate_batched": ([C.POINTER(rsi_instance), C.c_int, C.c_int, C.c_void_p], C.c_int),
    "rsi_plan_create_chain": ([C.POINTER(C.c_void_p), C.POINTER(rsi_transducer),
                               C.POINTER(rsi_interface), C.c_int, C.POINTER(rsi_medium),
                               C.POINTER(rsi_points), _dp, C.c_int, C.c_int, C.c_int,
                               C.c_void_p], C.c_int),
    "rsi_plan_create_chain_ex": ([C.POINTER(C.c_void_p), C.POINTER(rsi_transducer),
                                  C.POINTER(rsi_interface), C.c_int, C.POINTER(rsi_medium),
                                  C.POINTER(rsi_points), _dp, C.c_int, C.c_int, C.c_int,
                                  C.c_uint32, C.c_void_p], C.c_int),
    "rsi_plan_create_batched": ([C.POINTER(C.c_void_p), C.POINTER(rsi_instance), C.c_int,
                                 C.c_int], C.c_int),
    "rsi_plan_execute": ([C.c_void_p, C.c_void_p], C.c_int),
    "rsi_plan_destroy": ([C.c_void_p], C.c_int),
    "rsi_autotune_batched": ([C.POINTER(rsi_instance), C.c_int, C.c_int], C.c_int),
    "rsi_to_pressure": ([C.c_int64, C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_void_p,
                         C.c_void_p], C.c_int),
}

_lib = None


def load():
    """Load librsi.so (once) and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError(
            f"{LIBPATH} is missing: build it with `python -m paper_2408_06765_amd.build`")
    lib = C.CDLL(LIBPATH)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


class RSIError(RuntimeError):
    pass


def check(status: int, what: str) -> None:
    if status != 0:
        lib = load()
        name = lib.rsi_status_string(status).decode()
        detail = lib.rsi_last_error().decode()
        raise RSIError(f"{what} failed: {name}" + (f" ({detail})" if detail else ""))

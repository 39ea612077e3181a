"""The C ABI library loads, exports every function include/rsi.h declares, and rejects
bad arguments before touching a device (no compute call runs here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rsi_[a-z0-9_]+|mlp_[a-z0-9_]+)\s*\(", text)))


def test_header_functions_exported_and_bound():
    from paper_2408_06765_amd import _lib
    lib = _lib.load()
    names = declared_functions("rsi.h")
    assert "rsi_propagate" in names and "rsi_chain" in names
    for n in names:
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, f"{n} has no Python binding"


def test_surrogate_header_functions_exported_and_bound():
    from paper_2408_06765_amd import _lib, surrogate
    lib = surrogate._load()
    names = declared_functions("rsi_mlp.h")
    assert "rsi_mlp_train_step" in names and "rsi_surrogate_carrier" in names
    for n in names:
        assert hasattr(lib, n), n
        assert n in surrogate.SIGNATURES, f"{n} has no Python binding"


def test_surrogate_argument_errors():
    import ctypes as C
    from paper_2408_06765_amd import surrogate
    lib = surrogate._load()
    h = C.c_void_p()
    B = (C.c_float * 10)()
    lo = (C.c_float * 5)(0, 0, 0, 0, 0)
    hi = (C.c_float * 5)(1, 1, 1, 1, 1)
    # width not a multiple of 64, depth out of range, empty box
    assert lib.rsi_mlp_create(C.byref(h), 32, 100, 3, B, lo, hi, 64) == 2
    assert lib.rsi_mlp_create(C.byref(h), 32, 64, 0, B, lo, hi, 64) == 2
    assert lib.rsi_mlp_create(C.byref(h), 32, 64, 3, B, lo, lo, 64) == 2
    assert lib.rsi_mlp_create(C.byref(h), 32, 64, 3, B, lo, hi, 0) == 3
    assert lib.rsi_mlp_destroy(None) == 0
    assert lib.rsi_mlp_forward(None, 1, None, None, None) == 1
    assert lib.rsi_surrogate_carrier(4, None, _lib_medium(1480, 1000), _lib_medium(5900, 7800), 3, None, None,
                                     None) == 2
    # ray frame: sigma <= 0, unknown mode, no reference values, missing arrays
    assert lib.rsi_surrogate_ray_frame(4, None, 4, None, 0.0, 0.0, 0, None, None, None) == 2
    assert lib.rsi_surrogate_ray_frame(4, None, 4, None, 0.02, 0.0, 2, None, None, None) == 2
    assert lib.rsi_surrogate_ray_frame(4, None, 0, None, 0.02, 0.0, 0, None, None, None) == 3
    assert lib.rsi_surrogate_ray_frame(4, None, 4, None, 0.02, 5.0, 1, None, None, None) == 1
    assert lib.rsi_surrogate_ray_frame(0, None, 0, None, 0.02, 5.0, 1, None, None, None) == 0


def _lib_medium(c, rho):
    from paper_2408_06765_amd import _lib
    return _lib.rsi_medium(c, rho)


def test_status_strings_and_version():
    from paper_2408_06765_amd import _lib
    lib = _lib.load()
    assert lib.rsi_status_string(0) == b"RSI_OK"
    assert lib.rsi_status_string(2) == b"RSI_ERR_ARG"
    assert lib.rsi_status_string(99) == b"RSI_UNKNOWN_STATUS"
    assert lib.rsi_version() >> 16 == 1


def test_finite_check_toggle():
    """rsi_set_check_finite returns the previous setting (host state only)."""
    from paper_2408_06765_amd import _lib
    lib = _lib.load()
    prev = lib.rsi_set_check_finite(1)
    try:
        assert lib.rsi_set_check_finite(1) == 1
        assert lib.rsi_set_check_finite(0) == 1
        assert lib.rsi_set_check_finite(0) == 0
    finally:
        lib.rsi_set_check_finite(prev)


def test_argument_errors_before_any_device_work():
    from paper_2408_06765_amd import _lib
    lib = _lib.load()
    L = _lib
    pts = L.rsi_points(None, None, None, 4)
    empty = L.rsi_points(None, None, None, 0)
    med = L.rsi_medium(1480.0, 1000.0)
    # NULL descriptors
    assert lib.rsi_propagate(None, None, None, None, None, med, 1e6, 0, 0, None, None) == 1
    # frequency and speed must be positive
    assert lib.rsi_propagate(C.byref(pts), None, None, None, C.byref(pts), med, -1.0, 0, 0, None, None) == 2
    assert lib.rsi_propagate(C.byref(pts), None, None, None, C.byref(pts), L.rsi_medium(0.0, 1.0), 1e6, 0, 0,
                             None, None) == 2
    # unknown kind / precision (0 monopole, 1 dipole, 2 omnidirectional)
    assert lib.rsi_propagate(C.byref(pts), None, None, None, C.byref(pts), med, 1e6, 7, 0, None, None) == 2
    assert lib.rsi_propagate(C.byref(pts), None, None, None, C.byref(empty), med, 1e6, 2, 0, None, None) == 0
    assert lib.rsi_propagate(C.byref(pts), None, None, None, C.byref(pts), med, 1e6, 0, 9, None, None) == 2
    # negative sizes
    neg = L.rsi_points(None, None, None, -1)
    assert lib.rsi_propagate(C.byref(neg), None, None, None, C.byref(pts), med, 1e6, 0, 0, None, None) == 3
    # zero targets: nothing to do
    assert lib.rsi_propagate(C.byref(pts), None, None, None, C.byref(empty), med, 1e6, 0, 0, None, None) == 0
    # sampling arguments
    assert lib.rsi_sample_disc(0, 10, -1.0, None, 0.0, None, None, None, None, None) == 2
    assert lib.rsi_sample_square(0, -1, 0, 0, 0, 0.01, None, None, None, None, None) == 3
    assert lib.rsi_sobol2d(0, (1 << 32) - 5, 10, None, None) == 3
    assert lib.rsi_sobol2d(0, 0, 0, None, None) == 0
    # pressure
    assert lib.rsi_to_pressure(4, None, 0, -1.0, 1e6, None, None) == 2
    # sequences, cap, apodisation, Halton range
    cen = (C.c_double * 3)(0, 0, 0)
    ax = (C.c_double * 3)(0, 0, 1)
    assert lib.rsi_sample_disc_ex(5, 0, 10, 0.01, cen, 0.0, None, None, None, None, None) == 2
    assert lib.rsi_sample_cap(0, 0, 10, 0.01, 0.005, cen, 0.0, None, None, None, None, None) == 2
    assert lib.rsi_sample_cap(1, 0, -1, 0.01, 0.05, cen, 0.0, None, None, None, None, None) == 3
    assert lib.rsi_sample_cap(1, 0, 0, 0.01, 0.05, cen, 0.0, None, None, None, None, None) == 0
    assert lib.rsi_halton2d((1 << 40) - 5, 10, None, None) == 3
    assert lib.rsi_apodise(10, None, None, None, cen, ax, 0.0, None, None) == 2
    assert lib.rsi_apodise(10, None, None, None, cen, (C.c_double * 3)(0, 0, 0), 1.0, None, None) == 2
    assert lib.rsi_apodise(0, None, None, None, cen, ax, 1.0, None, None) == 0


def test_chain_validation():
    from paper_2408_06765_amd import _lib as L
    lib = L.load()
    xd = L.rsi_transducer(L.rsi_points(None, None, None, 0), None, 1.0, (C.c_double * 3)(0, 0, 0),
                          (C.c_double * 3)(0, 0, 1))
    ifs = (L.rsi_interface * 2)(L.rsi_interface(L.rsi_points(None, None, None, 0), None, 0.05),
                                L.rsi_interface(L.rsi_points(None, None, None, 0), None, 0.04))
    media = (L.rsi_medium * 3)(L.rsi_medium(1480, 1000), L.rsi_medium(5900, 7800), L.rsi_medium(2700, 2700))
    tgt = L.rsi_points(None, None, None, 0)
    fr = (C.c_double * 1)(1e6)
    # planes must be strictly increasing in z
    assert lib.rsi_chain(C.byref(xd), ifs, 2, media, C.byref(tgt), fr, 1, 1, 0, None, None) == 2
    # non-positive density
    bad = (L.rsi_medium * 2)(L.rsi_medium(1480, 1000), L.rsi_medium(5900, 0.0))
    assert lib.rsi_chain(C.byref(xd), ifs, 1, bad, C.byref(tgt), fr, 1, 1, 0, None, None) == 2
    # unknown transmission mode
    assert lib.rsi_chain(C.byref(xd), ifs, 1, media, C.byref(tgt), fr, 1, 5, 0, None, None) == 2
    # too many interfaces
    assert lib.rsi_chain(C.byref(xd), ifs, 1000, media, C.byref(tgt), fr, 1, 1, 0, None, None) == 3
    # chain flags: unknown bits, and the above mode without an interface
    assert lib.rsi_chain_ex(C.byref(xd), ifs, 1, media, C.byref(tgt), fr, 1, 1, 0, 4, None, None) == 2
    assert lib.rsi_chain_ex(C.byref(xd), ifs, 0, media, C.byref(tgt), fr, 1, 1, 0, 2, None, None) == 2
    plan0 = C.c_void_p()
    assert lib.rsi_plan_create_chain_ex(C.byref(plan0), C.byref(xd), ifs, 1, media, C.byref(tgt), fr, 1, 1, 0,
                                        8, None) == 2
    # valid flags with no field points: nothing to do
    assert lib.rsi_chain_ex(C.byref(xd), ifs, 1, media, C.byref(tgt), fr, 1, 1, 0, 3, None, None) == 0
    # reflection coefficients: same argument checks as the transmission coefficients
    assert lib.rsi_reflection(5, 1, (C.c_double * 1)(0.05), media, None, None, 0, None, None, None, None) == 2
    assert lib.rsi_reflection(0, 0, (C.c_double * 1)(0.05), media, None, None, 0, None, None, None, None) == 3
    # batched: bad kind is rejected before any allocation
    inst = (L.rsi_instance * 1)()
    inst[0].kind = 5
    inst[0].freq = 1e6
    inst[0].medium = L.rsi_medium(1480, 1000)
    assert lib.rsi_propagate_batched(inst, 1, 0, None) == 2
    plan = C.c_void_p()
    assert lib.rsi_plan_create_batched(C.byref(plan), inst, 1, 0) == 2
    assert lib.rsi_plan_destroy(None) == 0
    assert lib.rsi_plan_execute(None, None) == 1


def test_ray_field_validation():
    from paper_2408_06765_amd import _lib as L
    lib = L.load()
    xd = L.rsi_transducer(L.rsi_points(None, None, None, 0), None, 1.0, (C.c_double * 3)(0, 0, 0),
                          (C.c_double * 3)(0, 0, 1))
    media = (L.rsi_medium * 3)(L.rsi_medium(1480, 1000), L.rsi_medium(5900, 7800), L.rsi_medium(2700, 2700))
    tgt = L.rsi_points(None, None, None, 0)
    fr = (C.c_double * 1)(1e6)
    zif = (C.c_double * 2)(0.05, 0.04)
    ok = (C.c_double * 2)(0.04, 0.05)
    # planes not strictly increasing, too many planes, negative count
    assert lib.rsi_ray_field(C.byref(xd), zif, 2, media, C.byref(tgt), fr, 1, 0, None, None) == 2
    assert lib.rsi_ray_field(C.byref(xd), ok, 9, media, C.byref(tgt), fr, 1, 0, None, None) == 3
    assert lib.rsi_ray_field(C.byref(xd), ok, -1, media, C.byref(tgt), fr, 1, 0, None, None) == 3
    # missing plane depths, bad medium, bad frequency, bad precision
    assert lib.rsi_ray_field(C.byref(xd), None, 1, media, C.byref(tgt), fr, 1, 0, None, None) == 1
    bad = (L.rsi_medium * 2)(L.rsi_medium(1480, 1000), L.rsi_medium(-5900, 7800))
    assert lib.rsi_ray_field(C.byref(xd), ok, 1, bad, C.byref(tgt), fr, 1, 0, None, None) == 2
    assert lib.rsi_ray_field(C.byref(xd), ok, 1, media, C.byref(tgt), (C.c_double * 1)(0.0), 1, 0, None,
                             None) == 2
    assert lib.rsi_ray_field(C.byref(xd), ok, 1, media, C.byref(tgt), fr, 1, 7, None, None) == 2
    # no field points: nothing to do; field points but no output buffer
    assert lib.rsi_ray_field(C.byref(xd), ok, 2, media, C.byref(tgt), fr, 1, 0, None, None) == 0
    one = (C.c_double * 1)(0.0)
    tgt1 = L.rsi_points(C.cast(one, C.c_void_p), C.cast(one, C.c_void_p), C.cast(one, C.c_void_p), 1)
    assert lib.rsi_ray_field(C.byref(xd), ok, 2, media, C.byref(tgt1), fr, 1, 0, None, None) == 1

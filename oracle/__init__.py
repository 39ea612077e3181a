"""FP64 reference implementation of the RSI quasi-Monte-Carlo beam model.

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this package.  The product library never calls it.

The arithmetic lives in ``rsi_oracle.c`` (plain C, FP64, Neumaier sums); this file
only marshals numpy arrays through ctypes.  Every function names the passage of
the paper it follows; see the header of ``rsi_oracle.c`` for the readings taken
where the paper is silent.  ``mlp_oracle`` holds the reference for the learned
surrogate.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "librsi_oracle.so")
_lib = None

_dp = C.POINTER(C.c_double)
_u32p = C.POINTER(C.c_uint32)
_i64p = C.POINTER(C.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b  # noqa: F401  (build on first use in a fresh tree)
        _b.build()
    lib = C.CDLL(_LIBPATH)
    lib.orc_sobol2d.argtypes = [C.c_uint32, C.c_int64, C.c_int64, _u32p]
    lib.orc_sample_disc.argtypes = [C.c_uint32, C.c_int64, C.c_double, _dp, C.c_double,
                                    _dp, _dp, _dp, _dp]
    lib.orc_sample_square.argtypes = [C.c_uint32, C.c_int64, C.c_double, C.c_double,
                                      C.c_double, C.c_double, _dp, _dp, _dp, _dp]
    lib.orc_propagate.argtypes = [C.c_int, C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp,
                                  C.c_int64, _dp, _dp, _dp, C.c_double, C.c_double, _dp]
    lib.orc_transmission_coefficient.argtypes = [C.c_double] * 5 + [_dp]
    lib.orc_transmission_coefficient.restype = None
    lib.orc_reflection_coefficient.argtypes = [C.c_double] * 5 + [_dp]
    lib.orc_reflection_coefficient.restype = None
    lib.orc_ray_slowness.argtypes = [C.c_double, C.c_int, _dp, _dp]
    lib.orc_ray_slowness.restype = C.c_double
    lib.orc_transmission.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp, C.c_int64,
                                     _dp, _dp, _dp]
    lib.orc_chain.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, C.c_double, _dp, _dp, C.c_int,
                              _i64p, C.POINTER(_dp), C.POINTER(_dp), C.POINTER(_dp),
                              C.POINTER(_dp), _dp, _dp, _dp, C.c_int64, _dp, _dp, _dp,
                              C.c_int, _dp, C.c_int, _dp]
    lib.orc_chain_ex.argtypes = lib.orc_chain.argtypes[:-1] + [C.c_int, _dp]
    lib.orc_reflection.argtypes = lib.orc_transmission.argtypes
    lib.orc_halton2d.argtypes = [C.c_int64, C.c_int64, _dp]
    lib.orc_sample_disc_ex.argtypes = [C.c_int] + lib.orc_sample_disc.argtypes
    lib.orc_sample_square_ex.argtypes = [C.c_int] + lib.orc_sample_square.argtypes
    lib.orc_sample_cap.argtypes = [C.c_int, C.c_uint32, C.c_int64, C.c_double, C.c_double, _dp,
                                   C.c_double, _dp, _dp, _dp, _dp]
    lib.orc_apodise.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, C.c_double, _dp]
    lib.orc_ray_field.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, C.c_double, C.c_int, _dp, _dp,
                                  _dp, C.c_int64, _dp, _dp, _dp, C.c_int, _dp, _dp]
    lib.orc_to_pressure.argtypes = [C.c_int64, _dp, C.c_double, C.c_double, _dp]
    lib.orc_to_pressure.restype = None
    lib.orc_num_threads.restype = C.c_int
    _lib = lib
    return lib


def _d(a):
    """Contiguous float64 view and its ctypes pointer (keeps the array alive)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _cplx_in(s, n):
    s = np.broadcast_to(np.asarray(s, dtype=np.complex128), (n,))
    out = np.empty(2 * n, dtype=np.float64)
    out[0::2] = s.real
    out[1::2] = s.imag
    return out


def _cplx_out(buf):
    return buf[0::2] + 1j * buf[1::2]


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with status {rc}")


def sobol2d(seed: int, n: int, first: int = 0) -> np.ndarray:
    """Scrambled 2-D Sobol points as uint32 [n, 2] (Sec. 2.3, Sobol in place of Halton)."""
    lib = _load()
    out = np.zeros((n, 2), dtype=np.uint32)
    _check(lib.orc_sobol2d(seed & 0xFFFFFFFF, first, n, out.ctypes.data_as(_u32p)), "sobol2d")
    return out


SEQ_SOBOL, SEQ_HALTON = 0, 1


def halton2d(n: int, first: int = 0) -> np.ndarray:
    """Halton points (bases 2, 3) of indices first .. first+n-1 as float64 [n, 2]."""
    lib = _load()
    out = np.zeros((n, 2))
    _check(lib.orc_halton2d(first, n, out.ctypes.data_as(_dp)), "halton2d")
    return out


def sample_disc(seed: int, n: int, radius: float, centre=(0.0, 0.0, 0.0), tilt: float = 0.0,
                seq: int = SEQ_SOBOL):
    """Transducer face samples, eq. (18); returns x, y, z, w."""
    lib = _load()
    bufs = [np.zeros(n) for _ in range(4)]
    cen, cp = _d(centre)
    _check(lib.orc_sample_disc_ex(seq, seed & 0xFFFFFFFF, n, radius, cp, tilt,
                                  *[b.ctypes.data_as(_dp) for b in bufs]), "sample_disc")
    return tuple(bufs)


def sample_square(seed: int, n: int, cx: float, cy: float, z0: float, half_width: float,
                  seq: int = SEQ_SOBOL):
    """Interface patch samples, eq. (17); returns x, y, z, w."""
    lib = _load()
    bufs = [np.zeros(n) for _ in range(4)]
    _check(lib.orc_sample_square_ex(seq, seed & 0xFFFFFFFF, n, cx, cy, z0, half_width,
                                    *[b.ctypes.data_as(_dp) for b in bufs]), "sample_square")
    return tuple(bufs)


def sample_cap(seed: int, n: int, radius: float, curvature: float, centre=(0.0, 0.0, 0.0),
               tilt: float = 0.0, seq: int = SEQ_SOBOL):
    """Focused transducer: spherical cap samples (Sec. 3.3); returns x, y, z, w."""
    lib = _load()
    bufs = [np.zeros(n) for _ in range(4)]
    cen, cp = _d(centre)
    _check(lib.orc_sample_cap(seq, seed & 0xFFFFFFFF, n, radius, curvature, cp, tilt,
                              *[b.ctypes.data_as(_dp) for b in bufs]), "sample_cap")
    return tuple(bufs)


def apodise(pts, w, centre, axis, width: float) -> np.ndarray:
    """Gaussian apodisation of the weights: w * exp(-rho^2 / width^2) (returns a copy)."""
    lib = _load()
    x, xp = _d(pts[0]); y, yp = _d(pts[1]); z, zp = _d(pts[2])
    out = np.array(w, dtype=np.float64, copy=True)
    _, cp = _d(centre); _, ap = _d(axis)
    _check(lib.orc_apodise(x.shape[0], xp, yp, zp, cp, ap, width, out.ctypes.data_as(_dp)), "apodise")
    return out


MONOPOLE, DIPOLE, OMNI = 0, 1, 2
T_GLOBAL, T_LOCAL, T_UNITY = 0, 1, 2
CHAIN_OMNI, CHAIN_ABOVE = 1, 2


def propagate(kind: int, src, weights, strength, tgt, c: float, freq: float, normal=None):
    """Pair sum of eq. (3) (kind 0) or eq. (7) kernel (kind 1) at every target.

    src, tgt: tuples (x, y, z) of float64 arrays.  strength: complex per source
    (broadcast).  Returns the complex velocity potential at the targets.
    """
    lib = _load()
    sx, sxp = _d(src[0]); sy, syp = _d(src[1]); sz, szp = _d(src[2])
    w, wp = _d(weights)
    ns = sx.shape[0]
    s, spp = _d(_cplx_in(strength, ns))
    tx, txp = _d(tgt[0]); ty, typ = _d(tgt[1]); tz, tzp = _d(tgt[2])
    nt = tx.shape[0]
    out = np.zeros(2 * nt)
    if normal is None:
        nrm, nrmp = None, None
    else:
        nrm, nrmp = _d(normal)
    _check(lib.orc_propagate(kind, ns, sxp, syp, szp, wp, spp, nrmp, nt, txp, typ, tzp,
                             c, freq, out.ctypes.data_as(_dp)), "propagate")
    return _cplx_out(out)


def transmission_coefficient(sin_in: float, c1: float, rho1: float, c2: float, rho2: float) -> complex:
    """Eq. (11) with eq. (15) for the refracted angle; complex past the critical angle."""
    lib = _load()
    out = (C.c_double * 2)()
    lib.orc_transmission_coefficient(sin_in, c1, rho1, c2, rho2, out)
    return complex(out[0], out[1])


def reflection_coefficient(sin_in: float, c1: float, rho1: float, c2: float, rho2: float) -> complex:
    """Eq. (8)."""
    lib = _load()
    out = (C.c_double * 2)()
    lib.orc_reflection_coefficient(sin_in, c1, rho1, c2, rho2, out)
    return complex(out[0], out[1])


def ray_slowness(rho_h: float, h, c) -> float:
    """Conserved slowness C of eqs. (14)-(15) through len(h) layers."""
    lib = _load()
    h, hp = _d(h)
    c, cp = _d(c)
    return lib.orc_ray_slowness(rho_h, len(h), hp, cp)


def transmission(tmode: int, m: int, zif, c, rho, xc, axis, qx, qy) -> np.ndarray:
    """Per-point transmission coefficient at interface m (1-based)."""
    lib = _load()
    zif, zp = _d(zif); c, cp = _d(c); rho, rp = _d(rho)
    xc, xcp = _d(xc); axis, ap = _d(axis)
    qx, qxp = _d(qx); qy, qyp = _d(qy)
    out = np.zeros(2 * qx.shape[0])
    _check(lib.orc_transmission(tmode, m, zp, cp, rp, xcp, ap, qx.shape[0], qxp, qyp,
                                out.ctypes.data_as(_dp)), "transmission")
    return _cplx_out(out)


def reflection(tmode: int, m: int, zif, c, rho, xc, axis, qx, qy) -> np.ndarray:
    """Per-point reflection coefficient R (eq. 8) at interface m (1-based); 0 in the
    display mode."""
    lib = _load()
    zif, zp = _d(zif); c, cp = _d(c); rho, rp = _d(rho)
    xc, xcp = _d(xc); axis, ap = _d(axis)
    qx, qxp = _d(qx); qy, qyp = _d(qy)
    out = np.zeros(2 * qx.shape[0])
    _check(lib.orc_reflection(tmode, m, zp, cp, rp, xcp, ap, qx.shape[0], qxp, qyp,
                              out.ctypes.data_as(_dp)), "reflection")
    return _cplx_out(out)


def chain(xd, v0: float, xc, axis, ifaces, zif, c, rho, tgt, freqs, tmode: int,
          flags: int = 0) -> np.ndarray:
    """Transducer -> interfaces -> field points (eqs. 3, 7, 11 chained).

    xd: (x, y, z, w) of the transducer samples; ifaces: list of (x, y, z, w), one per
    interface plane z = zif[m] (normal +z); c, rho: media 0..n_if.  Returns complex
    [n_freq, n_tgt].  flags: CHAIN_OMNI (interface samples as omnidirectional sources),
    CHAIN_ABOVE (field points above the last interface: incident + reflected field).
    """
    lib = _load()
    keep = []

    def p(a):
        a, ap = _d(a)
        keep.append(a)
        return ap

    n_if = len(ifaces)
    nq = np.array([len(f[0]) for f in ifaces] + [0], dtype=np.int64)
    arrs = [(C_ptr_array([p(f[k]) for f in ifaces])) for k in range(4)]
    freqs = np.atleast_1d(np.asarray(freqs, dtype=np.float64))
    tx = np.ascontiguousarray(tgt[0], dtype=np.float64)
    out = np.zeros(2 * len(freqs) * tx.shape[0])
    rc = lib.orc_chain_ex(len(xd[0]), p(xd[0]), p(xd[1]), p(xd[2]), p(xd[3]), v0, p(xc), p(axis),
                          n_if, nq.ctypes.data_as(_i64p), *arrs, p(zif if n_if else [0.0]), p(c),
                          p(rho), tx.shape[0], p(tgt[0]), p(tgt[1]), p(tgt[2]), len(freqs),
                          p(freqs), tmode, flags, out.ctypes.data_as(_dp))
    _check(rc, "chain")
    return _cplx_out(out).reshape(len(freqs), tx.shape[0])


def ray_field(xd, v0: float, zif, c, rho, tgt, freqs) -> np.ndarray:
    """Ray-tracing model (Sec. 2.2, eq. 12 with the slowness of eq. 14 through the planes
    z = zif[l], normal +z): transducer samples xd = (x, y, z, w) straight to the field
    points, no interface sampled.  c, rho: media 0..n_if.  Returns complex
    [n_freq, n_tgt]."""
    lib = _load()
    keep = []

    def p(a):
        a, ap = _d(a)
        keep.append(a)
        return ap

    zif = np.atleast_1d(np.asarray(zif, dtype=np.float64))
    freqs = np.atleast_1d(np.asarray(freqs, dtype=np.float64))
    tx = np.ascontiguousarray(tgt[0], dtype=np.float64)
    out = np.zeros(2 * len(freqs) * tx.shape[0])
    rc = lib.orc_ray_field(len(xd[0]), p(xd[0]), p(xd[1]), p(xd[2]), p(xd[3]), v0, len(zif),
                           p(zif if len(zif) else [0.0]), p(c), p(rho), tx.shape[0], p(tgt[0]),
                           p(tgt[1]), p(tgt[2]), len(freqs), p(freqs), out.ctypes.data_as(_dp))
    _check(rc, "ray_field")
    return _cplx_out(out).reshape(len(freqs), tx.shape[0])


def C_ptr_array(ptrs):
    arr = (_dp * max(len(ptrs), 1))()
    for i, q in enumerate(ptrs):
        arr[i] = q
    return arr


def to_pressure(phi, rho: float, freq: float) -> np.ndarray:
    """p = i omega rho phi (velocity potential to pressure, exp(-i omega t))."""
    lib = _load()
    phi = np.asarray(phi, dtype=np.complex128)
    n = phi.size
    src = _cplx_in(phi.ravel(), n)
    out = np.zeros(2 * n)
    lib.orc_to_pressure(n, src.ctypes.data_as(_dp), rho, freq, out.ctypes.data_as(_dp))
    return _cplx_out(out).reshape(phi.shape)


def num_threads() -> int:
    """OpenMP threads the reference uses."""
    return int(_load().orc_num_threads())

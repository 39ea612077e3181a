"""Python binding of librsi: same names as the C ABI, argument marshalling only.

Tensors are torch CUDA (HIP) tensors; every call enqueues on
``torch.cuda.current_stream()``.  Point coordinates and weights are float64; complex
strengths are complex128; outputs are complex64 (RSI_FP32) or complex128 (RSI_FP64).
No arithmetic of the method happens here: every step runs in the library's kernels.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Optional, Sequence

import torch

from . import _lib as L

RSI_MONOPOLE, RSI_DIPOLE, RSI_OMNI = 0, 1, 2
RSI_FP32, RSI_FP64 = 0, 1
RSI_T_GLOBAL, RSI_T_LOCAL, RSI_T_UNITY = 0, 1, 2
RSI_FLAG_PLANAR_Z = 1
RSI_CHAIN_OMNI, RSI_CHAIN_ABOVE = 1, 2
RSI_SEQ_SOBOL, RSI_SEQ_HALTON = 0, 1

_OUT_DTYPE = {RSI_FP32: torch.complex64, RSI_FP64: torch.complex128}
RSIError = L.RSIError


def rsi_set_check_finite(enable: bool) -> bool:
    """Turn the library's non-finite input check on or off; returns the previous setting."""
    return bool(L.load().rsi_set_check_finite(1 if enable else 0))


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype: torch.dtype, what: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return t


def _ptr(t: Optional[torch.Tensor]) -> C.c_void_p:
    return C.c_void_p(t.data_ptr() if t is not None and t.numel() > 0 else None)


def _points(x, y, z, what: str) -> L.rsi_points:
    for t, nm in ((x, "x"), (y, "y"), (z, "z")):
        _dev(t, torch.float64, f"{what}.{nm}")
    n = x.numel()
    if y.numel() != n or z.numel() != n:
        raise ValueError(f"{what}: x, y, z lengths differ")
    return L.rsi_points(_ptr(x), _ptr(y), _ptr(z), n)


def _dvec(v) -> C.Array:
    arr = (C.c_double * len(v))(*[float(a) for a in v])
    return arr


def _media(media) -> C.Array:
    arr = (L.rsi_medium * len(media))()
    for i, (c, rho) in enumerate(media):
        arr[i] = L.rsi_medium(float(c), float(rho))
    return arr


# ---------------------------------------------------------------------------- a1
def rsi_sobol2d(seed: int, n: int, first: int = 0, device="cuda") -> torch.Tensor:
    """Scrambled Sobol points as int32-stored uint32 pairs [n, 2] (bit patterns)."""
    out = torch.empty((n, 2), dtype=torch.int32, device=device)
    L.check(L.load().rsi_sobol2d(seed & 0xFFFFFFFF, first, n, _ptr(out), _stream()), "rsi_sobol2d")
    return out


def rsi_halton2d(n: int, first: int = 0, device="cuda") -> torch.Tensor:
    """Halton points (bases 2, 3) of indices first .. first+n-1, float64 [n, 2]."""
    out = torch.empty((n, 2), dtype=torch.float64, device=device)
    L.check(L.load().rsi_halton2d(first, n, _ptr(out), _stream()), "rsi_halton2d")
    return out


def rsi_sample_disc(seed: int, n: int, radius: float, centre=(0.0, 0.0, 0.0), tilt: float = 0.0,
                    device="cuda", seq: int = RSI_SEQ_SOBOL):
    """Piston face samples (eq. 18): returns x, y, z, w (float64)."""
    bufs = [torch.empty(n, dtype=torch.float64, device=device) for _ in range(4)]
    L.check(L.load().rsi_sample_disc_ex(seq, seed & 0xFFFFFFFF, n, radius, _dvec(centre), tilt,
                                        *[_ptr(b) for b in bufs], _stream()), "rsi_sample_disc_ex")
    return tuple(bufs)


def rsi_sample_square(seed: int, n: int, cx: float, cy: float, z0: float, half_width: float,
                      device="cuda", seq: int = RSI_SEQ_SOBOL):
    """Interface patch samples (eq. 17): returns x, y, z, w (float64)."""
    bufs = [torch.empty(n, dtype=torch.float64, device=device) for _ in range(4)]
    L.check(L.load().rsi_sample_square_ex(seq, seed & 0xFFFFFFFF, n, cx, cy, z0, half_width,
                                          *[_ptr(b) for b in bufs], _stream()), "rsi_sample_square_ex")
    return tuple(bufs)


def rsi_sample_cap(seed: int, n: int, radius: float, curvature: float, centre=(0.0, 0.0, 0.0),
                   tilt: float = 0.0, device="cuda", seq: int = RSI_SEQ_SOBOL):
    """Focused transducer (Sec. 3.3): spherical-cap samples; returns x, y, z, w."""
    bufs = [torch.empty(n, dtype=torch.float64, device=device) for _ in range(4)]
    L.check(L.load().rsi_sample_cap(seq, seed & 0xFFFFFFFF, n, radius, curvature, _dvec(centre), tilt,
                                    *[_ptr(b) for b in bufs], _stream()), "rsi_sample_cap")
    return tuple(bufs)


def rsi_apodise(pts, w: torch.Tensor, centre, axis, width: float) -> torch.Tensor:
    """Gaussian apodisation of the weights in place: w *= exp(-rho^2 / width^2)."""
    for a, name in zip(pts, "xyz"):
        _dev(a, torch.float64, name)
    _dev(w, torch.float64, "w")
    L.check(L.load().rsi_apodise(w.numel(), _ptr(pts[0]), _ptr(pts[1]), _ptr(pts[2]), _dvec(centre),
                                 _dvec(axis), width, _ptr(w), _stream()), "rsi_apodise")
    return w


# ---------------------------------------------------------------------------- a2
def rsi_transmission(tmode: int, m: int, zif: Sequence[float], media, xc, axis,
                     qx: torch.Tensor, qy: torch.Tensor) -> torch.Tensor:
    """Per-sample transmission coefficient at interface m (1-based), complex128."""
    _dev(qx, torch.float64, "qx")
    _dev(qy, torch.float64, "qy")
    out = torch.empty(qx.numel(), dtype=torch.complex128, device=qx.device)
    L.check(L.load().rsi_transmission(tmode, m, _dvec(zif), _media(media), _dvec(xc), _dvec(axis),
                                      qx.numel(), _ptr(qx), _ptr(qy), _ptr(out), _stream()),
            "rsi_transmission")
    return out


def rsi_reflection(tmode: int, m: int, zif: Sequence[float], media, xc, axis,
                   qx: torch.Tensor, qy: torch.Tensor) -> torch.Tensor:
    """Per-sample reflection coefficient (eq. 8) at interface m (1-based), complex128."""
    _dev(qx, torch.float64, "qx")
    _dev(qy, torch.float64, "qy")
    out = torch.empty(qx.numel(), dtype=torch.complex128, device=qx.device)
    L.check(L.load().rsi_reflection(tmode, m, _dvec(zif), _media(media), _dvec(xc), _dvec(axis),
                                    qx.numel(), _ptr(qx), _ptr(qy), _ptr(out), _stream()),
            "rsi_reflection")
    return out


# ---------------------------------------------------------------------------- a3/a4
def rsi_propagate(src, w: torch.Tensor, vel: torch.Tensor, tgt, c: float, freq: float,
                  kind: int, prec: int, normal=None, rho: float = 1000.0,
                  out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """phi at the targets (complex64 for RSI_FP32, complex128 for RSI_FP64)."""
    return rsi_propagate_ex(src, w, vel, tgt, c, freq, kind, prec, 0, normal, rho, out)


def rsi_propagate_ex(src, w: torch.Tensor, vel: torch.Tensor, tgt, c: float, freq: float,
                     kind: int, prec: int, flags: int, normal=None, rho: float = 1000.0,
                     out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """rsi_propagate with RSI_FLAG_* flags."""
    sp = _points(*src, "src")
    tp = _points(*tgt, "tgt")
    _dev(w, torch.float64, "w")
    _dev(vel, torch.complex128, "vel")
    if out is None:
        out = torch.empty(tp.n, dtype=_OUT_DTYPE[prec], device=tgt[0].device)
    _dev(out, _OUT_DTYPE[prec], "out")
    nrm = _dvec(normal) if normal is not None else None
    L.check(L.load().rsi_propagate_ex(C.byref(sp), _ptr(w), _ptr(vel), nrm, C.byref(tp),
                                      L.rsi_medium(c, rho), freq, kind, prec, flags, _ptr(out),
                                      _stream()), "rsi_propagate_ex")
    return out


def rsi_propagate_multifreq(src, w: torch.Tensor, vel: Optional[torch.Tensor], tgt, c: float, freqs,
                            kind: int, prec: int, flags: int = 0, normal=None, rho: float = 1000.0,
                            out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """phi at the targets for every frequency, complex [n_freq, n_tgt]; vel: complex128
    [n_freq, n_src] per-frequency strengths, or None for 1 everywhere."""
    sp = _points(*src, "src")
    tp = _points(*tgt, "tgt")
    _dev(w, torch.float64, "w")
    freqs = [float(f) for f in freqs]
    if vel is not None:
        _dev(vel, torch.complex128, "vel")
        if vel.numel() != len(freqs) * sp.n:
            raise ValueError("vel must hold n_freq x n_src strengths")
    if out is None:
        out = torch.empty((len(freqs), tp.n), dtype=_OUT_DTYPE[prec], device=tgt[0].device)
    _dev(out, _OUT_DTYPE[prec], "out")
    nrm = _dvec(normal) if normal is not None else None
    L.check(L.load().rsi_propagate_multifreq(C.byref(sp), _ptr(w), _ptr(vel), nrm, C.byref(tp),
                                             L.rsi_medium(c, rho), _dvec(freqs) if freqs else None,
                                             len(freqs), kind, prec, flags, _ptr(out), _stream()),
            "rsi_propagate_multifreq")
    return out


def rsi_propagate_noalloc(src, w: torch.Tensor, vel: torch.Tensor, tgt, c: float, freq: float,
                          kind: int, prec: int, flags: int, out: torch.Tensor, normal=None,
                          rho: float = 1000.0) -> torch.Tensor:
    """rsi_propagate_ex with its workspace in the library's fixed device array (no device
    allocation); `out` is required so that the call allocates nothing."""
    sp = _points(*src, "src")
    tp = _points(*tgt, "tgt")
    _dev(w, torch.float64, "w")
    _dev(vel, torch.complex128, "vel")
    _dev(out, _OUT_DTYPE[prec], "out")
    if out.numel() != tp.n:
        raise ValueError("out must hold one value per field point")
    nrm = _dvec(normal) if normal is not None else None
    L.check(L.load().rsi_propagate_noalloc(C.byref(sp), _ptr(w), _ptr(vel), nrm, C.byref(tp),
                                           L.rsi_medium(c, rho), freq, kind, prec, flags, _ptr(out),
                                           _stream()), "rsi_propagate_noalloc")
    return out


# ---------------------------------------------------------------------------- a5
@dataclass
class Transducer:
    x: torch.Tensor
    y: torch.Tensor
    z: torch.Tensor
    w: torch.Tensor
    v0: float = 1.0
    centre: Sequence[float] = (0.0, 0.0, 0.0)
    axis: Sequence[float] = (0.0, 0.0, 1.0)

    def c_struct(self) -> L.rsi_transducer:
        _dev(self.w, torch.float64, "transducer.w")
        return L.rsi_transducer(_points(self.x, self.y, self.z, "transducer"), _ptr(self.w),
                                float(self.v0), _dvec(self.centre), _dvec(self.axis))


@dataclass
class Interface:
    x: torch.Tensor
    y: torch.Tensor
    z: torch.Tensor
    w: torch.Tensor
    depth: float

    def c_struct(self) -> L.rsi_interface:
        _dev(self.w, torch.float64, "interface.w")
        return L.rsi_interface(_points(self.x, self.y, self.z, "interface"), _ptr(self.w),
                               float(self.depth))


def _chain_args(xd: Transducer, ifaces: Sequence[Interface], media, tgt, freqs):
    xs = xd.c_struct()
    arr = (L.rsi_interface * max(len(ifaces), 1))()
    for i, f in enumerate(ifaces):
        arr[i] = f.c_struct()
    if len(media) != len(ifaces) + 1:
        raise ValueError("need one medium per layer: len(media) == len(ifaces) + 1")
    tp = _points(*tgt, "tgt")
    fr = _dvec(list(freqs))
    return xs, arr, _media(media), tp, fr


def rsi_chain(xd: Transducer, ifaces: Sequence[Interface], media, tgt, freqs, tmode: int,
              prec: int, out: Optional[torch.Tensor] = None, flags: int = 0) -> torch.Tensor:
    """Field after the whole stack, complex [n_freq, n_tgt] (rsi_chain_ex with
    RSI_CHAIN_* flags: omnidirectional interface sources, or field points above the
    last interface with the reflected field)."""
    xs, arr, med, tp, fr = _chain_args(xd, ifaces, media, tgt, freqs)
    if out is None:
        out = torch.empty((len(freqs), tp.n), dtype=_OUT_DTYPE[prec], device=tgt[0].device)
    _dev(out, _OUT_DTYPE[prec], "out")
    L.check(L.load().rsi_chain_ex(C.byref(xs), arr, len(ifaces), med, C.byref(tp), fr, len(freqs),
                                  tmode, prec, flags, _ptr(out), _stream()), "rsi_chain_ex")
    return out


# ---------------------------------------------------------------------------- ray tracing
def rsi_ray_field(xd: Transducer, zif: Sequence[float], media, tgt, freqs, prec: int,
                  out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Ray-tracing model (Sec. 2.2, eq. 12): transducer samples straight to the field
    points through the planes z = zif[l]; complex [n_freq, n_tgt]."""
    xs = xd.c_struct()
    zif = [float(z) for z in zif]
    if len(media) != len(zif) + 1:
        raise ValueError("need one medium per layer: len(media) == len(zif) + 1")
    tp = _points(*tgt, "tgt")
    fr = _dvec(list(freqs))
    if out is None:
        out = torch.empty((len(freqs), tp.n), dtype=_OUT_DTYPE[prec], device=tgt[0].device)
    _dev(out, _OUT_DTYPE[prec], "out")
    L.check(L.load().rsi_ray_field(C.byref(xs), _dvec(zif) if zif else None, len(zif), _media(media),
                                   C.byref(tp), fr, len(freqs), prec, _ptr(out), _stream()),
            "rsi_ray_field")
    return out


# ---------------------------------------------------------------------------- a7
@dataclass
class Instance:
    src: tuple
    w: torch.Tensor
    tgt: tuple
    c: float
    freq: float
    kind: int = RSI_MONOPOLE
    vel: Optional[torch.Tensor] = None
    v0: float = 1.0
    normal: Sequence[float] = (0.0, 0.0, 1.0)
    rho: float = 1000.0
    out: Optional[torch.Tensor] = None

    def c_struct(self, prec: int) -> L.rsi_instance:
        sp = _points(*self.src, "instance.src")
        tp = _points(*self.tgt, "instance.tgt")
        _dev(self.w, torch.float64, "instance.w")
        if self.vel is not None:
            _dev(self.vel, torch.complex128, "instance.vel")
        if self.out is None:
            self.out = torch.empty(tp.n, dtype=_OUT_DTYPE[prec], device=self.tgt[0].device)
        _dev(self.out, _OUT_DTYPE[prec], "instance.out")
        return L.rsi_instance(sp, _ptr(self.w), _ptr(self.vel), float(self.v0), _dvec(self.normal),
                              tp, L.rsi_medium(self.c, self.rho), float(self.freq), int(self.kind),
                              _ptr(self.out))


def _instances(insts: Sequence[Instance], prec: int):
    arr = (L.rsi_instance * max(len(insts), 1))()
    for i, it in enumerate(insts):
        arr[i] = it.c_struct(prec)
    return arr


def rsi_propagate_batched(insts: Sequence[Instance], prec: int) -> None:
    """All instances in one persistent launch; results land in each instance's .out."""
    arr = _instances(insts, prec)
    L.check(L.load().rsi_propagate_batched(arr, len(insts), prec, _stream()), "rsi_propagate_batched")


def rsi_autotune_batched(insts: Sequence[Instance], prec: int) -> None:
    arr = _instances(insts, prec)
    L.check(L.load().rsi_autotune_batched(arr, len(insts), prec), "rsi_autotune_batched")


class Plan:
    """A captured chain or batched launch (hipGraph), replayed by execute()."""

    def __init__(self, handle: C.c_void_p, keep: list):
        self._h = handle
        self._keep = keep  # tensors whose addresses the graph binds

    @classmethod
    def chain(cls, xd: Transducer, ifaces: Sequence[Interface], media, tgt, freqs, tmode: int,
              prec: int, out: Optional[torch.Tensor] = None, flags: int = 0) -> "Plan":
        xs, arr, med, tp, fr = _chain_args(xd, ifaces, media, tgt, freqs)
        if out is None:
            out = torch.empty((len(freqs), tp.n), dtype=_OUT_DTYPE[prec], device=tgt[0].device)
        h = C.c_void_p()
        L.check(L.load().rsi_plan_create_chain_ex(C.byref(h), C.byref(xs), arr, len(ifaces), med,
                                                  C.byref(tp), fr, len(freqs), tmode, prec, flags,
                                                  _ptr(out)),
                "rsi_plan_create_chain_ex")
        plan = cls(h, [xd, list(ifaces), tgt])
        plan.out = out
        return plan

    @classmethod
    def batched(cls, insts: Sequence[Instance], prec: int) -> "Plan":
        arr = _instances(insts, prec)
        h = C.c_void_p()
        L.check(L.load().rsi_plan_create_batched(C.byref(h), arr, len(insts), prec),
                "rsi_plan_create_batched")
        return cls(h, list(insts))

    def execute(self) -> None:
        L.check(L.load().rsi_plan_execute(self._h, _stream()), "rsi_plan_execute")

    def destroy(self) -> None:
        if self._h:
            L.check(L.load().rsi_plan_destroy(self._h), "rsi_plan_destroy")
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


# ---------------------------------------------------------------------------- a8
def rsi_to_pressure(phi: torch.Tensor, rho: float, freq: float) -> torch.Tensor:
    prec = RSI_FP32 if phi.dtype == torch.complex64 else RSI_FP64
    _dev(phi, _OUT_DTYPE[prec], "phi")
    p = torch.empty_like(phi)
    L.check(L.load().rsi_to_pressure(phi.numel(), _ptr(phi), prec, rho, freq, _ptr(p), _stream()),
            "rsi_to_pressure")
    return p

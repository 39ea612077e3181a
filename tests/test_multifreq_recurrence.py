"""Float32 emulation of the multi-frequency kernel's per-pair arithmetic (host only): the
phasor e^{i k_q r} carried from one frequency to the next by the two-term recurrence
e_{q+1} = 2 cos(dk r) e_q - e_{q-1}, the dipole factor written as (1 - i k_q r) with k_q r
carried by adds, and blocks of 32 frequencies restarted at their 17th frequency from a third
phasor.  The recurrence's drift grows along a block, so without the restart a block of 32
loses accuracy; with it the error stays that of a block of 16, far inside the FP32 path's
1e-4 bar.  The exact sums are FP64 on the same points (multi-frequency superposition, Sec. 4;
dipole kernel, eqs. 2 and 7)."""
import numpy as np

F32 = np.float32


def _r32(x):
    return np.asarray(x, np.float64).astype(F32)


def _fma(a, b, c):
    return (np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64)).astype(F32)


def _stage(seed=3, ns=1 << 12, nt=24):
    """Sources on a 60 mm interface patch, field points 1-31 mm below it in the solid
    (c = 5900 m/s), 64 frequencies 1-10 MHz, complex strengths of a refracted beam."""
    rng = np.random.default_rng(seed)
    c = 5900.0
    freqs = 1e6 + 9e6 * np.arange(64) / 63
    sx, sy = 0.03 * (2 * rng.random(ns) - 1), 0.03 * (2 * rng.random(ns) - 1)
    tx, ty = 0.005 + 0.015 * (2 * rng.random(nt) - 1), 0.015 * (2 * rng.random(nt) - 1)
    tz = 0.001 + 0.030 * rng.random(nt)
    env = np.exp(-(sx ** 2 + sy ** 2) / 0.008 ** 2)
    S = env[None, :] * np.exp(1j * 2 * np.pi * freqs[:, None] / 2700.0 * 0.42 * sx[None, :])
    S = S * (-(0.06 ** 2 / ns) / (2 * np.pi))
    return c, freqs, (sx, sy), (tx, ty, tz), S


def _emulate(c, freqs, src, tgt, S, nb, restart):
    """The kernel's per-pair FP32 arithmetic, one block of nb frequencies at a time: phases
    in revolutions from the FP64 reference distance (hardware sin/cos modelled as the exact
    value of the rounded argument, rounded), the recurrence and the dipole factor in FP32;
    the terms are then summed in FP64 (the summation's rounding is not what this test is
    about)."""
    sx, sy = src
    tx, ty, tz = tgt
    df = freqs[1] - freqs[0]
    out = np.zeros((len(freqs), len(tx)), complex)
    Sx, Sy = S.real.astype(F32), S.imag.astype(F32)
    for i in range(len(tx)):
        rr = np.sqrt(tx[i] ** 2 + ty[i] ** 2 + tz[i] ** 2)
        r = np.sqrt((tx[i] - sx) ** 2 + (ty[i] - sy) ** 2 + tz[i] ** 2)
        ir = _r32(1 / r)
        dr = r - rr
        for q0 in range(0, len(freqs), nb):
            fb = freqs[q0]
            ph = lambda f: _r32((dr * f / c + (rr * f / c) % 1.0) % 1.0)
            phb, phd, phh = ph(fb), _r32((dr * df / c + (rr * df / c) % 1.0) % 1.0), ph(fb + 16 * df)
            cd, sd = _r32(np.cos(2 * np.pi * phd.astype(np.float64))), _r32(np.sin(2 * np.pi * phd.astype(np.float64)))
            amp = _r32(-_r32(_r32(tz[i] * ir) * ir) * ir)
            r32 = _r32(r)
            kr = _r32(_r32(2 * np.pi * fb / c) * r32)
            dkr = _r32(_r32(2 * np.pi * df / c) * r32)
            er = _r32(_r32(np.cos(2 * np.pi * phb.astype(np.float64))) * amp)
            ei = _r32(_r32(np.sin(2 * np.pi * phb.astype(np.float64))) * amp)
            nr, ni = _fma(er, cd, -_r32(ei * sd)), _fma(er, sd, _r32(ei * cd))
            tc = _r32(cd + cd)
            for q in range(nb):
                if q0 + q >= len(freqs):
                    break
                gr, gi = _fma(kr, ei, er), _fma(-kr, er, ei)
                kr = _r32(kr + dkr)
                acc = np.sum(Sx[q0 + q].astype(np.float64) * gr - Sy[q0 + q] * gi) + \
                    1j * np.sum(Sx[q0 + q].astype(np.float64) * gi + Sy[q0 + q] * gr)
                out[q0 + q, i] = acc
                if q == 15 and nb > 16 and restart:
                    er = _r32(_r32(np.cos(2 * np.pi * phh.astype(np.float64))) * amp)
                    ei = _r32(_r32(np.sin(2 * np.pi * phh.astype(np.float64))) * amp)
                    nr, ni = _fma(er, cd, -_r32(ei * sd)), _fma(er, sd, _r32(ei * cd))
                else:
                    tr, ti = _fma(tc, nr, -er), _fma(tc, ni, -ei)
                    er, ei, nr, ni = nr, ni, tr, ti
    return out


def _exact(c, freqs, src, tgt, S):
    sx, sy = src
    tx, ty, tz = tgt
    out = np.zeros((len(freqs), len(tx)), complex)
    for i in range(len(tx)):
        r = np.sqrt((tx[i] - sx) ** 2 + (ty[i] - sy) ** 2 + tz[i] ** 2)
        for q, f in enumerate(freqs):
            k = 2 * np.pi * f / c
            out[q, i] = np.sum(S[q] * (tz[i] / r ** 2) * (1j * k - 1 / r) * np.exp(1j * k * r))
    return out


def test_recurrence_and_restart_accuracy():
    c, freqs, src, tgt, S = _stage()
    ref = _exact(c, freqs, src, tgt, S)
    err = {}
    for name, nb, restart in (("16", 16, False), ("32", 32, False), ("32r", 32, True)):
        got = _emulate(c, freqs, src, tgt, S, nb, restart)
        err[name] = (np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)).max()
    print({k: f"{v:.2e}" for k, v in err.items()})
    assert err["32r"] < 1e-5 and err["16"] < 1e-5
    assert err["32r"] < 2 * err["16"]            # the restart keeps a block of 16's accuracy
    assert err["32"] > 1.5 * err["32r"]          # and without it a block of 32 drifts further

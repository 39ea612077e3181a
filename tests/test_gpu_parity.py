"""GPU parity: the HIP library (through its C ABI) against the FP64 reference.

Tolerances: rel-L2 <= 1e-4 for the FP32 path and <= 1e-10 for the FP64 path (the
FP64 path evaluates the same operations as the reference, in another order).  Integer
work (Sobol digits) must match bit for bit.
"""
import math

import numpy as np
import pytest

from paper_2408_06765_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {0: 1e-4, 1: 1e-10}


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def devpts(p):
    return tuple(dev(np.asarray(v, dtype=np.float64)) for v in p)


# ----------------------------------------------------------------------------- a1
@pytest.mark.parametrize("seed,n,first", [(0, 1, 0), (0, 4096, 0), (12345, 1000, 0), (7, 777, 99991)])
def test_sobol_bit_exact(gpu, orc, seed, n, first):
    got = host(gpu.rsi_sobol2d(seed, n, first)).view(np.uint32)
    assert np.array_equal(got, orc.sobol2d(seed, n, first))


def test_sample_maps_match(gpu, orc):
    tilt = math.radians(10.0)
    g = [host(t) for t in gpu.rsi_sample_disc(0, 5000, W.PISTON_RADIUS, (0.001, 0.002, -0.003), tilt)]
    o = orc.sample_disc(0, 5000, W.PISTON_RADIUS, (0.001, 0.002, -0.003), tilt)
    for a, b in zip(g, o):
        assert np.max(np.abs(a - b)) <= 1e-17 + 4e-16 * np.max(np.abs(b))
    g = [host(t) for t in gpu.rsi_sample_square(1, 3001, 0.00882, 0.0, 0.05, 0.03)]
    o = orc.sample_square(1, 3001, 0.00882, 0.0, 0.05, 0.03)
    for a, b in zip(g, o):
        assert np.max(np.abs(a - b)) <= 1e-17 + 4e-16 * np.max(np.abs(b))


def test_halton_bit_exact(gpu, orc):
    for first, n in ((0, 4097), (1, 3000), (2 ** 39 - 2000, 2000)):
        g = host(gpu.rsi_halton2d(n, first))
        o = orc.halton2d(n, first)
        assert np.array_equal(g.view(np.uint64), o.view(np.uint64)), first


@pytest.mark.parametrize("seq", [0, 1])
def test_sample_maps_sequences_and_cap(gpu, orc, seq):
    """Disc, square and cap samplers with Sobol and Halton points match the reference's
    maps (FP64, libm vs device sin/cos/sqrt: a few ulp)."""
    def close(g, o):
        for a, b in zip(g, o):
            assert np.max(np.abs(host(a) - b)) <= 1e-17 + 4e-16 * np.max(np.abs(b))
    close(gpu.rsi_sample_disc(7, 5001, 0.00635, (0.001, 0.0, 0.002), 0.2, seq=seq),
          orc.sample_disc(7, 5001, 0.00635, (0.001, 0.0, 0.002), 0.2, seq=seq))
    close(gpu.rsi_sample_square(3, 4097, 0.008, -0.001, 0.05, 0.02, seq=seq),
          orc.sample_square(3, 4097, 0.008, -0.001, 0.05, 0.02, seq=seq))
    close(gpu.rsi_sample_cap(5, 6000, 0.00635, 0.033, (0.0, 0.0, 0.001), 0.1, seq=seq),
          orc.sample_cap(5, 6000, 0.00635, 0.033, (0.0, 0.0, 0.001), 0.1, seq=seq))


def test_apodise_matches(gpu, orc):
    x, y, z, w = orc.sample_cap(1, 3000, 0.00635, 0.033, (0.0, 0.0, 0.0), 0.15)
    wg = dev(w.copy())
    gpu.rsi_apodise(devpts((x, y, z)), wg, (0.0, 0.0, 0.0), (math.sin(0.15), 0.0, math.cos(0.15)), 0.004)
    ref = orc.apodise((x, y, z), w, (0.0, 0.0, 0.0), (math.sin(0.15), 0.0, math.cos(0.15)), 0.004)
    assert np.max(np.abs(host(wg) / ref - 1)) < 1e-14


# ----------------------------------------------------------------------------- a2
@pytest.mark.parametrize("tmode", [0, 1, 2])
def test_transmission_matches(gpu, orc, tmode):
    cfg = W.LayeredStack()
    c = [m[0] for m in cfg.media]
    rho = [m[1] for m in cfg.media]
    xc, axis = (0.0, 0.0, 0.0), cfg.axis
    qx, qy = W.random_cloud(5, 3000, (0.01, 0.0, 0.0), (0.03, 0.03, 0.0))[:2]
    for m in (1, 2, 3):
        got = host(gpu.rsi_transmission(tmode, m, cfg.z_if[:m], cfg.media[:m + 1], xc, axis, dev(qx), dev(qy)))
        ref = orc.transmission(tmode, m, cfg.z_if[:m], c[:m + 1], rho[:m + 1], xc, axis, qx, qy)
        assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("tmode", [0, 1, 2])
def test_reflection_matches(gpu, orc, tmode):
    cfg = W.LayeredStack()
    c = [m[0] for m in cfg.media]
    rho = [m[1] for m in cfg.media]
    xc, axis = (0.0, 0.0, 0.0), cfg.axis
    qx, qy = W.random_cloud(6, 3000, (0.01, 0.0, 0.0), (0.03, 0.03, 0.0))[:2]
    for m in (1, 2, 3):
        got = host(gpu.rsi_reflection(tmode, m, cfg.z_if[:m], cfg.media[:m + 1], xc, axis, dev(qx), dev(qy)))
        ref = orc.reflection(tmode, m, cfg.z_if[:m], c[:m + 1], rho[:m + 1], xc, axis, qx, qy)
        assert np.max(np.abs(got - ref)) < 1e-12


# ----------------------------------------------------------------------------- a3/a4
SIZES = [(1, 1), (37, 5), (1000, 1237), (5000, 3001), (70001, 613)]


def _case(seed, ns, nt, kind):
    src = W.random_cloud(seed, ns, (0.0, 0.0, 0.0), (0.015, 0.015, 0.0 if kind == 1 else 0.002))
    tgt = W.random_cloud(seed + 1, nt, (0.005, 0.0, 0.02), (0.02, 0.01, 0.015))
    s = W.random_complex(seed + 2, ns)
    w = W.random_weights(seed + 3, ns, 1e-4)
    return src, w, s, tgt


# (precision, launch): the FP64 path has one launch; FP32 also runs with each launch forced
PREC_LAUNCH = [(0, "auto"), (0, "0"), (0, "1"), (1, "auto")]


@pytest.mark.parametrize("prec,launch", PREC_LAUNCH)
@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("ns,nt", SIZES)
def test_propagate_matches_reference(gpu, orc, kind, prec, ns, nt, launch, monkeypatch):
    """Pair sums of every kind and precision; launch forces the FP32 launch with one field
    point per lane ("0") or one wave per field point ("1"), which these sizes would
    otherwise choose ("auto")."""
    if launch != "auto":
        monkeypatch.setenv("RSI_PAIRSUM_FEW", launch)
    src, w, s, tgt = _case(11 + ns, ns, nt, kind)
    c, f = (5900.0, 5.0e6) if kind == 1 else (1480.0, 5.0e6)
    ref = orc.propagate(kind, src, w, s, tgt, c, f, normal=(0.0, 0.0, 1.0))
    got = host(gpu.rsi_propagate(devpts(src), dev(w), dev(s), devpts(tgt), c, f, kind, prec,
                                 normal=(0.0, 0.0, 1.0)))
    assert rel(got, ref) <= TOL[prec], (kind, prec, ns, nt, rel(got, ref))


@pytest.mark.parametrize("launch", ["0", "1"])
@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("ns,nt", [(5, 3), (70001, 613)])
def test_propagate_planar_flag(gpu, orc, kind, ns, nt, launch, monkeypatch):
    """RSI_FLAG_PLANAR_Z (sources on one z plane): the reduced FP32 kernel keeps parity, in
    both FP32 launches."""
    monkeypatch.setenv("RSI_PAIRSUM_FEW", launch)
    src, w, s, tgt = _case(31 + ns, ns, nt, 1)
    src = (src[0], src[1], np.full(ns, 0.0123))
    tgt = (tgt[0], tgt[1], tgt[2] + 0.0123)
    ref = orc.propagate(kind, src, w, s, tgt, 5900.0, 5e6, normal=(0.0, 0.0, 1.0))
    got = host(gpu.rsi_propagate_ex(devpts(src), dev(w), dev(s), devpts(tgt), 5900.0, 5e6, kind, 0,
                                    gpu.RSI_FLAG_PLANAR_Z, normal=(0.0, 0.0, 1.0)))
    assert rel(got, ref) <= 1e-4


def test_planar_flag_rejects_tilted_normal(gpu):
    from paper_2408_06765_amd._lib import RSIError
    src, w, s, tgt = _case(1, 10, 10, 1)
    with pytest.raises(RSIError):
        gpu.rsi_propagate_ex(devpts(src), dev(w), dev(s), devpts(tgt), 1480.0, 1e6, 1, 0,
                             gpu.RSI_FLAG_PLANAR_Z, normal=(0.1, 0.0, 1.0))



@pytest.mark.parametrize("kind", [0, 1])
def test_propagate_large_target_count(gpu, orc, kind):
    """2^25 field points (a 131072-workgroup grid, one source split) from 37 sources, and
    2^22 sources onto 3 field points (the one-wave-per-point launch at its widest split):
    sampled outputs against the reference, FP32."""
    import torch
    rng = np.random.default_rng(77 + kind)
    src, w, s, _ = _case(31 + kind, 37, 1, kind)
    nt = 1 << 25
    tgt = tuple(torch.as_tensor(rng.uniform(lo, hi, nt), device="cuda")
                for lo, hi in ((-0.02, 0.03), (-0.01, 0.01), (0.006, 0.04)))
    got = gpu.rsi_propagate(devpts(src), dev(w), dev(s), tgt, 5900.0, 5.0e6, kind, 0, normal=(0.0, 0.0, 1.0))
    pick = torch.as_tensor(np.sort(rng.choice(nt, 2000, replace=False)), device="cuda")
    sub = tuple(host(t[pick]) for t in tgt)
    ref = orc.propagate(kind, src, w, s, sub, 5900.0, 5.0e6, normal=(0.0, 0.0, 1.0))
    assert rel(host(got[pick]), ref) <= TOL[0]
    del got, tgt
    ns = 1 << 22
    src2 = W.random_cloud(41 + kind, ns, (0.0, 0.0, 0.0), (0.015, 0.015, 0.0 if kind == 1 else 0.002))
    w2, s2 = W.random_weights(42, ns, 1e-6), W.random_complex(43, ns)
    tgt2 = W.random_cloud(44, 3, (0.005, 0.0, 0.02), (0.02, 0.01, 0.015))
    got2 = host(gpu.rsi_propagate(devpts(src2), dev(w2), dev(s2), devpts(tgt2), 5900.0, 5.0e6, kind, 0,
                                  normal=(0.0, 0.0, 1.0)))
    ref2 = orc.propagate(kind, src2, w2, s2, tgt2, 5900.0, 5.0e6, normal=(0.0, 0.0, 1.0))
    assert rel(got2, ref2) <= TOL[0]

@pytest.mark.parametrize("prec", [0, 1])
def test_propagate_empty_sources_give_zero(gpu, prec):
    import torch
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    tgt = devpts(W.random_cloud(1, 300, (0, 0, 0.02), (0.01, 0.01, 0.01)))
    out = gpu.rsi_propagate((e, e, e), e, torch.empty(0, dtype=torch.complex128, device="cuda"), tgt,
                            1480.0, 1e6, 0, prec)
    assert np.all(host(out) == 0)


def test_fp32_bitwise_repeatable(gpu):
    src, w, s, tgt = _case(3, 70001, 2000, 1)
    args = (devpts(src), dev(w), dev(s), devpts(tgt), 5900.0, 5e6, 1, 0)
    a = host(gpu.rsi_propagate(*args, normal=(0, 0, 1)))
    b = host(gpu.rsi_propagate(*args, normal=(0, 0, 1)))
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_high_frequency_phase_accuracy(gpu, orc):
    """10 MHz in water over 0.1 m: k r ~ 4e3 rad; the FP32 path keeps 1e-4."""
    src = W.random_cloud(21, 20000, (0.0, 0.0, 0.0), (0.03, 0.03, 0.0))
    tgt = W.random_cloud(22, 500, (0.0, 0.0, 0.08), (0.02, 0.02, 0.02))
    s = W.random_complex(23, 20000)
    w = W.random_weights(24, 20000)
    ref = orc.propagate(1, src, w, s, tgt, 1480.0, 10e6, normal=(0, 0, 1))
    got = host(gpu.rsi_propagate(devpts(src), dev(w), dev(s), devpts(tgt), 1480.0, 10e6, 1, 0, normal=(0, 0, 1)))
    assert rel(got, ref) <= 1e-4


@pytest.mark.parametrize("f", [12.0e6, 14.0e6])
@pytest.mark.parametrize("flags", [0, 1])
def test_phase_argument_on_both_sides_of_sin_range(gpu, orc, f, flags):
    """The FP32 kernels skip the explicit fract of the phase when the source set's half
    diagonal R satisfies R f / c < 250 revolutions: a 40 mm square in water has
    R f / c ~ 230 at 12 MHz and ~ 270 at 14 MHz, one case on each side."""
    src = W.random_cloud(41, 20000, (0.0, 0.0, 0.0), (0.02, 0.02, 0.0))
    tgt = W.random_cloud(42, 700, (0.0, 0.0, 0.045), (0.02, 0.02, 0.015))
    s = W.random_complex(43, 20000)
    w = W.random_weights(44, 20000)
    half_diag = 0.5 * math.sqrt(sum((float(np.ptp(v))) ** 2 for v in src))
    assert (half_diag * f / 1480.0 < 250.0) == (f < 13e6)
    ref = orc.propagate(1, src, w, s, tgt, 1480.0, f, normal=(0, 0, 1))
    got = host(gpu.rsi_propagate_ex(devpts(src), dev(w), dev(s), devpts(tgt), 1480.0, f, 1, 0, flags,
                                    normal=(0, 0, 1)))
    assert rel(got, ref) <= 1e-4


# ----------------------------------------------------------------------------- a5
def _small_chain(orc, n_if_pts, ifaces_z, media, tilt, n_tgt, seed=0):
    a = W.PISTON_RADIUS
    xd = orc.sample_disc(seed, 4096, a, (0.0, 0.0, 0.0), tilt)
    centres = W.snell_intercepts(0.0, tilt, list(ifaces_z), [m[0] for m in media])
    ifs = [orc.sample_square(seed + 1 + m, n_if_pts, centres[m], 0.0, ifaces_z[m], 0.02)
           for m in range(len(ifaces_z))]
    tgt = W.random_cloud(seed + 9, n_tgt, (centres[-1] + 0.005, 0.0, ifaces_z[-1] + 0.012), (0.01, 0.004, 0.01))
    return xd, ifs, tgt


def _gpu_chain(gpu, xd, ifs, zs, media, tgt, freqs, tmode, prec, axis):
    T = gpu.Transducer(*devpts(xd[:3]), dev(xd[3]), 1.0, (0.0, 0.0, 0.0), axis)
    I = [gpu.Interface(*devpts(q[:3]), dev(q[3]), z) for q, z in zip(ifs, zs)]
    return host(gpu.rsi_chain(T, I, media, devpts(tgt), freqs, tmode, prec))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("tmode", [0, 1, 2])
def test_one_interface_chain(gpu, orc, prec, tmode):
    tilt = math.radians(10.0)
    axis = (math.sin(tilt), 0.0, math.cos(tilt))
    media = (W.WATER, W.STEEL_5900)
    xd, ifs, tgt = _small_chain(orc, 1 << 13, (0.05,), media, tilt, 1500)
    freqs = [2.5e6]
    ref = orc.chain(xd, 1.0, (0, 0, 0), axis, ifs, [0.05], [m[0] for m in media], [m[1] for m in media],
                    tgt, freqs, tmode)
    got = _gpu_chain(gpu, xd, ifs, [0.05], media, tgt, freqs, tmode, prec, axis)
    assert rel(got, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
def test_layered_chain_three_frequencies(gpu, orc, prec):
    cfg = W.LayeredStack()
    axis = cfg.axis
    xd, ifs, tgt = _small_chain(orc, 1 << 12, cfg.z_if, cfg.media, cfg.tilt, 700)
    freqs = [1.0e6, 5.5e6, 10.0e6]
    ref = orc.chain(xd, 1.0, (0, 0, 0), axis, ifs, list(cfg.z_if), [m[0] for m in cfg.media],
                    [m[1] for m in cfg.media], tgt, freqs, 1)
    got = _gpu_chain(gpu, xd, ifs, cfg.z_if, cfg.media, tgt, freqs, 1, prec, axis)
    for f in range(len(freqs)):
        assert rel(got[f], ref[f]) <= TOL[prec], (f, rel(got[f], ref[f]))


@pytest.mark.parametrize("prec", [0, 1])
def test_chain_nonuniform_frequency_list(gpu, orc, prec):
    """A frequency list that is not a uniform grid (multi-frequency superposition, Sec. 4):
    the chain runs stage by stage for each frequency; every frequency of 1.0, 2.2, 2.9,
    7.3 MHz through the three-interface stack against the reference."""
    cfg = W.LayeredStack()
    xd, ifs, tgt = _small_chain(orc, 1 << 12, cfg.z_if, cfg.media, cfg.tilt, 600, seed=5)
    freqs = [1.0e6, 2.2e6, 2.9e6, 7.3e6]
    ref = orc.chain(xd, 1.0, (0, 0, 0), cfg.axis, ifs, list(cfg.z_if), [m[0] for m in cfg.media],
                    [m[1] for m in cfg.media], tgt, freqs, 1)
    got = _gpu_chain(gpu, xd, ifs, cfg.z_if, cfg.media, tgt, freqs, 1, prec, cfg.axis)
    for f in range(len(freqs)):
        assert rel(got[f], ref[f]) <= TOL[prec], (f, rel(got[f], ref[f]))


@pytest.mark.parametrize("flags,nf", [(0, 20), (1, 20), (2, 20), (0, 40), (0, 50)])
def test_chain_uniform_grid_ragged_block(gpu, orc, flags, nf):
    """Uniform grids of 20, 40 and 50 frequencies, 1-10 MHz, whose FP32 multi-frequency
    stages end in a ragged block (zero-padded strengths, outputs masked): 20 in one block
    of 32, 40 in blocks of 16 (16 + 16 + 8), 50 in blocks of 32 (32 + 18, past the restart
    of the recurrence at a block's 17th frequency).  Plain chain, omnidirectional interface
    sources, and field points above the last interface with the reflected field; every
    frequency against the reference."""
    cfg = W.LayeredStack()
    xd, ifs, tgt = _small_chain(orc, 1 << 11, cfg.z_if, cfg.media, cfg.tilt, 500, seed=6)
    if flags & 2:
        tgt = _above_targets(ifs, cfg.z_if, 500, 19)
    freqs = list(np.linspace(1.0e6, 10.0e6, nf))
    ref = orc.chain(xd, 1.0, (0, 0, 0), cfg.axis, ifs, list(cfg.z_if), [m[0] for m in cfg.media],
                    [m[1] for m in cfg.media], tgt, freqs, 1, flags=flags)
    T = gpu.Transducer(*devpts(xd[:3]), dev(xd[3]), 1.0, (0.0, 0.0, 0.0), cfg.axis)
    I = [gpu.Interface(*devpts(q[:3]), dev(q[3]), z) for q, z in zip(ifs, cfg.z_if)]
    got = host(gpu.rsi_chain(T, I, cfg.media, devpts(tgt), freqs, 1, 0, flags=flags))
    assert got.shape == (nf, len(tgt[0]))
    for f in range(len(freqs)):
        assert rel(got[f], ref[f]) <= TOL[0], (f, rel(got[f], ref[f]))


@pytest.mark.parametrize("kind", [0, 1])
def test_fp32_field_points_near_a_source(gpu, orc, kind):
    """The FP32 path does not test for close pairs; its documented behaviour: with
    s = |P - C| + R (C the sources' bounding-box centre, R its half diagonal), a field
    point at distance r >= 1e-3 s from a source gets a finite value, and at r = 1e-2 s it
    stays within 1e-2 of the reference (the close term's rounding, about 3e-7 (s/r)^2).
    Field points are placed at those distances from 64 sources in random directions
    (above the plane for the planar dipole sources)."""
    rng = np.random.default_rng(7 + kind)
    src, w, s, _ = _case(91 + kind, 5000, 1, kind)
    C = np.array([(v.max() + v.min()) / 2 for v in src])
    R = 0.5 * math.sqrt(sum(float(np.ptp(v)) ** 2 for v in src))
    idx = rng.choice(len(w), 64, replace=False)
    P = np.stack([v[idx] for v in src], 1)
    d = rng.normal(size=(64, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    if kind == 1:
        d[:, 2] = np.abs(d[:, 2]) + 0.1
        d /= np.linalg.norm(d, axis=1, keepdims=True)
    sc = np.linalg.norm(P - C, axis=1) + R
    for rho, bound in ((1e-3, None), (1e-2, 1e-2)):
        T = P + rho * sc[:, None] * d
        tgt = tuple(T[:, k].copy() for k in range(3))
        got = host(gpu.rsi_propagate(devpts(src), dev(w), dev(s), devpts(tgt), 1480.0, 2.0e6, kind, 0,
                                     normal=(0.0, 0.0, 1.0)))
        assert np.all(np.isfinite(got.view(np.float32))), rho
        if bound is not None:
            ref = orc.propagate(kind, src, w, s, tgt, 1480.0, 2.0e6, normal=(0.0, 0.0, 1.0))
            err = np.abs(got - ref) / np.abs(ref)
            assert err.max() <= bound, (rho, err.max())


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_fp64_field_point_on_a_source(gpu, orc, kind):
    """The kernel is singular on the radiating surface (Sec. 3.2): the FP64 path drops
    pairs closer than 1e-12 m.  Field points placed exactly on sources get the sum over
    the other sources -- the reference with that source removed -- and the output is
    finite everywhere."""
    src, w, s, tgt = _case(71, 3000, 400, kind)
    on = [5, 777, 2999]
    tgt = tuple(np.concatenate([t, v[on]]) for t, v in zip(tgt, src))
    got = host(gpu.rsi_propagate(devpts(src), dev(w), dev(s), devpts(tgt), 1480.0, 2.0e6, kind, 1,
                                 normal=(0.0, 0.0, 1.0)))
    assert np.all(np.isfinite(got.view(np.float64)))
    ref = orc.propagate(kind, src, w, s, tgt, 1480.0, 2.0e6, normal=(0.0, 0.0, 1.0))
    assert rel(got, ref) <= TOL[1]
    for i, j in enumerate(on):
        keep = np.arange(len(w)) != j
        p = tuple(np.array([v[j]]) for v in src)
        alone = orc.propagate(kind, tuple(v[keep] for v in src), w[keep], s[keep], p, 1480.0, 2.0e6,
                              normal=(0.0, 0.0, 1.0))
        k = len(tgt[0]) - len(on) + i
        assert abs(got[k] - alone[0]) <= 1e-10 * abs(alone[0]), (j, got[k], alone[0])


def _above_targets(ifs, zs, n, seed):
    """Field points in the medium above the last interface (between it and the one
    before, or the transducer)."""
    z_hi = zs[-1] - 0.0005
    z_lo = zs[-2] + 0.0005 if len(zs) > 1 else zs[-1] - 0.02
    cx = float(np.mean(ifs[-1][0]))
    return W.random_cloud(seed, n, (cx, 0.0, 0.5 * (z_lo + z_hi)), (0.006, 0.004, 0.5 * (z_hi - z_lo)))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("flags", [1, 2, 3])
@pytest.mark.parametrize("layout", ["one", "stack"])
@pytest.mark.parametrize("nf", [1, 3])
def test_chain_modes_match_reference(gpu, orc, prec, flags, layout, nf):
    """rsi_chain_ex: omnidirectional interface sources (flag 1) and field points above the
    last interface with the reflected field (flag 2), single frequency and a uniform
    three-frequency grid (one multi-frequency launch per stage in FP32)."""
    if layout == "one":
        tilt = math.radians(10.0)
        media, zs = (W.WATER, W.STEEL_5900), (0.05,)
    else:
        cfg = W.LayeredStack()
        tilt, media, zs = cfg.tilt, cfg.media, cfg.z_if
    axis = (math.sin(tilt), 0.0, math.cos(tilt))
    xd, ifs, tgt = _small_chain(orc, 1 << 12, zs, media, tilt, 600, seed=3)
    if flags & 2:
        tgt = _above_targets(ifs, zs, 600, 17)
    freqs = [2.5e6] if nf == 1 else [1.0e6, 3.0e6, 5.0e6]
    ref = orc.chain(xd, 1.0, (0, 0, 0), axis, ifs, list(zs), [m[0] for m in media], [m[1] for m in media],
                    tgt, freqs, 1, flags=flags)
    T = gpu.Transducer(*devpts(xd[:3]), dev(xd[3]), 1.0, (0.0, 0.0, 0.0), axis)
    I = [gpu.Interface(*devpts(q[:3]), dev(q[3]), z) for q, z in zip(ifs, zs)]
    got = host(gpu.rsi_chain(T, I, media, devpts(tgt), freqs, 1, prec, flags=flags))
    for f in range(nf):
        assert rel(got[f], ref[f]) <= TOL[prec], (f, rel(got[f], ref[f]))


def test_chain_modes_plan_replay(gpu, orc):
    """A plan of the above mode with omnidirectional sources replays to the eager result
    bit for bit, with eager work between replays."""
    import torch
    cfg = W.LayeredStack()
    xd, ifs, _ = _small_chain(orc, 1 << 11, cfg.z_if[:2], cfg.media[:3], cfg.tilt, 10)
    tg = devpts(_above_targets(ifs, cfg.z_if[:2], 500, 5))
    T = gpu.Transducer(*devpts(xd[:3]), dev(xd[3]), 1.0, (0.0, 0.0, 0.0), cfg.axis)
    I = [gpu.Interface(*devpts(q[:3]), dev(q[3]), z) for q, z in zip(ifs, cfg.z_if[:2])]
    freqs = [2e6, 3e6, 4e6]
    for prec in (0, 1):
        eager = host(gpu.rsi_chain(T, I, cfg.media[:3], tg, freqs, 1, prec, flags=3))
        plan = gpu.Plan.chain(T, I, cfg.media[:3], tg, freqs, 1, prec, flags=3)
        for rep in range(3):
            plan.out.zero_()
            plan.execute()
            torch.cuda.synchronize()
            _ = torch.randn(100, device="cuda").sum().item()
            assert np.array_equal(host(plan.out).view(np.uint64), eager.view(np.uint64))
        plan.destroy()


@pytest.mark.parametrize("prec", [0, 1])
def test_focused_apodised_chain(gpu, orc, prec):
    """Focused transducer (spherical cap, Sec. 3.3) with a Gaussian apodisation (Sec. 4)
    at normal incidence through a water/steel interface 10 mm away, Halton points as in
    the paper (Sec. 2.3)."""
    R, L, f = 0.033, 0.01, 2.5e6
    media = (W.WATER, W.STEEL_5900)
    xd = list(orc.sample_cap(0, 4096, W.PISTON_RADIUS, R, seq=orc.SEQ_HALTON))
    xd[3] = orc.apodise(xd[:3], xd[3], (0, 0, 0), (0, 0, 1), 0.005)
    q = orc.sample_square(0, 1 << 13, 0.0, 0.0, L, 0.012, seq=orc.SEQ_HALTON)
    tgt = W.random_cloud(7, 700, (0.0, 0.0, L + 0.008), (0.004, 0.004, 0.007))
    ref = orc.chain(xd, 1.0, (0, 0, 0), (0, 0, 1), [q], [L], [m[0] for m in media], [m[1] for m in media],
                    tgt, [f], 0)
    got = _gpu_chain(gpu, xd, [q], [L], media, tgt, [f], 0, prec, (0.0, 0.0, 1.0))
    assert rel(got, ref) <= TOL[prec]


def test_piston_axis_workload(gpu, orc):
    """The 1 MHz piston workload in full: GPU sampling + pair sum vs the reference's own
    samples + sum, and vs the closed-form axis pressure."""
    cfg = W.PistonAxis()
    k = 2 * math.pi * cfg.freq / cfg.medium[0]
    tgt = cfg.targets()
    o = orc.sample_disc(cfg.seed, cfg.n_src, cfg.radius)
    ref = orc.propagate(0, o[:3], o[3], 1.0, tgt, cfg.medium[0], cfg.freq)
    g = gpu.rsi_sample_disc(cfg.seed, cfg.n_src, cfg.radius)
    import torch
    vel = torch.ones(cfg.n_src, dtype=torch.complex128, device="cuda")
    pex = cfg.medium[1] * cfg.medium[0] * (np.exp(1j * k * tgt[2]) - np.exp(1j * k * np.sqrt(tgt[2] ** 2 + cfg.radius ** 2)))
    for prec in (0, 1):
        phi = gpu.rsi_propagate(g[:3], g[3], vel, devpts(tgt), cfg.medium[0], cfg.freq, 0, prec)
        assert rel(host(phi), ref) <= TOL[prec]
        p = host(gpu.rsi_to_pressure(phi, cfg.medium[1], cfg.freq))
        assert rel(p, pex) < 5e-4


# ----------------------------------------------------------------------------- a7
MF_CASES = [  # (kind, planar, normal z, frequencies, strengths given)
    (0, False, 1.0, "grid20", True), (0, False, 1.0, "grid20", False), (1, True, 1.0, "grid20", True),
    (1, True, -1.0, "grid20", True), (1, True, -1.0, "grid3", False), (2, False, 1.0, "grid20", True),
    (1, False, 1.0, "grid20", True), (1, True, 1.0, "list", True), (0, False, 1.0, "one", True),
    (1, True, 1.0, "grid40", True), (1, True, 1.0, "grid50", True), (0, False, 1.0, "grid50", False),
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind,planar,nz,fr,given", MF_CASES)
def test_propagate_multifreq_matches_reference(gpu, orc, kind, planar, nz, fr, given, prec):
    """rsi_propagate_multifreq (multi-frequency superposition, Sec. 4): every frequency
    against the reference's single-frequency pair sum with that frequency's strengths.
    FP32 uniform grids with a monopole, omnidirectional or planar +-z dipole kernel run
    the multi-frequency launch: 3 and 40 frequencies in blocks of 16 (40: two full blocks
    and a ragged one of 8), 20 and 50 in blocks of 32 (one ragged block of 20; a full block
    and a ragged one of 18, which crosses the restart of the recurrence at its 17th
    frequency); a general dipole, a non-uniform list and FP64 run one pair sum per
    frequency."""
    freqs = {"grid20": list(np.linspace(1.0e6, 10.0e6, 20)), "grid3": [2.0e6, 2.5e6, 3.0e6],
             "grid40": list(np.linspace(1.0e6, 10.0e6, 40)), "grid50": list(np.linspace(1.0e6, 10.0e6, 50)),
             "list": [1.0e6, 1.7e6, 4.2e6], "one": [3.3e6]}[fr]
    ns, nt = 3001, 700
    src, w, _, tgt = _case(51 + kind, ns, nt, 1 if planar else 0)
    if planar:
        src = (src[0], src[1], np.full(ns, 0.004))
    rng = np.random.default_rng(5)
    vel = rng.normal(size=(len(freqs), ns)) + 1j * rng.normal(size=(len(freqs), ns)) if given else None
    normal = (0.0, 0.0, nz)
    c = 5900.0
    got = host(gpu.rsi_propagate_multifreq(devpts(src), dev(w), dev(vel) if given else None, devpts(tgt), c,
                                           freqs, kind, prec, gpu.RSI_FLAG_PLANAR_Z if planar else 0,
                                           normal=normal))
    assert got.shape == (len(freqs), nt)
    for q, f in enumerate(freqs):
        s = vel[q] if given else np.ones(ns, dtype=complex)
        ref = orc.propagate(kind, src, w, s, tgt, c, f, normal=normal)
        assert rel(got[q], ref) <= TOL[prec], (q, rel(got[q], ref))


def test_propagate_multifreq_empty_and_errors(gpu):
    import torch
    from paper_2408_06765_amd._lib import RSIError
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    tgt = devpts(W.random_cloud(1, 300, (0, 0, 0.02), (0.01, 0.01, 0.01)))
    out = gpu.rsi_propagate_multifreq((e, e, e), e, None, tgt, 1480.0, [1e6, 2e6, 3e6], 0, 0)
    assert out.shape == (3, 300) and np.all(host(out) == 0)
    src, w, s, _ = _case(3, 10, 1, 0)
    with pytest.raises(RSIError):
        gpu.rsi_propagate_multifreq(devpts(src), dev(w), None, tgt, 1480.0, [1e6, -2e6], 0, 0)


def _instances(gpu, n_inst, prec, seed=0):
    rng = np.random.default_rng(seed)
    insts, refs = [], []
    for i in range(n_inst):
        ns = int(rng.integers(1, 9000)) if i % 5 else 0
        nt = int(rng.integers(1, 3000))
        kind = i % 3  # monopole, dipole, omnidirectional
        src, w, s, tgt = _case(100 + i, max(ns, 1), nt, kind)
        src = tuple(v[:ns] for v in src)
        w, s = w[:ns], s[:ns]
        c = 5900.0 if kind == 1 else 1480.0
        f = 1e6 * (1 + i % 7)
        insts.append(gpu.Instance(devpts(src), dev(w), devpts(tgt), c, f, kind, vel=dev(s),
                                  normal=(0.0, 0.0, 1.0)))
        refs.append((kind, src, w, s, tgt, c, f))
    return insts, refs


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_matches_reference(gpu, orc, prec):
    insts, refs = _instances(gpu, 23, prec)
    gpu.rsi_propagate_batched(insts, prec)
    for it, (kind, src, w, s, tgt, c, f) in zip(insts, refs):
        ref = orc.propagate(kind, src, w, s, tgt, c, f, normal=(0, 0, 1))
        got = host(it.out)
        if len(src[0]) == 0:
            assert np.all(got == 0)
        else:
            assert rel(got, ref) <= TOL[prec]


def test_batched_plan_replay_bitwise(gpu):
    import torch
    insts, _ = _instances(gpu, 17, 0, seed=3)
    gpu.rsi_propagate_batched(insts, 0)
    eager = [host(i.out).copy() for i in insts]
    plan = gpu.Plan.batched(insts, 0)
    for rep in range(3):
        for i in insts:
            i.out.zero_()
        plan.execute()
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
        for i, e in zip(insts, eager):
            assert np.array_equal(host(i.out).view(np.uint64), e.view(np.uint64))
    plan.destroy()


def test_autotune_cache_and_corrupt_cache(gpu, orc, tmp_path, monkeypatch):
    """The autotuner writes its choice to the cache file; a later call reads it (results
    still match the reference); garbage appended to the file is skipped line by line (the
    last valid entry still wins: same bits); a file of random bytes leaves the default
    shape (results still match the reference)."""
    import os
    cache = tmp_path / "autotune.txt"
    monkeypatch.setenv("RSI_AUTOTUNE_CACHE", str(cache))
    insts, refs = _instances(gpu, 9, 0, seed=5)

    def run_and_check():
        for i in insts:
            i.out.zero_()
        gpu.rsi_propagate_batched(insts, 0)
        outs = [host(i.out).copy() for i in insts]
        for got, (kind, src, w, s, tgt, c, f) in zip(outs, refs):
            if len(src[0]) == 0:
                assert np.all(got == 0)
            else:
                assert rel(got, orc.propagate(kind, src, w, s, tgt, c, f, normal=(0, 0, 1))) <= TOL[0]
        return outs

    gpu.rsi_autotune_batched(insts, 0)
    lines = [ln.split() for ln in cache.read_text().splitlines() if ln.strip()]
    assert lines and all(len(ln) == 4 for ln in lines)
    key, tpl, chunk = lines[-1][0], int(lines[-1][1]), int(lines[-1][2])
    assert tpl in (1, 2, 4) and chunk in (4096, 16384, 65536)
    tuned = run_and_check()
    with open(cache, "ab") as fh:
        fh.write(b"\x00\xff not a line of the cache\n" + f"{key} 3 4096 1.0\n".encode()
                 + f"{key} 2 12\n".encode() + f"{key} 1 -5 2.0\n".encode() + b"truncated " + key.encode())
    again = run_and_check()
    for a, b in zip(again, tuned):
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    cache.write_bytes(os.urandom(4096))
    run_and_check()


@pytest.mark.parametrize("prec", [0, 1])
def test_chain_plan_replay(gpu, orc, prec):
    import torch
    cfg = W.LayeredStack()
    xd, ifs, tgt = _small_chain(orc, 1 << 11, cfg.z_if[:2], cfg.media[:3], cfg.tilt, 400)
    T = gpu.Transducer(*devpts(xd[:3]), dev(xd[3]), 1.0, (0.0, 0.0, 0.0), cfg.axis)
    I = [gpu.Interface(*devpts(q[:3]), dev(q[3]), z) for q, z in zip(ifs, cfg.z_if[:2])]
    tg = devpts(tgt)
    freqs = [2e6, 3e6]
    eager = host(gpu.rsi_chain(T, I, cfg.media[:3], tg, freqs, 1, prec))
    plan = gpu.Plan.chain(T, I, cfg.media[:3], tg, freqs, 1, prec)
    for rep in range(3):
        plan.out.zero_()
        plan.execute()
        torch.cuda.synchronize()
        _ = torch.randn(100, device="cuda").sum().item()
        assert np.array_equal(host(plan.out).view(np.uint64), eager.view(np.uint64))
    plan.destroy()


def test_calls_on_two_streams_match_one_stream(gpu, orc):
    """Calls are asynchronous on the caller's stream and independent across streams: a
    pair sum, a chain plan and a ray field enqueued on two side streams at once give the
    bits of the same calls run one after another on the default stream."""
    import torch
    cfg = W.LayeredStack()
    src, w, s, tgt = _case(21, 5000, 3001, 1)
    pargs = (devpts(src), dev(w), dev(s), devpts(tgt), 5900.0, 5.0e6, 1, 0)
    xd, ifs, ctgt = _small_chain(orc, 1 << 11, cfg.z_if[:2], cfg.media[:3], cfg.tilt, 400)
    T = gpu.Transducer(*devpts(xd[:3]), dev(xd[3]), 1.0, (0.0, 0.0, 0.0), cfg.axis)
    I = [gpu.Interface(*devpts(q[:3]), dev(q[3]), z) for q, z in zip(ifs, cfg.z_if[:2])]
    ctg = devpts(ctgt)
    rxd, zs, media, rtgt = _ray_case(orc, "one", 3000, 500)
    RT = gpu.Transducer(*devpts(rxd[:3]), dev(rxd[3]), 1.0, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    rtg = devpts(rtgt)
    ref_p = host(gpu.rsi_propagate(*pargs, normal=(0.0, 0.0, 1.0)))
    ref_c = host(gpu.rsi_chain(T, I, cfg.media[:3], ctg, [2e6, 3e6], 1, 0))
    ref_r = host(gpu.rsi_ray_field(RT, zs, media, rtg, [2.5e6], 0))
    plan = gpu.Plan.chain(T, I, cfg.media[:3], ctg, [2e6, 3e6], 1, 0)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for rep in range(3):
        with torch.cuda.stream(s1):
            p = gpu.rsi_propagate(*pargs, normal=(0.0, 0.0, 1.0))
        with torch.cuda.stream(s2):
            plan.execute()
            c = plan.out.clone()
        with torch.cuda.stream(s1):
            r = gpu.rsi_ray_field(RT, zs, media, rtg, [2.5e6], 0)
        outs.append((p, c, r))
    torch.cuda.synchronize()
    for p, c, r in outs:
        assert np.array_equal(host(p).view(np.uint64), ref_p.view(np.uint64))
        assert np.array_equal(host(c).view(np.uint64), ref_c.view(np.uint64))
        assert np.array_equal(host(r).view(np.uint64), ref_r.view(np.uint64))
    plan.destroy()


# ----------------------------------------------------------------------------- ray tracing (Sec. 2.2)
def _ray_case(orc, layout, n_xd, n_tgt, seed=0):
    tilt = math.radians(10.0)
    xd = orc.sample_disc(seed, n_xd, W.PISTON_RADIUS, (0.0, 0.0, 0.0), tilt)
    if layout == "water":
        zs, media = [], (W.WATER,)
        centre = (0.004, 0.0, 0.04)
    elif layout == "one":
        zs, media = [0.05], (W.WATER, W.STEEL_5900)
        centre = (0.05 * math.tan(tilt) + 0.012, 0.0, 0.05 + 0.015)
    else:
        cfg = W.LayeredStack()
        zs, media = list(cfg.z_if), cfg.media
        centre = (cfg.volume_centre_x(), 0.0, cfg.z_if[-1] + 0.012)
    tgt = W.random_cloud(seed + 5, n_tgt, centre, (0.012, 0.006, 0.01))
    return xd, zs, media, tgt


def _ray_gpu(gpu, xd, zs, media, tgt, freqs, prec):
    T = gpu.Transducer(*devpts(xd[:3]), dev(xd[3]), 1.0, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    return host(gpu.rsi_ray_field(T, zs, media, devpts(tgt), freqs, prec))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("layout", ["water", "one", "stack"])
@pytest.mark.parametrize("nf", [1, 11])
def test_ray_field_matches_reference(gpu, orc, prec, layout, nf):
    """eq. (12) through 0, 1 and 3 planes; one frequency, and eleven (a block of eight
    and a ragged block of three in one call).  1000 field points: three full tiles and a
    ragged one."""
    xd, zs, media, tgt = _ray_case(orc, layout, 2048, 1000)
    freqs = [2.5e6] if nf == 1 else list(np.linspace(1.0e6, 10.0e6, nf))
    ref = orc.ray_field(xd, 1.0, zs, [m[0] for m in media], [m[1] for m in media], tgt, freqs)
    got = _ray_gpu(gpu, xd, zs, media, tgt, freqs, prec)
    for q in range(nf):
        assert rel(got[q], ref[q]) <= TOL[prec], (q, rel(got[q], ref[q]))


@pytest.mark.parametrize("prec", [0, 1])
def test_ray_field_split_sources_and_masked_pairs(gpu, orc, prec):
    """Enough samples for several source splits (fixed-order reduction), field points
    above the last plane (no ray: exactly zero on both sides), and samples on both sides
    of the first plane (only those above it radiate)."""
    xd, zs, media, tgt = _ray_case(orc, "one", 9000, 300, seed=2)
    tgt = tuple(np.concatenate([a, b]) for a, b in zip(tgt, W.random_cloud(11, 40, (0.01, 0.0, 0.045),
                                                                              (0.01, 0.01, 0.004))))
    freqs = [3.0e6, 4.0e6]
    ref = orc.ray_field(xd, 1.0, zs, [m[0] for m in media], [m[1] for m in media], tgt, freqs)
    got = _ray_gpu(gpu, xd, zs, media, tgt, freqs, prec)
    assert rel(got, ref) <= TOL[prec]
    assert np.all(got[:, 300:] == 0) and np.all(ref[:, 300:] == 0)
    # a transducer straddling the first plane: the samples below it are masked
    xs = list(orc.sample_disc(4, 3000, W.PISTON_RADIUS, (0.0, 0.0, 0.05), math.radians(30.0)))
    tg = W.random_cloud(12, 300, (0.02, 0.0, 0.065), (0.01, 0.006, 0.008))
    ref = orc.ray_field(xs, 1.0, zs, [m[0] for m in media], [m[1] for m in media], tg, [2.0e6])
    got = _ray_gpu(gpu, xs, zs, media, tg, [2.0e6], prec)
    assert rel(got, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
def test_ray_field_empty_transducer_gives_zero(gpu, prec):
    import torch
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    T = gpu.Transducer(e, e, e, e, 1.0)
    tg = devpts(W.random_cloud(1, 100, (0, 0, 0.06), (0.01, 0.01, 0.005)))
    out = gpu.rsi_ray_field(T, [0.05], (W.WATER, W.STEEL_5900), tg, [1e6, 2e6], prec)
    assert host(out).shape == (2, 100) and np.all(host(out) == 0)


@pytest.mark.parametrize("launch", ["0", "1"])
@pytest.mark.parametrize("nf", [1, 3])
def test_ray_field_both_fp32_launches(gpu, orc, nf, launch, monkeypatch):
    """The two FP32 launches, forced (RSI_RAY_FEW): one field point per lane with the
    samples as wave-uniform records ("0", chosen for large workloads), and one wave per
    field point with the samples across its lanes ("1", chosen when the first would not
    fill the chip).  9000 points: 35 full tiles and a ragged one; 5000 samples: several
    source ranges and a ragged block."""
    monkeypatch.setenv("RSI_RAY_FEW", launch)
    xd, zs, media, tgt = _ray_case(orc, "one", 5000, 9000, seed=4)
    freqs = [2.5e6] if nf == 1 else [1.5e6, 2.5e6, 3.5e6]
    ref = orc.ray_field(xd, 1.0, zs, [m[0] for m in media], [m[1] for m in media], tgt, freqs)
    got = _ray_gpu(gpu, xd, zs, media, tgt, freqs, 0)
    for q in range(nf):
        assert rel(got[q], ref[q]) <= TOL[0], (q, rel(got[q], ref[q]))



def test_ray_field_large_counts(gpu, orc):
    """Ray model at the size limits of its launches, FP32: 2^22 field points from 64
    samples (16384 workgroups, one per 256 points) on sampled outputs, and 2^18 samples
    onto 5 field points (the one-wave-per-point launch, 1024 source splits)."""
    import torch
    rng = np.random.default_rng(5)
    media = (W.WATER, W.STEEL_5900)
    xd = orc.sample_disc(3, 64, W.PISTON_RADIUS, (0.0, 0.0, 0.0), math.radians(10.0))
    T = gpu.Transducer(*devpts(xd[:3]), dev(xd[3]), 1.0, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    nt = 1 << 22
    tgt = tuple(torch.as_tensor(rng.uniform(lo, hi, nt), device="cuda")
                for lo, hi in ((-0.01, 0.04), (-0.01, 0.01), (0.051, 0.08)))
    got = gpu.rsi_ray_field(T, [0.05], media, tgt, [2.5e6], 0)[0]
    pick = torch.as_tensor(np.sort(rng.choice(nt, 1500, replace=False)), device="cuda")
    sub = tuple(host(t[pick]) for t in tgt)
    ref = orc.ray_field(xd, 1.0, [0.05], [m[0] for m in media], [m[1] for m in media], sub, [2.5e6])[0]
    assert rel(host(got[pick]), ref) <= TOL[0]
    del got, tgt
    xd2 = orc.sample_disc(4, 1 << 18, W.PISTON_RADIUS, (0.0, 0.0, 0.0), math.radians(10.0))
    T2 = gpu.Transducer(*devpts(xd2[:3]), dev(xd2[3]), 1.0, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    tgt2 = W.random_cloud(6, 5, (0.015, 0.0, 0.065), (0.01, 0.005, 0.01))
    got2 = host(gpu.rsi_ray_field(T2, [0.05], media, devpts(tgt2), [2.5e6], 0))
    ref2 = orc.ray_field(xd2, 1.0, [0.05], [m[0] for m in media], [m[1] for m in media], tgt2, [2.5e6])
    assert rel(got2, ref2) <= TOL[0]

@pytest.mark.parametrize("prec", [0, 1])
def test_ray_field_extreme_geometry(gpu, orc, prec):
    """Edge cases of the root of eq. 14: field points 0.05-1 mm under the last plane far to
    the side (rays within a few degrees of grazing in the fast layer), points straight
    under samples (horizontal distance 0), a thin fast layer (aluminium, 0.5 mm) between
    water and steel, and a near-normal point; FP32 and FP64 against the reference."""
    rng = np.random.default_rng(21)
    xd = orc.sample_disc(6, 3000, W.PISTON_RADIUS, (0.0, 0.0, 0.0), math.radians(5.0))
    zs = [0.02, 0.0205]
    media = (W.WATER, W.ALU_PAPER, W.STEEL_PAPER)
    n = 400
    depth = np.concatenate([rng.uniform(5e-5, 1e-3, n // 2), rng.uniform(1e-3, 0.02, n // 2)])
    x = rng.uniform(-0.04, 0.04, n)
    y = rng.uniform(-0.01, 0.01, n)
    # straight under samples
    x[:10], y[:10] = xd[0][:10], xd[1][:10]
    tgt = (x, y, zs[-1] + depth)
    ref = orc.ray_field(xd, 1.0, zs, [m[0] for m in media], [m[1] for m in media], tgt, [3.0e6])
    got = _ray_gpu(gpu, xd, zs, media, tgt, [3.0e6], prec)
    assert np.all(np.isfinite(got))
    assert rel(got, ref) <= TOL[prec], rel(got, ref)


# ----------------------------------------------------------------------------- boundary
def test_nonfinite_inputs_rejected_when_checked(gpu):
    """With the finite check on, a NaN or an infinity in any device input of the pair-sum
    entry points gives RSI_ERR_NONFINITE before anything launches; finite inputs pass.
    (With the check off nothing is scanned: that path is every other test here.)"""
    import torch
    src, w, s, tgt = _case(5, 300, 70, 1)
    xd = W.random_cloud(8, 200, (0.0, 0.0, 0.0), (0.005, 0.005, 0.0))
    q = W.random_cloud(9, 300, (0.0, 0.0, 0.02), (0.02, 0.02, 0.0))
    wx, wq = W.random_weights(10, 200, 1e-6), W.random_weights(11, 300, 1e-6)
    media = [(1480.0, 1000.0), (5900.0, 7800.0)]
    prev = gpu.rsi_set_check_finite(True)

    def spoil(a, i, v):
        b = np.array(a, copy=True)
        b[i] = v
        return b

    def propagate(src_, w_, s_, tgt_):
        return gpu.rsi_propagate(devpts(src_), dev(w_), dev(s_), devpts(tgt_), 5900.0, 5.0e6, 1, 0,
                                 normal=(0.0, 0.0, 1.0))

    def chain(xd_, q_, tgt_):
        T = gpu.Transducer(*devpts(xd_[:3]), dev(wx), 1.0, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0))
        I = [gpu.Interface(*devpts(q_[:3]), dev(wq), 0.02)]
        return gpu.rsi_chain(T, I, media, devpts(tgt_), [2.0e6], 1, 0)

    def ray(wx_, tgt_):
        T = gpu.Transducer(*devpts(xd[:3]), dev(wx_), 1.0, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0))
        return gpu.rsi_ray_field(T, [0.02], media, devpts(tgt_), [2.0e6], 0)

    def batched(tgt_):
        out = torch.empty(len(tgt_[0]), dtype=torch.complex64, device="cuda")
        inst = gpu.Instance(devpts(src), dev(w), devpts(tgt_), 1480.0, 1.0e6, out=out)
        gpu.rsi_propagate_batched([inst], 0)

    tgt_below = (tgt[0], tgt[1], tgt[2] + 0.02)
    try:
        propagate(src, w, s, tgt)
        chain(xd, q, tgt_below)
        ray(wx, tgt_below)
        batched(tgt)
        bad_calls = [
            lambda: propagate(src, w, s, (tgt[0], tgt[1], spoil(tgt[2], 7, np.nan))),
            lambda: propagate((spoil(src[0], 0, np.inf), src[1], src[2]), w, s, tgt),
            lambda: propagate(src, spoil(w, 299, -np.inf), s, tgt),
            lambda: propagate(src, w, spoil(s, 3, complex(np.nan, 0.0)), tgt),
            lambda: chain(xd, (q[0], spoil(q[1], 5, np.nan), q[2]), tgt_below),
            lambda: ray(spoil(wx, 0, np.nan), tgt_below),
            lambda: batched((tgt[0], spoil(tgt[1], 69, np.inf), tgt[2])),
        ]
        for k, call in enumerate(bad_calls):
            with pytest.raises(gpu.RSIError, match="RSI_ERR_NONFINITE"):
                call()
    finally:
        gpu.rsi_set_check_finite(prev)

"""Full-size parity on the one-interface workload, in the launch configuration the
benchmark times (chain plan, FP32, local transmission coefficient), against reference
samples stored by tests/golden/make_golden.py (FP64 reference only)."""
import json
import os

import numpy as np
import pytest

from paper_2408_06765_amd import workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def golden(name):
    path = os.path.join(HERE, "golden", f"{name}_samples.json")
    if not os.path.exists(path):
        pytest.fail(f"missing {path}: run tests/golden/make_golden.py {name}")
    return json.load(open(path))


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _setup(gpu):
    import torch
    cfg = W.OneInterface()
    cx, cy = cfg.patch_centre
    xs = gpu.rsi_sample_disc(cfg.xd_seed, cfg.n_xd, cfg.radius, (0.0, 0.0, 0.0), cfg.tilt)
    qs = gpu.rsi_sample_square(cfg.if_seed, cfg.n_if, cx, cy, cfg.z_if, cfg.half_width)
    tgt = tuple(torch.as_tensor(a, device="cuda") for a in cfg.targets())
    T = gpu.Transducer(*xs[:3], xs[3], 1.0, (0.0, 0.0, 0.0), cfg.axis)
    I = [gpu.Interface(*qs[:3], qs[3], cfg.z_if)]
    return cfg, xs, qs, tgt, T, I


def test_one_interface_full_size_plan_fp32(gpu):
    import torch
    g = golden("one_interface")
    cfg, xs, qs, tgt, T, I = _setup(gpu)
    plan = gpu.Plan.chain(T, I, cfg.media, tgt, [cfg.freq], gpu.RSI_T_LOCAL, gpu.RSI_FP32)
    plan.execute()
    torch.cuda.synchronize()
    out = plan.out[0].cpu().numpy()
    ref = np.array(g["re"]) + 1j * np.array(g["im"])
    err = rel(out[np.array(g["index"])], ref)
    print(f"one_interface fp32 plan: rel-L2 {err:.3e} on {len(ref)} samples")
    assert err <= 1e-4
    assert np.all(np.isfinite(out))
    plan.destroy()


@pytest.mark.parametrize("prec", [0, 1])
def test_one_interface_piston_stage_full_size(gpu, prec):
    """The piston stage (2^16 sources) at sampled interface points."""
    import torch
    g = golden("one_interface")
    cfg, xs, qs, tgt, T, I = _setup(gpu)
    qi = torch.as_tensor(np.array(g["iface_index"]), device="cuda")
    pts = tuple(q[qi].contiguous() for q in qs[:3])
    vel = torch.ones(cfg.n_xd, dtype=torch.complex128, device="cuda")
    out = gpu.rsi_propagate(xs[:3], xs[3], vel, pts, cfg.media[0][0], cfg.freq, gpu.RSI_MONOPOLE, prec)
    ref = np.array(g["iface_re"]) + 1j * np.array(g["iface_im"])
    assert rel(out.cpu().numpy(), ref) <= (1e-4 if prec == 0 else 1e-10)


def test_one_interface_full_size_fp64(gpu):
    g = golden("one_interface")
    cfg, xs, qs, tgt, T, I = _setup(gpu)
    out = gpu.rsi_chain(T, I, cfg.media, tgt, [cfg.freq], gpu.RSI_T_LOCAL, gpu.RSI_FP64)[0].cpu().numpy()
    ref = np.array(g["re"]) + 1j * np.array(g["im"])
    err = rel(out[np.array(g["index"])], ref)
    print(f"one_interface fp64: rel-L2 {err:.3e}")
    assert err <= 1e-10


def test_layered_stack_full_size_plan_fp32(gpu):
    """Three interfaces x 2^18 samples, 128^3 volume, 64 frequencies in multi-frequency
    launches (chain plan), against the reference at 1 MHz and 10 MHz."""
    import torch
    g = golden("layered_stack")
    cfg = W.LayeredStack()
    xs = gpu.rsi_sample_disc(cfg.xd_seed, cfg.n_xd, cfg.radius, (0.0, 0.0, 0.0), cfg.tilt)
    ifs = []
    for seed, (cx, cy), z in zip(cfg.if_seeds, cfg.patch_centres, cfg.z_if):
        q = gpu.rsi_sample_square(seed, cfg.n_if, cx, cy, z, cfg.half_width)
        ifs.append(gpu.Interface(*q[:3], q[3], z))
    tgt = tuple(torch.as_tensor(a, device="cuda") for a in cfg.targets())
    T = gpu.Transducer(*xs[:3], xs[3], 1.0, (0.0, 0.0, 0.0), cfg.axis)
    plan = gpu.Plan.chain(T, ifs, cfg.media, tgt, list(cfg.freqs), gpu.RSI_T_LOCAL, gpu.RSI_FP32)
    plan.execute()
    torch.cuda.synchronize()
    idx = np.array(g["index"])
    ref = np.array(g["re"]) + 1j * np.array(g["im"])
    for fi, r in zip(g["freq_index"], ref):
        got = plan.out[fi].cpu().numpy()[idx]
        err = rel(got, r)
        print(f"layered_stack f={cfg.freqs[fi] / 1e6:.3f} MHz fp32 rel-L2 {err:.3e}")
        assert err <= 1e-4
    plan.destroy()


def test_scan_batch_full_size_plan(gpu, orc):
    """256 uneven instances in one persistent launch (batched plan), 16 sampled field
    points per instance against the reference (its own samples of each piston)."""
    import torch
    cfg = W.ScanBatch()
    insts, meta = [], []
    rng = np.random.default_rng(7)
    for it in cfg.instances():
        xs = gpu.rsi_sample_disc(it.seed, it.n_src, cfg.radius, (it.x_offset, 0.0, 0.0), it.tilt)
        pts = cfg.field_points(it)
        tgt = tuple(torch.as_tensor(a, device="cuda") for a in pts)
        insts.append(gpu.Instance(xs[:3], xs[3], tgt, cfg.medium[0], cfg.freq, gpu.RSI_MONOPOLE))
        meta.append((it, pts, np.sort(rng.choice(it.n_fld, min(16, it.n_fld), replace=False))))
    plan = gpu.Plan.batched(insts, gpu.RSI_FP32)
    plan.execute()
    torch.cuda.synchronize()
    worst = 0.0
    for inst, (it, pts, sel) in zip(insts, meta):
        o = orc.sample_disc(it.seed, it.n_src, cfg.radius, (it.x_offset, 0.0, 0.0), it.tilt)
        ref = orc.propagate(0, o[:3], o[3], 1.0, tuple(a[sel] for a in pts), cfg.medium[0], cfg.freq)
        got = inst.out.cpu().numpy()[sel]
        worst = max(worst, rel(got, ref))
    print(f"scan_batch worst instance rel-L2 {worst:.3e}")
    assert worst <= 1e-4
    plan.destroy()


def test_focused_normal_full_size_fp32(gpu):
    """Focused transducer (Sec. 3.3) at the benchmark's size: 10^5 Halton samples on the cap
    and on the interface, the 401 x 401 slice (chain plan, FP32, global T), against stored
    reference samples."""
    import torch
    g = golden("focused_normal")
    cfg = W.FocusedNormal()
    xs = gpu.rsi_sample_cap(cfg.xd_seed, cfg.n_xd, cfg.radius, cfg.curvature, (0.0, 0.0, 0.0), 0.0,
                            seq=gpu.RSI_SEQ_HALTON)
    q = gpu.rsi_sample_square(cfg.if_seed, cfg.n_if, 0.0, 0.0, cfg.water_path, cfg.half_width,
                              seq=gpu.RSI_SEQ_HALTON)
    T = gpu.Transducer(*xs[:3], xs[3], 1.0, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    I = [gpu.Interface(*q[:3], q[3], cfg.water_path)]
    tgt = tuple(torch.as_tensor(a, device="cuda") for a in cfg.grid())
    plan = gpu.Plan.chain(T, I, cfg.media, tgt, [cfg.freq], gpu.RSI_T_GLOBAL, gpu.RSI_FP32)
    plan.execute()
    torch.cuda.synchronize()
    out = plan.out[0].cpu().numpy()
    ref = np.array(g["re"]) + 1j * np.array(g["im"])
    err = rel(out[np.array(g["index"])], ref)
    print(f"focused_normal fp32 plan: rel-L2 {err:.3e} on {len(ref)} samples")
    assert err <= 1e-4
    plan.destroy()


@pytest.mark.parametrize("stack", [1, 2])
def test_ray_field_full_size_fp32(gpu, orc, stack):
    """The ray model at the benchmark's sizes: 10^5 Halton samples of the tilted piston
    through one plane onto the 401 x 401 slice (the ray_field configuration) and through
    four planes onto 10^5 field points (the largest crossover row but one); 48 sampled
    points against the reference computed here (one root per pair)."""
    import torch
    cfg = W.RayCrossover()
    media = cfg.stacks[stack]
    zs = cfg.planes(media)
    xs = gpu.rsi_sample_disc(cfg.xd_seed, cfg.n_samples, cfg.radius, (0.0, 0.0, 0.0), cfg.tilt,
                             seq=gpu.RSI_SEQ_HALTON)
    o = orc.sample_disc(cfg.xd_seed, cfg.n_samples, cfg.radius, (0.0, 0.0, 0.0), cfg.tilt, seq=orc.SEQ_HALTON)
    if stack == 1:
        xc = cfg.patch_centres(media)[0]
        X, Z = np.meshgrid(np.linspace(xc - 0.01, xc + 0.04, 401), zs[0] + np.linspace(0.001, 0.04, 401))
        pts = (X.ravel(), 0 * X.ravel(), Z.ravel())
    else:
        pts = cfg.field(media, 100000)
    T = gpu.Transducer(*xs[:3], xs[3], 1.0, (0.0, 0.0, 0.0), cfg.axis)
    tgt = tuple(torch.as_tensor(np.ascontiguousarray(a), device="cuda") for a in pts)
    out = gpu.rsi_ray_field(T, zs, media, tgt, [cfg.freq], gpu.RSI_FP32)[0].cpu().numpy()
    sel = np.sort(np.random.default_rng(9).choice(pts[0].size, 48, replace=False))
    ref = orc.ray_field(o, 1.0, zs, [m[0] for m in media], [m[1] for m in media],
                        tuple(a[sel] for a in pts), [cfg.freq])[0]
    err = rel(out[sel], ref)
    print(f"ray field ({len(zs)} planes) fp32 full size: rel-L2 {err:.3e} on 48 samples")
    assert err <= 1e-4
    assert np.all(np.isfinite(out))

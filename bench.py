"""Benchmark of the RSI-QMC hot path on one MI355X.

A step (the default workload, layered_stack) is one pass of the whole chained model over
the layered stack, every stage for 64 frequencies at once:
  piston (2^16 Sobol samples, tilted 10 deg) -> three planar interfaces at 50, 52, 54 mm
  (2^18 samples each, media c = 1480, 5900, 2700, 5900 m/s, local transmission
  coefficients) -> 128^3 volume 1-31 mm below the last interface, for 64 frequencies
  uniformly spanning 1-10 MHz, FP32 path (FP64 reference distance and phase).
  Pair-frequencies per step: 64 x (2^16 2^18 + 2 x 2^18 2^18 + 2^18 2^21) = 4.51e13.
  Inputs (sample points, weights, field points) are resident in HBM before the timed
  region; the step is one replay of the chain plan (hipGraph).

Printed: one JSON line with G pair-frequencies/s, the roofline of the dominant kernel (the
multi-frequency dipole pair sum of the last interface onto the volume, timed with HIP
events on its own stream) and the FP64 reference timed on the host cores over a bounded
sample of the same stages.  --workload one_interface gives the single-frequency chain
(piston -> one interface -> 512 x 512 image at 5 MHz) in the same format; the other
workloads are secondary measurements.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--no-cpu] [--workload NAME]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic FP32 flops per pair (FMA = 2, transcendental = 1), a convention fixed before
# measuring: monopole 25, dipole 33 (the per-step counts are listed with each kernel)
FLOPS_MONOPOLE = 25
FLOPS_DIPOLE = 33
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector (256 CU x 2.4 GHz x 256 flop/CU/clk)
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense bf16 MFMA
PEAK_HBM_GBPS = 8000.0  # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU reference timing")
    ap.add_argument("--kernel-reps", type=int, default=None,
                    help="launches for the roofline timing (default 2 for layered_stack, 5 otherwise)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (HBM counter calibration)")
    ap.add_argument("--workload", default="layered_stack",
                    choices=["layered_stack", "one_interface", "scan_batch", "surrogate",
                             "interface_continuity", "focused_normal", "ray_field",
                             "ray_crossover", "multilayer_noise", "surrogate_inference",
                             "surrogate_training"],
                    help="layered_stack is the benchmark line; the others are secondary "
                         "measurements printed in the same format")
    ap.add_argument("--autotune", action="store_true",
                    help="scan_batch: run the autotuner (writes the cache) before planning")
    ap.add_argument("--sur-train-f-max", type=float, default=None,
                    help="surrogate: highest training frequency (Hz; default the recipe's)")
    ap.add_argument("--sur-train-tilt-max", type=float, default=None,
                    help="surrogate: largest training tilt (degrees; default the recipe's)")
    ap.add_argument("--sur-carrier-samples", type=int, default=None,
                    help="surrogate: transducer samples of the ray-model carrier (default the recipe's)")
    ap.add_argument("--sur-judge-scale", type=int, default=None,
                    help="surrogate: interface sample-count multiplier of the judging / fallback RSI (default the recipe's)")
    ap.add_argument("--sur-train-if-scale", type=int, default=None,
                    help="surrogate: interface sample-count multiplier of the training fields (default the recipe's)")
    ap.add_argument("--sur-depth", type=int, default=None,
                    help="surrogate, surrogate_inference, surrogate_training: hidden layers (default the recipe's)")
    ap.add_argument("--sur-epochs", type=int, default=None,
                    help="surrogate: training epochs (default the recipe's)")
    ap.add_argument("--fp64-compare", action="store_true",
                    help="layered_stack: FP32 vs FP64 rel-L2 per frequency on a volume subsample")
    return ap.parse_args()


def cpu_model():
    """The host CPU's model name (first 'model name' line of /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline_layered(cfg, target_seconds=15.0):
    """The FP64 reference, as it stands, on a bounded sample of the layered stack: the
    three stage kinds at one frequency of the grid (the middle one), each onto m field
    points -- the piston (2^16 samples) onto interface 1, interface 1 (2^18 samples) onto
    interface 2, interface 3 (2^18 samples) onto the volume -- with unit strengths.  The
    reference has no multi-frequency path, so its pair-frequencies per second are its
    pairs per second."""
    import oracle

    xd = oracle.sample_disc(cfg.xd_seed, cfg.n_xd, cfg.radius, (0.0, 0.0, 0.0), cfg.tilt)
    qs = [oracle.sample_square(seed, cfg.n_if, cx, cy, z, cfg.half_width)
          for seed, (cx, cy), z in zip(cfg.if_seeds, cfg.patch_centres, cfg.z_if)]
    tx, ty, tz = cfg.targets()
    rng = np.random.default_rng(0)
    pick = rng.choice(tx.size, size=tx.size, replace=False)
    f = float(cfg.freqs[cfg.n_freq // 2])
    c = [m[0] for m in cfg.media]

    def run(m):
        t0 = time.perf_counter()
        oracle.propagate(0, xd[:3], xd[3], 1.0, tuple(a[:m] for a in qs[0][:3]), c[0], f)
        oracle.propagate(1, qs[0][:3], qs[0][3], 1.0, tuple(a[:m] for a in qs[1][:3]), c[1], f,
                         normal=(0.0, 0.0, 1.0))
        oracle.propagate(1, qs[2][:3], qs[2][3], 1.0, (tx[pick[:m]], ty[pick[:m]], tz[pick[:m]]), c[3], f,
                         normal=(0.0, 0.0, 1.0))
        return time.perf_counter() - t0, m * (cfg.n_xd + 2 * cfg.n_if)
    dt, pairs = run(64)
    m = int(max(64, min(cfg.n_if, target_seconds * pairs / max(dt, 1e-9) / (cfg.n_xd + 2 * cfg.n_if))))
    dt, pairs = run(m)
    return {"value": pairs / dt / 1e9, "unit": "Gpairs/s", "cores": oracle.num_threads(),
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": f"one frequency ({f / 1e6:.4f} MHz): piston stage onto {m} interface-1 points, "
                      f"interface 1 -> {m} interface-2 points, interface 3 -> {m} volume points (2^16 / 2^18 "
                      f"sources): {pairs:.3e} pairs in {dt:.2f} s"}


def cpu_baseline(cfg, target_seconds=12.0):
    """The FP64 reference, as it stands, on a bounded sample of the same workload:
    the piston stage onto a subset of interface points and the interface stage (all
    2^18 sources, unit strengths) onto a subset of image points."""
    import oracle

    xd = oracle.sample_disc(cfg.xd_seed, cfg.n_xd, cfg.radius, (0.0, 0.0, 0.0), cfg.tilt)
    cx, cy = cfg.patch_centre
    q = oracle.sample_square(cfg.if_seed, cfg.n_if, cx, cy, cfg.z_if, cfg.half_width)
    tx, ty, tz = cfg.targets()
    (c0, _), (c1, _) = cfg.media
    # calibrate on a small sample, then size the sample for ~target_seconds
    def run(m_if, m_img):
        t0 = time.perf_counter()
        oracle.propagate(0, xd[:3], xd[3], 1.0, tuple(a[:m_if] for a in q[:3]), c0, cfg.freq)
        oracle.propagate(1, q[:3], q[3], 1.0, (tx[:m_img], ty[:m_img], tz[:m_img]), c1, cfg.freq,
                         normal=(0.0, 0.0, 1.0))
        return time.perf_counter() - t0, cfg.n_xd * m_if + cfg.n_if * m_img
    dt, pairs = run(64, 64)
    rate = pairs / max(dt, 1e-9)
    # keep the workload's mix: interface points and image points in proportion 1 : 1
    m = int(max(64, min(cfg.n_if, target_seconds * rate / (cfg.n_xd + cfg.n_if))))
    dt, pairs = run(m, m)
    return {"value": pairs / dt / 1e9, "unit": "Gpairs/s", "cores": oracle.num_threads(),
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": f"piston stage onto {m} interface points + interface stage (2^18 sources) onto "
                      f"{m} image points: {pairs:.3e} pairs in {dt:.2f} s"}


# What a kernel's counters depend on, per committed summary: the device header and
# record layout, the kernel's definition, its shape rule and its launcher.  Host code
# elsewhere in those files does not invalidate the counters.
KERNEL_SOURCES = {
    "pairsum": [
        ("paper_2408_06765_amd/csrc/rsi_device.h", None),
        ("paper_2408_06765_amd/csrc/rsi_pairsum.hip",
         ["pairsum_f32_kernel(", "PairShape default_shape(", "rsi_status pairsum_f32("]),
        ("paper_2408_06765_amd/csrc/rsi_internal.h",
         ["struct alignas(32) SrcRecF", "constexpr int kBlock", "constexpr int64_t kFewWaves"]),
    ],
    "multifreq": [
        ("paper_2408_06765_amd/csrc/rsi_device.h",
         ["constexpr int kSub", "bool phase_in_sin_range("]),
        ("paper_2408_06765_amd/csrc/rsi_multifreq.hip",
         ["struct TargetMF", "struct BlockMF", "void multifreq_sum(", "multifreq_f32_kernel(",
          "int mf_block(", "rsi_status pairsum_multifreq_f32("]),
        ("paper_2408_06765_amd/csrc/rsi_internal.h",
         ["struct alignas(32) SrcRecF", "constexpr int kBlock"]),
    ],
}


def _region(text, anchor):
    """The source from the line holding `anchor` to the end of its braced block (or of the
    statement, when a ';' comes before any '{')."""
    i = text.rfind("\n", 0, text.index(anchor)) + 1
    brace, semi = text.find("{", i), text.find(";", i)
    if semi != -1 and (brace == -1 or semi < brace):
        return text[i:semi + 1]
    depth = 0
    for k in range(brace, len(text)):
        depth += {"{": 1, "}": -1}.get(text[k], 0)
        if depth == 0:
            return text[i:k + 1]
    raise ValueError(anchor)


def kernel_sources_digest(kernel="pairsum"):
    import hashlib
    h = hashlib.sha256()
    for f, anchors in KERNEL_SOURCES[kernel]:
        text = open(os.path.join(ROOT, f)).read()
        for part in ([text] if anchors is None else [_region(text, a) for a in anchors]):
            h.update(part.encode())
    return h.hexdigest()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pairsum_dipole_one_interface_traffic.txt")
VALU_FILE = os.path.join(ROOT, "profiles", "pairsum_valu_counters.md")
MF_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "multifreq_dipole_layered_stack_traffic.txt")
MF_VALU_FILE = os.path.join(ROOT, "profiles", "multifreq_valu_counters.md")


def _counter_summary(path, kernel="pairsum"):
    """The key: value lines of a committed counter summary, or None when the file is missing
    or the kernel sources changed since its counters were taken."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if line.startswith("#") or ":" not in line:
            continue
        k, v = line.split(":", 1)
        kv[k.strip()] = v.strip()
    try:
        digest = kernel_sources_digest(kernel)
    except (OSError, ValueError):  # a source or an anchor moved: the counters are stale
        return None
    if kv.get("kernel_sources_sha256") != digest:
        return None
    return kv


def measured_traffic(path=None, kernel="pairsum"):
    """HBM bytes per launch of a kernel from its committed counter summary (default: the
    single-frequency dipole pair sum's), or None when the summary is missing or the kernel
    sources changed since the counters were taken."""
    kv = _counter_summary(path or TRAFFIC_FILE, kernel)
    return None if kv is None else int(float(kv["traffic_bytes_per_launch"]))


def measured_valu(path=None, kernel="pairsum"):
    """Executed FP32 FLOPs and VALU occupancy of a kernel from its committed VALU counter
    summary (the metric's "% FP32 VALU peak" as counted by the hardware), or None when the
    summary is missing or the kernel sources changed since the counters were taken."""
    path = path or VALU_FILE
    kv = _counter_summary(path, kernel)
    if kv is None:
        return None
    return {"executed_tflops": float(kv["dipole_executed_fp32_tflops"]),
            "executed_frac": float(kv["dipole_executed_fp32_frac"]),
            "valu_lane_util_pct": float(kv["dipole_valu_lane_util_pct"]),
            "cu_busy_pct": float(kv["dipole_cu_busy_pct"]),
            "issue_model_frac": float(kv["dipole_issue_model_frac"]),
            "source": os.path.relpath(path, ROOT)}


def calib_copy():
    """A plain device copy of known size (256 MiB read + 256 MiB written) in the same run,
    whose HBM counters scale the kernel's."""
    import torch
    a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    return a.numel() * 4


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def base_line(metric_value, steps, warmup, dt, config, unit="Gpairs/s"):
    return {
        "metric": "Gpairs/s RSI-QMC (chained pair sum) + % FP32 VALU peak",
        "value": round(metric_value, 3), "unit": unit, "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": round(1e3 * dt / max(steps, 1), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "config": config,
    }


def flops_multifreq_pair(n_freq, block=16):
    """Algorithmic FP32 flops of one dipole pair for n_freq frequencies on a uniform grid,
    evaluated in blocks of `block` (FMA = 2, transcendental = 1): 33 for each block's first
    frequency (the single-frequency dipole pair) and 21 for each further one (carrying
    e^{ikr} to the next frequency, the (ik - 1/r) factor, the complex multiply-accumulate
    with that frequency's strength).  The convention was fixed with blocks of 16 and stays
    there whatever block the kernel runs (32 on 64 frequencies: 1368 per pair instead of
    1392)."""
    nb = (n_freq + block - 1) // block
    return FLOPS_DIPOLE * nb + 21 * (n_freq - nb)


def layered_stack(args):
    """Three interfaces, 64 frequencies (one multi-frequency launch per stage), 128^3: the
    benchmark line."""
    import torch
    from paper_2408_06765_amd import rsi
    from paper_2408_06765_amd import workloads as W

    cfg = W.LayeredStack()
    xs = rsi.rsi_sample_disc(cfg.xd_seed, cfg.n_xd, cfg.radius, (0.0, 0.0, 0.0), cfg.tilt)
    ifs = []
    for seed, (cx, cy), z in zip(cfg.if_seeds, cfg.patch_centres, cfg.z_if):
        q = rsi.rsi_sample_square(seed, cfg.n_if, cx, cy, z, cfg.half_width)
        ifs.append(rsi.Interface(*q[:3], q[3], z))
    tgt = tuple(torch.as_tensor(a, device="cuda") for a in cfg.targets())
    T = rsi.Transducer(*xs[:3], xs[3], 1.0, (0.0, 0.0, 0.0), cfg.axis)
    freqs = [float(f) for f in cfg.freqs]
    plan = rsi.Plan.chain(T, ifs, cfg.media, tgt, freqs, rsi.RSI_T_LOCAL, rsi.RSI_FP32)
    torch.cuda.synchronize()
    print(f"layered_stack: plan built, {args.warmup} warmup + {args.steps} timed steps", file=sys.stderr,
          flush=True)
    dt = timed(plan.execute, args.steps, args.warmup)
    n_t = tgt[0].numel()
    nf = len(freqs)
    pairs = nf * (cfg.n_xd * cfg.n_if + 2 * cfg.n_if * cfg.n_if + cfg.n_if * n_t)
    line = base_line(pairs * args.steps / dt / 1e9, args.steps, args.warmup, dt,
                     {"workload": "layered_stack: piston 2^16 (10 deg, 6.35 mm) -> 3 interfaces x 2^18 "
                                  "(c = 1480/5900/2700/5900 m/s, 2 mm apart, local T) -> 128^3 volume, "
                                  "64 frequencies 1-10 MHz", "pair_frequencies_per_step": pairs,
                      "precision": "fp32 (fp64 reference distance + phase)"})
    print(f"layered_stack: {1e3 * dt / max(args.steps, 1):.1f} ms per step", file=sys.stderr, flush=True)

    # dominant kernel: the multi-frequency dipole pair sum of interface 3 onto the volume,
    # the same launch as the chain's last stage, through rsi_propagate_multifreq with HIP
    # events on the stream it runs on (per-frequency strengths seeded, 2^18 x 64)
    rng = np.random.default_rng(0)
    last = ifs[-1]
    vel = torch.as_tensor(rng.normal(size=(nf, cfg.n_if)) + 1j * rng.normal(size=(nf, cfg.n_if)), device="cuda")
    mf_out = torch.empty((nf, n_t), dtype=torch.complex64, device="cuda")
    reps = args.kernel_reps if args.kernel_reps is not None else 2
    s = torch.cuda.Stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    with torch.cuda.stream(s):
        for e0, e1 in ev:
            e0.record(s)
            rsi.rsi_propagate_multifreq((last.x, last.y, last.z), last.w, vel, tgt, cfg.media[-1][0], freqs,
                                        rsi.RSI_DIPOLE, rsi.RSI_FP32, rsi.RSI_FLAG_PLANAR_Z,
                                        normal=(0.0, 0.0, 1.0), out=mf_out)
            e1.record(s)
    s.synchronize()
    kms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev]))
    fl = flops_multifreq_pair(nf)
    kpairs = cfg.n_if * n_t
    achieved = fl * kpairs / (kms * 1e-3) / 1e12
    line["roofline"] = {"bound": "alu", "achieved": round(achieved, 2), "peak": PEAK_FP32_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                        "traffic": measured_traffic(MF_TRAFFIC_FILE, "multifreq"),
                        "kernel": f"multifreq_f32_kernel<dipole, planar, per-frequency strengths, blocks of 32 "
                                  f"frequencies> (interface 3 -> volume: one call, launched per chunk of 8192 "
                                  f"sources), {fl} flop per pair for {nf} frequencies (convention of blocks of 16; "
                                  f"{flops_multifreq_pair(nf, 32)} counted in blocks of 32) x {kpairs:.4e} pairs "
                                  f"/ {kms:.3f} ms"}
    line["fp32_valu_counters"] = measured_valu(MF_VALU_FILE, "multifreq")
    del vel, mf_out
    if args.fp64_compare:
        # FP64 chain per frequency on every 64th volume point; FP32 from the timed plan
        sub = torch.arange(0, n_t, 64, device="cuda")
        tsub = tuple(a[sub].contiguous() for a in tgt)
        f32 = plan.out[:, sub].cpu().numpy()
        errs = []
        for qi, f in enumerate(freqs):
            ref = rsi.rsi_chain(T, ifs, cfg.media, tsub, [f], rsi.RSI_T_LOCAL, rsi.RSI_FP64)[0].cpu().numpy()
            errs.append(float(np.linalg.norm(f32[qi] - ref) / np.linalg.norm(ref)))
            print(f"freq {f/1e6:.4f} MHz  fp32 vs fp64 rel-L2 {errs[-1]:.3e}", file=sys.stderr, flush=True)
        line["fp32_vs_fp64_rel_l2_per_frequency"] = errs
    gold = os.path.join(ROOT, "tests", "golden", "layered_stack_samples.json")
    if os.path.exists(gold):
        g = json.load(open(gold))
        idx = np.array(g["index"])
        ref = np.array(g["re"]) + 1j * np.array(g["im"])
        got = plan.out[g["freq_index"]].cpu().numpy()[:, idx]
        line["parity_vs_oracle_samples"] = [float(np.linalg.norm(a - b) / np.linalg.norm(b))
                                            for a, b in zip(got, ref)]
    plan.destroy()
    if args.calib_copy:
        line["calib_copy_bytes"] = calib_copy()
    if not args.no_cpu:
        print("layered_stack: timing the FP64 reference on the host", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline_layered(cfg)
    print(json.dumps(line), flush=True)


def interface_continuity(args):
    """Pressure on both sides of the interface along the beam axis (eq. 6 continuity),
    for the dipole interface sources of eq. 7 and for the omnidirectional sources of the
    ablation; |p| normalised by rho1 c1 v0."""
    import torch
    from paper_2408_06765_amd import rsi
    from paper_2408_06765_amd import workloads as W

    cfg = W.InterfaceContinuity()
    (c1, r1), (c2, r2) = cfg.media
    xs = rsi.rsi_sample_disc(cfg.xd_seed, cfg.n_xd, cfg.radius, (0.0, 0.0, 0.0), cfg.tilt)
    q = rsi.rsi_sample_square(cfg.if_seed, cfg.n_if, cfg.patch_centre[0], cfg.patch_centre[1], cfg.z_if,
                              cfg.half_width)
    T = rsi.Transducer(*xs[:3], xs[3], 1.0, (0.0, 0.0, 0.0), cfg.axis)
    I = [rsi.Interface(*q[:3], q[3], cfg.z_if)]
    above = tuple(torch.as_tensor(a, device="cuda") for a in cfg.points("above"))
    below = tuple(torch.as_tensor(a, device="cuda") for a in cfg.points("below"))
    om = 2 * math.pi * cfg.freq
    res, timing = {}, {}
    for name, fl in (("dipole", 0), ("omni", rsi.RSI_CHAIN_OMNI)):
        for prec in (rsi.RSI_FP32, rsi.RSI_FP64):
            def run():
                a = rsi.rsi_chain(T, I, cfg.media, above, [cfg.freq], rsi.RSI_T_LOCAL, prec,
                                  flags=fl | rsi.RSI_CHAIN_ABOVE)[0]
                b = rsi.rsi_chain(T, I, cfg.media, below, [cfg.freq], rsi.RSI_T_LOCAL, prec, flags=fl)[0]
                return a, b
            run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            a, b = run()
            torch.cuda.synchronize()
            timing[(name, prec)] = time.perf_counter() - t0
            p1 = (om * r1 * a.abs() / (r1 * c1)).cpu().numpy()  # |p| / (rho1 c1 v0)
            p2 = (om * r2 * b.abs() / (r1 * c1)).cpu().numpy()
            res[(name, prec)] = (p1, p2, a.cpu().numpy(), b.cpu().numpy())
    # pairs per chain evaluation: piston -> interface, interface -> points, plus the
    # incident field at the points above
    n_d = cfg.n_d
    pairs = 2 * cfg.n_xd * cfg.n_if + cfg.n_if * 2 * n_d + cfg.n_xd * n_d
    # Above the plane incident and reflected waves interfere (a standing wave of period
    # about lambda/2), so the upper face is taken at the plane itself: the boundary
    # value (1 + R) phi_i(Q0) of the model at the axis intercept Q0.  Below, |p| varies
    # slowly and is extrapolated to the plane from the three nearest points.
    q0 = tuple(torch.tensor([v], dtype=torch.float64, device="cuda")
               for v in (cfg.patch_centre[0], cfg.patch_centre[1], cfg.z_if))
    phi_i = rsi.rsi_propagate(xs[:3], xs[3], torch.ones(cfg.n_xd, dtype=torch.complex128, device="cuda"),
                              q0, c1, cfg.freq, rsi.RSI_MONOPOLE, rsi.RSI_FP64)[0].item()
    R0 = rsi.rsi_reflection(rsi.RSI_T_LOCAL, 1, [cfg.z_if], cfg.media, (0.0, 0.0, 0.0), cfg.axis,
                            q0[0], q0[1])[0].item()
    p_face_above = om * r1 * abs((1 + R0) * phi_i) / (r1 * c1)
    d3 = cfg.distances[:3]

    def at_plane(y):
        return float(np.polyval(np.polyfit(d3, y[:3], 1), 0.0))
    p_face_dip, p_face_omni = at_plane(res[("dipole", 0)][1]), at_plane(res[("omni", 0)][1])
    jd, jo = p_face_dip / p_face_above, p_face_omni / p_face_above
    f32_vs_f64 = max(float(np.linalg.norm(res[(m, 0)][k] - res[(m, 1)][k]) / np.linalg.norm(res[(m, 1)][k]))
                     for m in ("dipole", "omni") for k in (2, 3))
    s2 = c2 / c1 * math.sin(cfg.tilt)
    line = {
        "metric": "pressure ratio |p2/p1| across the interface on the beam axis (eq. 6)",
        "value": round(float(jd), 4), "unit": "ratio", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(1e3 * timing[("dipole", 0)], 3), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "interface_continuity: tilted piston (10 deg) 2^16 -> water/5900 m/s "
                               "interface 2^22 samples, 2.5 MHz, local T; 10 points 0.1-1 mm each side"},
        "omni_ratio": round(float(jo), 4),
        "p_face_above_boundary_value": round(float(p_face_above), 5),
        "p_face_below_dipole_extrapolated": round(p_face_dip, 5),
        "p_face_below_omni_extrapolated": round(p_face_omni, 5),
        "omni_ratio_expected_plane_wave": round(1.0 / math.sqrt(1 - s2 * s2), 4),
        "distance_mm": [round(1e3 * d, 4) for d in cfg.distances],
        "p_above_dipole": [round(float(v), 5) for v in res[("dipole", 0)][0]],
        "p_below_dipole": [round(float(v), 5) for v in res[("dipole", 0)][1]],
        "p_above_omni": [round(float(v), 5) for v in res[("omni", 0)][0]],
        "p_below_omni": [round(float(v), 5) for v in res[("omni", 0)][1]],
        "fp32_vs_fp64_rel_l2": f32_vs_f64,
        "gpairs_per_s_fp32": round(pairs / timing[("dipole", 0)] / 1e9, 1),
        "gpairs_per_s_fp64": round(pairs / timing[("dipole", 1)] / 1e9, 1),
    }
    print(json.dumps(line), flush=True)


def focused_normal(args):
    """Focused transducer at normal incidence (Sec. 3.3): cap R = 33 mm, 10 mm water path,
    steel, 2.5 MHz, 10^5 Halton samples per surface.  Timed: the chain onto the 401 x 401
    y-z slice (FP32, one plan replay per step).  Reported beside it: the on-axis velocity
    amplitude k2 |phi| / v0 in the steel, its peak depth against the paper's 14 mm, the
    -6 dB width of the focal spot, the focal gain over a flat piston, the apodised
    variant, and the on-axis error of 10^5 Halton and 10^5 Sobol samples against a
    2^20-sample Sobol field (FP32 vs FP64 stated)."""
    import torch
    from paper_2408_06765_amd import rsi
    from paper_2408_06765_amd import workloads as W

    cfg = W.FocusedNormal()
    (c1, r1), (c2, r2) = cfg.media
    zero, axis = (0.0, 0.0, 0.0), (0.0, 0.0, 1.0)
    freqs = [cfg.freq]

    def model(seq, n_xd, n_if, apod=False, flat=False):
        if flat:
            xs = rsi.rsi_sample_disc(cfg.xd_seed, n_xd, cfg.radius, zero, 0.0, seq=seq)
        else:
            xs = rsi.rsi_sample_cap(cfg.xd_seed, n_xd, cfg.radius, cfg.curvature, zero, 0.0, seq=seq)
        w = xs[3]
        if apod:
            rsi.rsi_apodise(xs[:3], w, zero, axis, cfg.apod_width)
        q = rsi.rsi_sample_square(cfg.if_seed, n_if, 0.0, 0.0, cfg.water_path, cfg.half_width, seq=seq)
        return rsi.Transducer(*xs[:3], w, 1.0, zero, axis), [rsi.Interface(*q[:3], q[3], cfg.water_path)]

    dev = lambda pts: tuple(torch.as_tensor(a, device="cuda") for a in pts)
    grid, line, focal = dev(cfg.grid()), dev(cfg.axis_line()), dev(cfg.focal_line())
    H = rsi.RSI_SEQ_HALTON
    T, I = model(H, cfg.n_xd, cfg.n_if)
    plan = rsi.Plan.chain(T, I, cfg.media, grid, freqs, rsi.RSI_T_GLOBAL, rsi.RSI_FP32)
    dt = timed(plan.execute, args.steps, args.warmup)
    n_g = grid[0].numel()
    pairs = cfg.n_xd * cfg.n_if + cfg.n_if * n_g
    k2 = 2 * math.pi * cfg.freq / c2
    vel = lambda phi: k2 * np.abs(phi)                      # k2 |phi| / v0, v0 = 1

    def on(T_, I_, tgt, prec=rsi.RSI_FP32):
        return rsi.rsi_chain(T_, I_, cfg.media, tgt, freqs, rsi.RSI_T_GLOBAL, prec)[0].cpu().numpy()

    z = cfg.axis_z
    ax_h32 = on(T, I, line)
    ax_h64 = on(T, I, line, rsi.RSI_FP64)
    ax_s32 = on(*model(rsi.RSI_SEQ_SOBOL, cfg.n_xd, cfg.n_if), line)
    n_ref = 1 << 20
    ax_ref = on(*model(rsi.RSI_SEQ_SOBOL, n_ref, n_ref), line)
    ax_ref_h = on(*model(H, n_ref, n_ref), line)
    ax_apod = on(*model(H, cfg.n_xd, cfg.n_if, apod=True), line)
    ax_flat = on(*model(H, cfg.n_xd, cfg.n_if, flat=True), line)
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))

    def peak(a):
        v = vel(a)
        i = int(np.argmax(v))
        if 0 < i < len(v) - 1:                               # parabolic refinement
            y0, y1, y2 = v[i - 1], v[i], v[i + 1]
            d = 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2)
            return float(z[i] + d * (z[1] - z[0])), float(y1 - 0.25 * (y0 - y2) * d)
        return float(z[i]), float(v[i])

    zp, vp = peak(ax_h32)
    zp_apod, vp_apod = peak(ax_apod)
    _, vp_flat = peak(ax_flat)
    fl = vel(on(T, I, focal))
    y = cfg.focal_line()[1]
    above = y[fl >= 0.5 * fl.max()]
    img = plan.out[0].cpu().numpy().reshape(cfg.n_grid, cfg.n_grid)
    iz, iy = np.unravel_index(int(np.argmax(np.abs(img))), img.shape)
    line_out = base_line(pairs * args.steps / dt / 1e9, args.steps, args.warmup, dt,
                         {"workload": "focused_normal: spherical cap a 6.35 mm R 33 mm, 10 mm water -> "
                                      "steel 5840 m/s, 2.5 MHz, 10^5 Halton per surface, interface +-3a, "
                                      "global T -> 401 x 401 y-z slice 1-25 mm below the interface",
                          "pairs_per_step": pairs})
    line_out.update({
        "axis_peak_z_mm": round(1e3 * zp, 3),
        "paper_focal_z_mm": round(1e3 * cfg.z_focus_paper, 3),
        "paraxial_geometric_focus_z_mm": round(1e3 * (cfg.water_path + (cfg.curvature - cfg.water_path) * c1 / c2), 3),
        "axis_peak_k2phi_over_v0": round(vp, 4),
        "image_peak_z_mm": round(1e3 * cfg.grid()[2].reshape(cfg.n_grid, cfg.n_grid)[iz, iy], 3),
        "focal_gain_over_flat_piston": round(vp / vp_flat, 3),
        "focal_spot_minus6db_width_mm_at_paper_focus": round(1e3 * (above.max() - above.min()), 3),
        "apodised_axis_peak_z_mm": round(1e3 * zp_apod, 3),
        "apodised_peak_over_uniform": round(vp_apod / vp, 4),
        "axis_rel_l2_halton_1e5_vs_sobol_2p20": rel(ax_h32, ax_ref),
        "axis_rel_l2_sobol_1e5_vs_sobol_2p20": rel(ax_s32, ax_ref),
        "axis_rel_l2_halton_2p20_vs_sobol_2p20": rel(ax_ref_h, ax_ref),
        "axis_fp32_vs_fp64_rel_l2": rel(ax_h32, ax_h64),
    })
    print(json.dumps(line_out), flush=True)
    plan.destroy()


def _event_ms(fn, reps=3):
    """Median time of fn() in ms, HIP events on torch's current stream (the library
    launches on it), after one untimed call."""
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def flops_ray_pair(n_layers, n_freq=1, newton=2):
    """Algorithmic FP32 flops of one ray pair (FMA = 2, transcendental = 1), frozen at
    two Newton evaluations: fixed 14 (geometry, predictor) + per evaluation 9 per layer
    + 8, + 13 per layer + 3 after the root (travel time, spreading, transmission), + 9
    per frequency (phase, sin, cos, accumulation)."""
    L = n_layers
    return 14 + newton * (9 * L + 8) + 13 * L + 3 + 9 * n_freq


def ray_field_leg(args):
    """Ray tracing (Sec. 2.2, eq. 12) on the oblique-incidence configuration of Sec. 3.1:
    tilted piston (10 deg, 2.5 MHz), 10^5 Halton samples, one water/steel plane at 0.1 m,
    a 401 x 401 slice of the x-z plane below it, FP32; FP64 and the RSI chain on a
    sample of the slice for the error."""
    import torch
    from paper_2408_06765_amd import rsi
    from paper_2408_06765_amd import workloads as W

    cfg = W.RayCrossover()
    media = cfg.stacks[1]
    zs = cfg.planes(media)
    H = rsi.RSI_SEQ_HALTON
    xs = rsi.rsi_sample_disc(cfg.xd_seed, cfg.n_samples, cfg.radius, (0.0, 0.0, 0.0), cfg.tilt, seq=H)
    T = rsi.Transducer(*xs[:3], xs[3], 1.0, (0.0, 0.0, 0.0), cfg.axis)
    n = 401
    xc = cfg.patch_centres(media)[0]
    X, Z = np.meshgrid(np.linspace(xc - 0.01, xc + 0.04, n), zs[0] + np.linspace(0.001, 0.04, n))
    tgt = tuple(torch.as_tensor(a.ravel().copy(), device="cuda") for a in (X, 0 * X, Z))
    out = torch.empty((1, n * n), dtype=torch.complex64, device="cuda")
    run = lambda: rsi.rsi_ray_field(T, zs, media, tgt, [cfg.freq], rsi.RSI_FP32, out=out)
    dt = timed(run, args.steps, args.warmup)
    pairs = cfg.n_samples * n * n
    # errors on every 97th point: FP32 vs FP64 ray model, ray model vs RSI chain
    sub = torch.arange(0, n * n, 97, device="cuda")
    ts = tuple(a[sub].contiguous() for a in tgt)
    f32 = out[0, sub].cpu().numpy()
    f64 = rsi.rsi_ray_field(T, zs, media, ts, [cfg.freq], rsi.RSI_FP64)[0].cpu().numpy()
    q = rsi.rsi_sample_square(1 << 20, cfg.n_samples, xc, 0.0, zs[0], cfg.half_width, seq=H)
    I = [rsi.Interface(*q[:3], q[3], zs[0])]
    ch = rsi.rsi_chain(T, I, media, ts, [cfg.freq], rsi.RSI_T_LOCAL, rsi.RSI_FP64)[0].cpu().numpy()
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    fl = flops_ray_pair(len(media))
    tflops = pairs * fl * args.steps / dt / 1e12
    line = base_line(pairs * args.steps / dt / 1e9, args.steps, args.warmup, dt,
                     {"workload": "ray_field: tilted piston (10 deg, 2.5 MHz) 10^5 Halton -> ray tracing "
                                  "through water/steel (5840 m/s) at 0.1 m -> 401 x 401 x-z slice 1-40 mm "
                                  "below", "pairs_per_step": pairs})
    line["metric"] = "Gpairs/s ray tracing (eq. 12, one root of eq. 14 per pair) + % FP32 VALU peak"
    line.update({
        "flops_per_pair_convention": fl,
        "tflops_algorithmic": round(tflops, 2),
        "frac_fp32_peak": round(tflops / PEAK_FP32_TFLOPS, 4),
        "fp32_vs_fp64_rel_l2": rel(f32, f64),
        "ray_vs_rsi_chain_rel_l2": rel(f64, ch),
    })
    print(json.dumps(line), flush=True)


def ray_crossover(args):
    """Sec. 3.5 / Fig. 8: time of the RSI chain and of the ray model against the number
    of field points through 0, 1 and 4 planes (FP32, one-shot calls, HIP events), and
    where the two curves cross."""
    import torch
    from paper_2408_06765_amd import rsi
    from paper_2408_06765_amd import workloads as W

    cfg = W.RayCrossover()
    H = rsi.RSI_SEQ_HALTON
    xs = rsi.rsi_sample_disc(cfg.xd_seed, cfg.n_samples, cfg.radius, (0.0, 0.0, 0.0), cfg.tilt, seq=H)
    T = rsi.Transducer(*xs[:3], xs[3], 1.0, (0.0, 0.0, 0.0), cfg.axis)
    freqs = [cfg.freq]
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    table = {}
    for media in cfg.stacks:
        zs = cfg.planes(media)
        I = []
        for m, (z, xc) in enumerate(zip(zs, cfg.patch_centres(media))):
            q = rsi.rsi_sample_square((m + 1) << 20, cfg.n_samples, xc, 0.0, z, cfg.half_width, seq=H)
            I.append(rsi.Interface(*q[:3], q[3], z))
        rows = []
        for nf in cfg.n_field:
            tgt = tuple(torch.as_tensor(a, device="cuda") for a in cfg.field(media, nf))
            o1 = torch.empty((1, nf), dtype=torch.complex64, device="cuda")
            o2 = torch.empty((1, nf), dtype=torch.complex64, device="cuda")
            t_rsi = _event_ms(lambda: rsi.rsi_chain(T, I, media, tgt, freqs, rsi.RSI_T_LOCAL, rsi.RSI_FP32, out=o1))
            t_ray = _event_ms(lambda: rsi.rsi_ray_field(T, zs, media, tgt, freqs, rsi.RSI_FP32, out=o2))
            row = {"n_field": nf, "rsi_ms": round(t_rsi, 3), "ray_ms": round(t_ray, 3)}
            if nf == 1000:
                row["ray_vs_rsi_rel_l2"] = rel(o2.cpu().numpy(), o1.cpu().numpy())
            rows.append(row)
            print(f"planes {len(zs)} n_field {nf}: rsi {t_rsi:.3f} ms ray {t_ray:.3f} ms", file=sys.stderr,
                  flush=True)
        # crossover: first interval where the ray time overtakes the RSI time (log-log);
        # without a plane both calls run the same monopole pair sum, so there is none
        cross = None
        for a, b in zip(rows[:-1], rows[1:]) if zs else ():
            da, db = math.log(a["ray_ms"] / a["rsi_ms"]), math.log(b["ray_ms"] / b["rsi_ms"])
            if da < 0 <= db:
                u = da / (da - db)
                cross = round(math.exp(math.log(a["n_field"]) + u * math.log(b["n_field"] / a["n_field"])))
                break
        table[len(zs)] = {"rows": rows, "crossover_n_field": cross}
    line = {
        "metric": "field points above which the RSI chain is faster than ray tracing (Fig. 8)",
        "value": table[1]["crossover_n_field"], "unit": "field points", "n_gpus": 1, "steps": 3,
        "warmup": 1, "ms_per_step": None, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "ray_crossover: tilted piston (10 deg, 2.5 MHz), 0.1 m water, 0/1/4 planes "
                               "(water/steel/aluminium/steel/water, 2 mm), 10^5 Halton samples per surface, "
                               "field points in the last medium"},
        "planes": {str(k): v for k, v in table.items()},
    }
    print(json.dumps(line), flush=True)


def scan_batch(args):
    """256 uneven scan positions in one persistent launch (batched plan)."""
    import torch
    from paper_2408_06765_amd import rsi
    from paper_2408_06765_amd import workloads as W

    cfg = W.ScanBatch()
    insts = []
    for it in cfg.instances():
        xs = rsi.rsi_sample_disc(it.seed, it.n_src, cfg.radius, (it.x_offset, 0.0, 0.0), it.tilt)
        tgt = tuple(torch.as_tensor(a, device="cuda") for a in cfg.field_points(it))
        insts.append(rsi.Instance(xs[:3], xs[3], tgt, cfg.medium[0], cfg.freq, rsi.RSI_MONOPOLE))
    if args.autotune:
        rsi.rsi_autotune_batched(insts, rsi.RSI_FP32)
    plan = rsi.Plan.batched(insts, rsi.RSI_FP32)
    dt = timed(plan.execute, args.steps, args.warmup)
    pairs = sum(i.w.numel() * i.tgt[0].numel() for i in insts)
    line = base_line(pairs * args.steps / dt / 1e9, args.steps, args.warmup, dt,
                     {"workload": "scan_batch: 256 piston scan positions, 2^12-2^18 sources, "
                                  "1e3-1e5 field points, 1 MHz water, one persistent launch",
                      "pairs_per_step": pairs})
    print(json.dumps(line), flush=True)
    plan.destroy()


def multilayer_noise(args):
    """QMC noise of the RSI chain through thin layers (Sec. 3.4): rel-L2 of the FP32 field
    at N Halton samples per surface against N_ref on the same points, through the seven
    planes of six 2 mm steel/aluminium layers and, for contrast, through one plane; and
    the time of each chain."""
    import torch
    from paper_2408_06765_amd import rsi
    from paper_2408_06765_amd import workloads as W

    cfg = W.MultilayerNoise()
    H = rsi.RSI_SEQ_HALTON

    def chain(media, n):
        zs = cfg.planes(media)
        xs = rsi.rsi_sample_disc(0, n, cfg.radius, (0.0, 0.0, 0.0), cfg.tilt, seq=H)
        T = rsi.Transducer(*xs[:3], xs[3], 1.0, (0.0, 0.0, 0.0), cfg.axis)
        ifs = []
        for m, (z, xc) in enumerate(zip(zs, cfg.patch_centres(media))):
            q = rsi.rsi_sample_square((m + 1) << 24, n, xc, 0.0, z, cfg.half_width, seq=H)
            ifs.append(rsi.Interface(*q[:3], q[3], z))
        tgt = tuple(torch.as_tensor(a, device="cuda") for a in cfg.field(media))
        f = lambda: rsi.rsi_chain(T, ifs, media, tgt, [cfg.freq], rsi.RSI_T_LOCAL, rsi.RSI_FP32)[0]
        out = f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = f()
        torch.cuda.synchronize()
        return out.cpu().numpy(), time.perf_counter() - t0

    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    res = {}
    for name, media in (("seven_planes", cfg.media), ("one_plane", cfg.one_plane)):
        ref, t_ref = chain(media, cfg.n_ref)
        rows = []
        for n in cfg.counts:
            got, dt = chain(media, n)
            rows.append({"samples_per_surface": n, "rel_l2_vs_ref": rel(got, ref), "ms": round(1e3 * dt, 3)})
            print(f"{name} N={n}: rel-L2 {rows[-1]['rel_l2_vs_ref']:.3e}, {1e3 * dt:.2f} ms", file=sys.stderr,
                  flush=True)
        lg = np.log([r["samples_per_surface"] for r in rows])
        le = np.log([r["rel_l2_vs_ref"] for r in rows])
        res[name] = {"rows": rows, "ref_samples": cfg.n_ref, "ref_ms": round(1e3 * t_ref, 1),
                     "loglog_slope": float(np.polyfit(lg, le, 1)[0])}
    at = {n: r for n, r in zip(cfg.counts, res["seven_planes"]["rows"])}
    line = {
        "metric": "RSI QMC error through six 2 mm steel/aluminium layers (Sec. 3.4) at 10^5 samples per surface",
        "value": at[100000]["rel_l2_vs_ref"], "unit": "rel-L2 vs 2e6 samples", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": at[100000]["ms"], "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "multilayer_noise: tilted piston (10 deg, 2.5 MHz), 10 mm water, six 2 mm "
                               "steel/aluminium layers over steel (7 planes), Halton samples, field on and "
                               "across the refracted axis"},
        "stacks": res,
    }
    print(json.dumps(line), flush=True)


def surrogate(args):
    """The learned surrogate: 10^7 RSI samples (5120 random configurations of the
    one-interface piston family x 1953 points, drawn where the recipe trains: f <= 7.75 MHz,
    tilt <= 10 deg; the chain at 2^16 piston and 2^20 interface samples), 7 x 256 MLP on the
    ray-model carrier trained with the MFMA kernels, held-out residual per (f, depth, tilt)
    cell (8 x 4 x 8 over the whole box) against the judge (the chain at the same counts),
    10^6 queries (64 random configurations over the whole box x 125^2) answered by the
    surrogate where its cell passes the threshold and by the judge elsewhere."""
    import torch
    from paper_2408_06765_amd import surrogate as S

    cfg = S.SurrogateConfig()
    if args.sur_train_f_max is not None:
        cfg.train_f_max = args.sur_train_f_max
    if args.sur_train_tilt_max is not None:
        cfg.train_tilt_max = math.radians(args.sur_train_tilt_max)
    if args.sur_carrier_samples is not None:
        cfg.n_carrier = args.sur_carrier_samples
    if args.sur_judge_scale is not None:
        cfg.judge_scale = args.sur_judge_scale
    if args.sur_epochs is not None:
        cfg.epochs = args.sur_epochs
    if args.sur_train_if_scale is not None:
        cfg.train_if_scale = args.sur_train_if_scale
    if args.sur_depth is not None:
        cfg.depth = args.sur_depth
    sur = S.Surrogate(cfg)
    t0 = time.perf_counter()
    q, t = sur.dataset(S.training_configs(cfg, 5120, 3), points_per_config=1953)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss = sur.train(q, t, log=lambda s: print(s, file=sys.stderr, flush=True))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    del q, t
    errs = sur.validate(S.cell_configs(cfg, 101))
    e = np.array([errs[c] for c in sorted(errs)])
    qc = S.random_configs(cfg, 64, 202)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    out, used = sur.answer(qc)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    for f, d, tl in qc:
        sur.judge(f, d, tl)
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    for f, d, tl in qc:
        sur.predict(f, d, tl)
    torch.cuda.synchronize()
    t6 = time.perf_counter()
    for f, d, tl in qc:
        sur.network(sur.src.queries(f, d, tl))
    torch.cuda.synchronize()
    t7 = time.perf_counter()
    # speedup where the surrogate answers: its time against RSI on the passing configurations
    ok = [not u for u in used]
    pass_cfgs = [c for c, o in zip(qc, ok) if o]
    rsi_pass = sur_pass = None
    if pass_cfgs:
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for f, d, tl in pass_cfgs:
            sur.judge(f, d, tl)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        for f, d, tl in pass_cfgs:
            sur.predict(f, d, tl)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        rsi_pass, sur_pass = tb - ta, tc - tb
    # the carrier alone (network output zero) against RSI: what the network adds
    carrier = []
    if cfg.carrier == "ray":
        for f, d, tl in S.cell_configs(cfg, 101):
            if f <= cfg.train_f_max and tl <= cfg.train_tilt_max:
                carrier.append(S.rel_l2(sur.src.ray_pressure(f, d, tl), sur.judge(f, d, tl)))
    # the judge's own noise: RSI against RSI with both sample counts doubled, per cell (a
    # cell whose RSI moves by more than the threshold cannot be matched by a smooth model)
    js = cfg.judge_scale
    judge = {}
    for f, d, tl in S.cell_configs(cfg, 101):
        judge[S.cell_of(cfg, f, d, tl)] = S.rel_l2(sur.src.rsi_pressure(f, d, tl, scale=2, if_scale=2 * js),
                                                  sur.judge(f, d, tl))
    # RSI at the training data's counts for the same queries (the cost the judge's counts add)
    torch.cuda.synchronize()
    tr0 = time.perf_counter()
    for f, d, tl in qc:
        sur.src.rsi_pressure(f, d, tl)
    torch.cuda.synchronize()
    rsi_base_s = time.perf_counter() - tr0
    jn = np.array([judge[c] for c in sorted(judge)])
    reach = [c for c in sorted(judge) if judge[c] <= cfg.threshold]
    rsi_s, routed_s, sur_s, net_s = t5 - t4, t4 - t3, t6 - t5, t7 - t6
    n_q = len(qc) * cfg.nx * cfg.nz
    thresholds = [1e-3, 1e-2, 1e-1, 0.3, 1.0]
    line = {
        "metric": "surrogate speedup over RSI at <= 1e-3 rel-L2 (held-out, per cell)",
        "value": round(rsi_s / routed_s, 3), "unit": "x", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(1e3 * routed_s, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 (MFMA, FP32 accumulation)", "data": "synthetic",
        "config": {"workload": "surrogate: piston + water/5900 m/s interface, x, z, f 1-10 MHz, depth "
                               "30-70 mm, tilt 0-20 deg; 5 x 256 Fourier-feature MLP on the "
                               + (f"ray-model carrier ({cfg.n_carrier} samples), trained on f <= {cfg.train_f_max / 1e6:g} MHz, "
                                  f"tilt <= {math.degrees(cfg.train_tilt_max):g} deg"
                                  if cfg.carrier == "ray" else "plane-wave carrier"),
                   "train_samples": 5120 * 1953, "queries": n_q},
        "judge_scale": js, "judge_samples": [cfg.n_xd, cfg.n_if * js],
        "train_samples_per_surface": [cfg.n_xd, cfg.n_if * cfg.train_if_scale],
        "epochs": cfg.epochs,
        "data_generation_s": round(t1 - t0, 2), "train_s": round(t2 - t1, 2), "final_loss": loss,
        "rsi_at_training_counts_s_for_queries": round(rsi_base_s, 4),
        "surrogate_speedup_all_queries_vs_rsi_at_training_counts": round(rsi_base_s / routed_s, 3),
        "cell_residual": {"min": float(e.min()), "median": float(np.median(e)), "max": float(e.max())},
        "cells_passing": {str(th): int((e <= th).sum()) for th in thresholds}, "cells": int(e.size),
        "cells_in_training_region": int(sum(1 for (f, d, tl) in S.cell_configs(cfg, 101)
                                            if f <= cfg.train_f_max and tl <= cfg.train_tilt_max)),
        "queries_on_rsi_fallback": int(sum(used)),
        "rsi_s_for_queries": round(rsi_s, 4), "surrogate_s_for_queries": round(sur_s, 4),
        "network_s_for_queries": round(net_s, 4), "surrogate_speedup_all_queries": round(rsi_s / sur_s, 2),
        "network_only_speedup": round(rsi_s / net_s, 2),
        "passing_configurations": len(pass_cfgs),
        "speedup_in_passing_cells": round(rsi_pass / sur_pass, 2) if pass_cfgs else None,
        "cells_passing_list": [int(c) for c in sorted(errs) if errs[c] <= cfg.threshold],
        "rsi_self_change_when_doubled": {"min": float(jn.min()), "median": float(np.median(jn)),
                                         "max": float(jn.max())},
        "cells_where_rsi_is_within_threshold_of_itself": len(reach),
        "of_those_passing": int(sum(1 for c in reach if errs[c] <= cfg.threshold)),
        "rsi_self_change_per_cell": [float(judge[c]) for c in sorted(judge)],
        "surrogate_residual_per_cell": [float(errs[c]) for c in sorted(errs)],
    }
    if carrier:
        cr = np.array(carrier)
        line["carrier_only_residual_in_training_region"] = {"min": float(cr.min()), "median": float(np.median(cr)),
                                                            "max": float(cr.max())}
    print(json.dumps(line), flush=True)


def flops_mlp_row(n_ff, width, depth):
    """Algorithmic flops of one query row of the surrogate network (FMA = 2): the hidden
    layers' products and the head; the features and the SiLU are not counted."""
    return 2 * (2 * n_ff * width + (depth - 1) * width * width + 2 * width)


def surrogate_inference(args):
    """The surrogate network's inference, one fused launch per call (features, the hidden
    SiLU layers on the bf16 MFMA, head), over 65536 query rows and over one configuration's
    125 x 125 image; weights of the recipe's shape, random-initialised and seeded (the
    time does not depend on their values)."""
    import torch
    from paper_2408_06765_amd import surrogate as S

    cfg = S.SurrogateConfig()
    if args.sur_depth is not None:
        cfg.depth = args.sur_depth
    lo, hi = S.lohi(cfg.box)
    net = S.MLP(cfg.n_ff, cfg.width, cfg.depth, S.fourier_matrix(cfg.n_ff, cfg.ff_scales, cfg.seed),
                lo, hi, cfg.batch)
    net.set_params(S.glorot_params(cfg.n_ff, cfg.width, cfg.depth, cfg.seed))
    rng = np.random.default_rng(0)

    def rows(n):
        q = np.stack([rng.uniform(lo[c], hi[c], n) for c in range(5)], 1).astype(np.float32)
        return torch.as_tensor(q, device="cuda"), torch.empty((n, 2), dtype=torch.float32, device="cuda")

    n, n_img = cfg.batch, cfg.nx * cfg.nz
    q, y = rows(n)
    q2, y2 = rows(n_img)
    run = lambda: net.forward(q, y)
    dt = timed(run, args.steps, args.warmup)
    # 20 back-to-back calls between the events: a single call's events add launch latency
    kms = _event_ms(lambda: [run() for _ in range(20)], reps=max(3, args.kernel_reps or 5)) / 20
    kms2 = _event_ms(lambda: [net.forward(q2, y2) for _ in range(20)], reps=max(3, args.kernel_reps or 5)) / 20
    net.destroy()
    fl = flops_mlp_row(cfg.n_ff, cfg.width, cfg.depth)
    achieved = n * fl / (kms * 1e-3) / 1e12
    line = base_line(n * args.steps / dt, args.steps, args.warmup, dt,
                     {"workload": f"surrogate_inference: {2 * cfg.n_ff} Fourier features -> "
                                  f"{cfg.depth} x {cfg.width} SiLU (bf16 MFMA, FP32 accumulation) -> 2, "
                                  f"{n} query rows per call", "rows_per_step": n}, unit="rows/s")
    line["metric"] = "surrogate inference rows/s (fused network launch) + % bf16 MFMA peak"
    line["dtype"] = "bf16"
    line["roofline"] = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_BF16_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / PEAK_BF16_TFLOPS, 4), "traffic": None,
                        "kernel": f"mlp_infer_fused_kernel<{cfg.width}, 128>, {fl} flop/row x {n} rows / "
                                  f"{kms:.4f} ms"}
    line["image_call"] = {"rows": n_img, "ms": round(kms2, 4),
                          "tflops": round(n_img * fl / (kms2 * 1e-3) / 1e12, 2)}
    print(json.dumps(line), flush=True)


def one_interface(args):
    """The single-frequency chain: piston (2^16, 5 MHz, tilted 10 deg) -> one interface
    (2^18) -> 512 x 512 image, local transmission coefficient."""
    import torch
    from paper_2408_06765_amd import rsi
    from paper_2408_06765_amd import workloads as W

    cfg = W.OneInterface()
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    cx, cy = cfg.patch_centre
    # inputs: generated on the device by the library's own sampler, resident in HBM
    xs = rsi.rsi_sample_disc(cfg.xd_seed, cfg.n_xd, cfg.radius, (0.0, 0.0, 0.0), cfg.tilt)
    qs = rsi.rsi_sample_square(cfg.if_seed, cfg.n_if, cx, cy, cfg.z_if, cfg.half_width)
    tgt = tuple(dev(a) for a in cfg.targets())
    T = rsi.Transducer(*xs[:3], xs[3], 1.0, (0.0, 0.0, 0.0), cfg.axis)
    I = [rsi.Interface(*qs[:3], qs[3], cfg.z_if)]
    freqs = [cfg.freq]
    plan = rsi.Plan.chain(T, I, cfg.media, tgt, freqs, rsi.RSI_T_LOCAL, rsi.RSI_FP32)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        plan.execute()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.execute()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1e3 * dt / max(args.steps, 1)
    pairs_stage0 = cfg.n_xd * cfg.n_if
    pairs_stage1 = cfg.n_if * cfg.nx * cfg.nz
    pairs = pairs_stage0 + pairs_stage1
    value = pairs * args.steps / dt / 1e9

    # dominant kernel: the interface (dipole) pair sum, one call per launch, timed with
    # HIP events on the stream it runs on
    reps = args.kernel_reps if args.kernel_reps is not None else 5
    s = torch.cuda.Stream()
    vel = torch.ones(cfg.n_if, dtype=torch.complex128, device="cuda")
    out = torch.empty(cfg.nx * cfg.nz, dtype=torch.complex64, device="cuda")
    with torch.cuda.stream(s):
        rsi.rsi_propagate_ex(qs[:3], qs[3], vel, tgt, cfg.media[1][0], cfg.freq, rsi.RSI_DIPOLE,
                             rsi.RSI_FP32, rsi.RSI_FLAG_PLANAR_Z, normal=(0.0, 0.0, 1.0), out=out)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for e0, e1 in ev:
            e0.record(s)
            rsi.rsi_propagate_ex(qs[:3], qs[3], vel, tgt, cfg.media[1][0], cfg.freq,
                                 rsi.RSI_DIPOLE, rsi.RSI_FP32, rsi.RSI_FLAG_PLANAR_Z,
                                 normal=(0.0, 0.0, 1.0), out=out)
            e1.record(s)
    s.synchronize()
    kms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev]))
    achieved = FLOPS_DIPOLE * pairs_stage1 / (kms * 1e-3) / 1e12

    # sanity of the timed output against stored reference samples, when present
    check = None
    gold = os.path.join(ROOT, "tests", "golden", "one_interface_samples.json")
    if os.path.exists(gold):
        g = json.load(open(gold))
        idx = np.array(g["index"])
        ref = np.array(g["re"]) + 1j * np.array(g["im"])
        got = plan.out[0].cpu().numpy()[idx]
        check = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))

    line = {
        "metric": "Gpairs/s RSI-QMC (chained pair sum) + % FP32 VALU peak",
        "value": round(value, 3),
        "unit": "Gpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "one_interface: piston 2^16 -> interface 2^18 -> image 512x512, "
                               "5 MHz, water->5900 m/s solid, tilt 10 deg, local T",
                   "pairs_per_step": pairs, "precision": "fp32 (fp64 reference distance + phase)"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                     "traffic": measured_traffic(),
                     "kernel": "pairsum_f32_kernel<dipole, planar> (interface -> image), "
                               f"{FLOPS_DIPOLE} flop/pair x {pairs_stage1:.3e} pairs / {kms:.3f} ms"},
    }
    line["fp32_valu_counters"] = measured_valu()
    if check is not None:
        line["parity_vs_oracle_samples"] = check
    if args.calib_copy:
        line["calib_copy_bytes"] = calib_copy()
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(line), flush=True)
    plan.destroy()




def flops_mlp_train_row(n_ff, width, depth):
    """Algorithmic flops of one row of a training step (FMA = 2): the forward products and
    head, the weight gradients of every layer and the head, and the input gradients of
    every layer but the first (the features need none)."""
    F, W, L = 2 * n_ff, width, depth
    fwd = 2 * (F * W + (L - 1) * W * W + 2 * W)
    dw = 2 * (F * W + (L - 1) * W * W + 2 * W)
    dx = 2 * ((L - 1) * W * W + 2 * W)
    return fwd + dw + dx


def bytes_mlp_train_step(n_ff, width, depth, n, splits):
    """HBM bytes one training step's kernels read and write, from the tensors' shapes (a
    traffic model, not a counter reading): bf16 features and activations, FP32
    pre-activations, bf16 layer gradients, the weight gradients' FP32 split partials
    (written and read once), the FP32 parameters and Adam moments and the weights' three
    bf16 copies.  Per row: features 2F; forward layer l reads 2 I_l, writes 2W + 4W; the head
    reads 2W + 4W, writes 2W, and its gradient reads 2W again; backward layer l reads dZ (2W)
    and H_l (2 I_l) for the weight gradient and dZ (2W) for the bias gradient, and (l >= 1)
    dZ (2W) and Z_{l-1} (4W) while writing dZ_{l-1} (2W)."""
    F, W, L = 2 * n_ff, width, depth
    ins = [F] + [W] * (L - 1)
    row = 2 * F
    row += sum(2 * i + 6 * W for i in ins)
    row += 8 * W + 2 * W
    row += sum(2 * W + 2 * i + 2 * W for i in ins) + (L - 1) * 8 * W
    weights = sum(W * i for i in ins)
    params = weights + L * W + 2 * W + 2
    step = 2 * 4 * splits * weights  # split partials, written and read
    step += params * (4 + 4 + 2 * 8) + weights * 3 * 2  # p read/write, m and v read/write, bf16 copies
    return n * row + step


def dw_splits(n):
    """The weight gradient's batch splits the library picks for n rows: the largest power of
    two up to 128 that leaves at least 256 rows per split."""
    mp, s = (n + 63) // 64 * 64, 1
    while s < 128 and mp // (2 * s) >= 256:
        s *= 2
    return s


def surrogate_training(args):
    """One Adam step of the surrogate network (the recipe's shape: 128 Fourier frequencies,
    7 x 256 SiLU, bf16 MFMA GEMMs with FP32 accumulation) on a batch of 65536 rows: features,
    forward, loss, backward, Adam, bf16 weight refresh.  Rows and targets are seeded
    synthetic values (the time does not depend on them)."""
    import torch
    from paper_2408_06765_amd import surrogate as S

    cfg = S.SurrogateConfig()
    if args.sur_depth is not None:
        cfg.depth = args.sur_depth
    lo, hi = S.lohi(cfg.box)
    n = cfg.batch
    net = S.MLP(cfg.n_ff, cfg.width, cfg.depth, S.fourier_matrix(cfg.n_ff, cfg.ff_scales, cfg.seed),
                lo, hi, n)
    net.set_params(S.glorot_params(cfg.n_ff, cfg.width, cfg.depth, cfg.seed))
    rng = np.random.default_rng(0)
    q = torch.as_tensor(np.stack([rng.uniform(lo[c], hi[c], n) for c in range(5)], 1).astype(np.float32),
                        device="cuda")
    t = torch.as_tensor(rng.normal(size=(n, 2)).astype(np.float32), device="cuda")
    run = lambda: net.train_step(q, t, 1e-5)
    dt = timed(run, args.steps, args.warmup)
    kms = _event_ms(lambda: [run() for _ in range(10)], reps=3) / 10
    net.destroy()
    fl = flops_mlp_train_row(cfg.n_ff, cfg.width, cfg.depth)
    achieved = n * fl / (kms * 1e-3) / 1e12
    line = base_line(n * args.steps / dt, args.steps, args.warmup, dt,
                     {"workload": f"surrogate_training: {2 * cfg.n_ff} Fourier features -> {cfg.depth} x "
                                  f"{cfg.width} SiLU -> 2, Adam, {n} rows per step", "rows_per_step": n},
                     unit="rows/s")
    line["metric"] = "surrogate training rows/s (one Adam step per batch) + % bf16 MFMA peak"
    line["dtype"] = "bf16"
    line["roofline"] = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_BF16_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / PEAK_BF16_TFLOPS, 4), "traffic": None,
                        "kernel": f"whole training step, {fl} flop/row x {n} rows / {kms:.4f} ms"}
    # the step is bound by memory traffic: the same time against the HBM peak
    nb = bytes_mlp_train_step(cfg.n_ff, cfg.width, cfg.depth, n, dw_splits(n))
    line["hbm_view"] = {"bytes_per_step": nb, "achieved": round(nb / (kms * 1e-3) / 1e9, 1),
                        "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                        "frac": round(nb / (kms * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4),
                        "basis": "tensor bytes the step's kernels read and write, from the shapes"}
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "one_interface":
        return one_interface(args)
    if args.workload == "interface_continuity":
        return interface_continuity(args)
    if args.workload == "focused_normal":
        return focused_normal(args)
    if args.workload == "ray_field":
        return ray_field_leg(args)
    if args.workload == "ray_crossover":
        return ray_crossover(args)
    if args.workload == "scan_batch":
        return scan_batch(args)
    if args.workload == "surrogate":
        return surrogate(args)
    if args.workload == "multilayer_noise":
        return multilayer_noise(args)
    if args.workload == "surrogate_inference":
        return surrogate_inference(args)
    if args.workload == "surrogate_training":
        return surrogate_training(args)
    return layered_stack(args)


if __name__ == "__main__":
    main()

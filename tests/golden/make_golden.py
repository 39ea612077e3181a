"""Write the stored reference samples used by the full-size GPU tests.

Calls only the FP64 reference (oracle/) and the seeded workload definitions.  The
full interface field is computed exactly (every interface sample), then the field at
a seeded subset of the image points.

    python tests/golden/make_golden.py one_interface      # ~1.7e10 pairs
    python tests/golden/make_golden.py layered_stack      # two frequencies, ~3e11 pairs
    python tests/golden/make_golden.py focused_normal     # ~1e10 pairs
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2408_06765_amd import workloads as W  # noqa: E402


def one_interface(n_samples=256):
    cfg = W.OneInterface()
    xd = oracle.sample_disc(cfg.xd_seed, cfg.n_xd, cfg.radius, (0.0, 0.0, 0.0), cfg.tilt)
    cx, cy = cfg.patch_centre
    q = oracle.sample_square(cfg.if_seed, cfg.n_if, cx, cy, cfg.z_if, cfg.half_width)
    tx, ty, tz = cfg.targets()
    rng = np.random.default_rng(2024)
    idx = np.sort(rng.choice(tx.size, n_samples, replace=False))
    t0 = time.time()
    phi = oracle.chain(xd, 1.0, (0.0, 0.0, 0.0), cfg.axis, [q], [cfg.z_if],
                       [m[0] for m in cfg.media], [m[1] for m in cfg.media],
                       (tx[idx], ty[idx], tz[idx]), [cfg.freq], oracle.T_LOCAL)[0]
    # the interface field itself at a subset of interface samples (stage 0)
    qidx = np.sort(rng.choice(cfg.n_if, n_samples, replace=False))
    phi0 = oracle.propagate(0, xd[:3], xd[3], 1.0, tuple(a[qidx] for a in q[:3]), cfg.media[0][0], cfg.freq)
    return {
        "workload": "one_interface", "seconds": time.time() - t0,
        "index": idx.tolist(), "re": phi.real.tolist(), "im": phi.imag.tolist(),
        "iface_index": qidx.tolist(), "iface_re": phi0.real.tolist(), "iface_im": phi0.imag.tolist(),
    }


def layered_stack(n_samples=128, freqs=(1.0e6, 10.0e6)):
    cfg = W.LayeredStack()
    xd = oracle.sample_disc(cfg.xd_seed, cfg.n_xd, cfg.radius, (0.0, 0.0, 0.0), cfg.tilt)
    ifs = [oracle.sample_square(s, cfg.n_if, c[0], c[1], z, cfg.half_width)
           for s, c, z in zip(cfg.if_seeds, cfg.patch_centres, cfg.z_if)]
    tx, ty, tz = cfg.targets()
    rng = np.random.default_rng(2025)
    idx = np.sort(rng.choice(tx.size, n_samples, replace=False))
    all_f = cfg.freqs
    fidx = [int(np.argmin(np.abs(all_f - f))) for f in freqs]
    t0 = time.time()
    phi = oracle.chain(xd, 1.0, (0.0, 0.0, 0.0), cfg.axis, ifs, list(cfg.z_if),
                       [m[0] for m in cfg.media], [m[1] for m in cfg.media],
                       (tx[idx], ty[idx], tz[idx]), all_f[fidx], oracle.T_LOCAL)
    return {
        "workload": "layered_stack", "seconds": time.time() - t0, "freq_index": fidx,
        "index": idx.tolist(), "re": phi.real.tolist(), "im": phi.imag.tolist(),
    }


def focused_normal(n_samples=64):
    """Focused transducer over water/steel (Sec. 3.3): cap and interface with 10^5 Halton
    samples each, the 401 x 401 slice sampled, global transmission coefficient."""
    cfg = W.FocusedNormal()
    xd = oracle.sample_cap(cfg.xd_seed, cfg.n_xd, cfg.radius, cfg.curvature, (0.0, 0.0, 0.0), 0.0,
                           seq=oracle.SEQ_HALTON)
    q = oracle.sample_square(cfg.if_seed, cfg.n_if, 0.0, 0.0, cfg.water_path, cfg.half_width,
                             seq=oracle.SEQ_HALTON)
    tx, ty, tz = cfg.grid()
    rng = np.random.default_rng(2026)
    idx = np.sort(rng.choice(tx.size, n_samples, replace=False))
    t0 = time.time()
    phi = oracle.chain(xd, 1.0, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), [q], [cfg.water_path],
                       [m[0] for m in cfg.media], [m[1] for m in cfg.media],
                       (tx[idx], ty[idx], tz[idx]), [cfg.freq], oracle.T_GLOBAL)[0]
    return {
        "workload": "focused_normal", "seconds": time.time() - t0,
        "index": idx.tolist(), "re": phi.real.tolist(), "im": phi.imag.tolist(),
    }


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "one_interface"
    res = {"one_interface": one_interface, "layered_stack": layered_stack,
           "focused_normal": focused_normal}[which]()
    path = os.path.join(HERE, f"{which}_samples.json")
    with open(path, "w") as f:
        json.dump(res, f)
    print(f"wrote {path} in {res['seconds']:.0f} s")

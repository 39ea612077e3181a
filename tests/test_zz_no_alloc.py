"""rsi_propagate_noalloc (workspace in the library's fixed device array, no allocation)
against rsi_propagate_ex, through the C ABI: same tolerances as the parity tests
(rel-L2 <= 1e-4 FP32, <= 1e-10 FP64), two calls in a row with the second smaller, and a
launch whose split partials do not fit the array (fewer splits)."""
import ctypes as C

import numpy as np
import pytest

from paper_2408_06765_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {0: 1e-4, 1: 1e-10}


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _case(seed, ns, nt, kind):
    src = W.random_cloud(seed, ns, (0.0, 0.0, 0.0), (0.015, 0.015, 0.0 if kind == 1 else 0.002))
    tgt = W.random_cloud(seed + 1, nt, (0.005, 0.0, 0.02), (0.02, 0.01, 0.015))
    return (tuple(dev(v) for v in src), dev(W.random_weights(seed + 3, ns, 1e-4)),
            dev(W.random_complex(seed + 2, ns)), tuple(dev(v) for v in tgt))


def _both(gpu, case, kind, prec, flags=0):
    import torch
    src, w, s, tgt = case
    c, f = (5900.0, 5.0e6) if kind == 1 else (1480.0, 5.0e6)
    ref = gpu.rsi_propagate_ex(src, w, s, tgt, c, f, kind, prec, flags, normal=(0.0, 0.0, 1.0))
    out = torch.full_like(ref, float("nan"))
    gpu.rsi_propagate_noalloc(src, w, s, tgt, c, f, kind, prec, flags, out, normal=(0.0, 0.0, 1.0))
    torch.cuda.synchronize()
    return out.cpu().numpy(), ref.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind", [0, 1, 2])
def test_noalloc_matches_propagate_two_calls(gpu, kind, prec):
    # first call: 70001 sources onto 3001 points (split sources); second, smaller: 1000
    # onto 37 (the few-point FP32 launch), so stale contents of the array must not matter
    for seed, ns, nt in ((11, 70001, 3001), (12, 1000, 37)):
        got, ref = _both(gpu, _case(seed, ns, nt, kind), kind, prec)
        assert np.all(np.isfinite(got.view(np.float64 if prec else np.float32)))
        assert rel(got, ref) <= TOL[prec], (kind, prec, ns, nt, rel(got, ref))


def test_noalloc_partials_beyond_the_array(gpu):
    """2^18 planar dipole sources onto 2^18 points: rsi_propagate_ex's 32 source splits
    would need 64 MiB of partials; the no-alloc call runs with as many splits as fit."""
    import torch
    n = 1 << 18
    src, w, s, _ = _case(21, n, 1, 1)
    src = (src[0], src[1], torch.zeros_like(src[2]))
    tgt = tuple(dev(v) for v in W.random_cloud(23, n, (0.0, 0.0, 0.02), (0.03, 0.0, 0.015)))
    for flags in (0, 1):
        got, ref = _both(gpu, (src, w, s, tgt), 1, 0, flags)
        assert rel(got, ref) <= TOL[0], (flags, rel(got, ref))


def test_noalloc_rejects_too_many_sources(gpu):
    from paper_2408_06765_amd import _lib as L
    import torch
    lib = L.load()
    x = torch.zeros(4, dtype=torch.float64, device="cuda")
    for prec, n in ((0, 2097041), (1, 1048573)):
        sp = L.rsi_points(x.data_ptr(), x.data_ptr(), x.data_ptr(), n)
        tp = L.rsi_points(x.data_ptr(), x.data_ptr(), x.data_ptr(), 4)
        st = lib.rsi_propagate_noalloc(C.byref(sp), x.data_ptr(), x.data_ptr(), None, C.byref(tp),
                                       L.rsi_medium(1480.0, 1000.0), 1e6, 0, prec, 0, x.data_ptr(), None)
        assert st == 3
        assert b"sources need" in lib.rsi_last_error()

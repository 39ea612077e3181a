"""The learned surrogate: its FP64 reference pinned on the CPU, and the GPU kernels
(bf16 MFMA forward/backward, Adam, checkpoint, carrier) against that reference."""
import math
import os
import tempfile

import numpy as np
import pytest

from oracle import mlp_oracle as MO
from paper_2408_06765_amd import workloads as W


def tiny_net(seed, n_ff=4, width=6, depth=2):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n_ff, 5))
    Ws, bs, fan = [], [], 2 * n_ff
    for _ in range(depth):
        Ws.append(rng.standard_normal((width, fan)) / math.sqrt(fan))
        bs.append(0.1 * rng.standard_normal(width))
        fan = width
    return B, Ws, bs, rng.standard_normal((2, width)) / math.sqrt(width), 0.1 * rng.standard_normal(2)


# ------------------------------------------------------------------ reference pins (CPU)
def test_reference_gradients_match_finite_differences():
    """Pure FP64 (no rounding): analytic gradients of the reference = central differences."""
    B, Ws, bs, Wo, bo = tiny_net(0)
    net = MO.MLPOracle(B, Ws, bs, Wo, bo, emulate_bf16=False)
    rng = np.random.default_rng(1)
    v = rng.uniform(-1, 1, (7, 5))
    t = rng.standard_normal((7, 2))
    _, _, g = net.loss_and_grads(v, t)
    ga = net.flat_grads(g)
    p0 = net.flat()
    gn = np.zeros_like(p0)
    h = 1e-6
    for i in range(p0.size):
        for sgn in (1, -1):
            p = p0.copy()
            p[i] += sgn * h
            net.set_flat(p)
            gn[i] += sgn * net.loss_and_grads(v, t)[0] / (2 * h)
    net.set_flat(p0)
    assert np.max(np.abs(ga - gn)) < 1e-7 * max(1.0, np.max(np.abs(ga)))


def test_bf16_rounding_is_nearest_even():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -2.5, 3.0e38, 1e-40])
    r = MO.bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                       # tie -> even mantissa
    assert r[2] == 1 + 2 ** -6               # tie -> even mantissa (upwards)
    assert r[3] == 1 + 2 ** -7               # above the tie -> up
    assert r[4] == -2.5
    assert np.isfinite(r[5]) and abs(r[5] / 3.0e38 - 1) < 2 ** -8
    assert r[6] == 2.0 ** -133              # subnormal: nearest multiple of 2^-133


def test_adam_first_step_is_sign_step():
    """Bias-corrected Adam moves every parameter by lr * g / (|g| + eps) on step 1."""
    p = np.array([0.5, -1.0, 2.0])
    g = np.array([1e-3, -4.0, 0.0])
    p1, m, v = MO.adam_step(p, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def _adam_broken_exponent(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam with the bias correction of step t taken at t - 1 (a plausible slip), used to
    show that the pins below fail for it."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** max(step - 1, 1))
    vh = v / (1 - beta2 ** max(step - 1, 1))
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def _adam_swapped_betas(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam with the two decay rates exchanged (a plausible slip)."""
    return MO.adam_step(p, g, m, v, step, lr, beta2, beta1, eps)


def _run_adam(step_fn, p0, grads, lr, **kw):
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    out = []
    for k, g in enumerate(grads, start=1):
        p, m, v = step_fn(p, g, m, v, k, lr, **kw)
        out.append(p.copy())
    return out


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are exactly g and g^2 at every
    step (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so step t moves each parameter by
    lr g / (|g| + eps): after t steps p0 - t lr g / (|g| + eps).  This pins the bias
    correction's exponents; the same closed form fails for a correction taken one step
    late."""
    p0 = np.array([0.5, -1.0, 2.0, 0.0])
    g = np.array([3e-3, -4.0, 0.25, 1e-6])
    lr = 0.01
    grads = [g] * 6
    expect = [p0 - t * lr * g / (np.abs(g) + 1e-8) for t in range(1, 7)]
    for got, want in zip(_run_adam(MO.adam_step, p0, grads, lr), expect):
        assert np.allclose(got, want, rtol=1e-12, atol=1e-14)
    bad = _run_adam(_adam_broken_exponent, p0, grads, lr)
    assert not np.allclose(bad[3], expect[3], rtol=1e-6, atol=1e-9)


def test_adam_three_steps_hand_expanded():
    """Three different gradients g1, g2, g3 with decay rates b1 = 0.8, b2 = 0.95: the
    moments written out as explicit sums (no recursion),
        m_t = (1 - b1) sum_{s<=t} b1^(t-s) g_s,   v_t = (1 - b2) sum_{s<=t} b2^(t-s) g_s^2,
    and p_3 = p0 - lr sum_t (m_t / (1 - b1^t)) / (sqrt(v_t / (1 - b2^t)) + eps).  This pins
    b1 and b2 (it fails with the two rates exchanged) and the order of the terms."""
    b1, b2, eps, lr = 0.8, 0.95, 1e-8, 0.003
    p0 = np.array([0.1, -0.2, 0.3])
    gs = [np.array([1.0, -2.0, 0.5]), np.array([-3.0, 0.5, 0.25]), np.array([2.0, 4.0, -1.0])]
    moves = np.zeros(3)
    for t in (1, 2, 3):
        m = (1 - b1) * sum(b1 ** (t - s) * gs[s - 1] for s in range(1, t + 1))
        v = (1 - b2) * sum(b2 ** (t - s) * gs[s - 1] ** 2 for s in range(1, t + 1))
        moves += (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    want = p0 - lr * moves
    got = _run_adam(MO.adam_step, p0, gs, lr, beta1=b1, beta2=b2, eps=eps)[-1]
    assert np.allclose(got, want, rtol=1e-13, atol=1e-15)
    swapped = _run_adam(_adam_swapped_betas, p0, gs, lr, beta1=b1, beta2=b2, eps=eps)[-1]
    assert not np.allclose(swapped, want, rtol=1e-6)
    late = _run_adam(_adam_broken_exponent, p0, gs, lr, beta1=b1, beta2=b2, eps=eps)[-1]
    assert not np.allclose(late, want, rtol=1e-6)


# ------------------------------------------------------------------ one exact layer
def _ambiguous(x, delta=2.0 ** -20):
    """Elements whose bf16 rounding could flip under a relative change of delta (FP32
    rounding between two correct implementations): bf16(x (1 - d)) != bf16(x (1 + d))."""
    x = np.asarray(x, dtype=np.float64)
    return MO.bf16(x * (1 - delta)) != MO.bf16(x * (1 + delta))


def exact_layer_case(seed):
    """A one-hidden-layer network whose bf16 operands are the same on any correct
    implementation: box [0, 1]^5 with rows at its corners (v = +-1 exactly), Fourier
    matrix of quarter integers (u = B v a quarter integer: every feature is 0 or +-1),
    weights and biases on the 2^-10 grid with |k| < 256 (exact in bf16; z = W h0 + b is
    exact in FP32 whatever the summation order), targets on the same grid.  Returns None
    unless every pre-rounding value (silu(z) and the output gradient dz) is clear of
    bf16 rounding boundaries by more than 2^-20 relative."""
    rng = np.random.default_rng(seed)
    n_ff, width, n = 32, 64, 64
    B = rng.integers(-8, 9, (n_ff, 5)) / 4.0
    corners = ((np.arange(32)[:, None] >> np.arange(5)) & 1).astype(np.float64)
    q = np.concatenate([corners, corners[rng.permutation(32)]])[:n]
    W1 = rng.integers(-255, 256, (width, 2 * n_ff)) / 1024.0
    b1 = rng.integers(-255, 256, width) / 1024.0
    Wo = rng.integers(-255, 256, (2, width)) / 1024.0
    bo = rng.integers(-255, 256, 2) / 1024.0
    t = rng.integers(-255, 256, (n, 2)) / 1024.0
    o = MO.MLPOracle(B, [W1], [b1], Wo, bo)
    v = MO.normalise(q, np.zeros(5), np.ones(5))
    y, (hs, zs) = o.forward(v)
    if np.any(_ambiguous(MO.silu(zs[0]))):
        return None
    dy = (y - t) / n
    if np.any(_ambiguous((dy @ Wo) * MO.silu_grad(zs[0]))):
        return None
    flat = np.concatenate([W1.ravel(), b1, Wo.ravel(), bo])
    return dict(n_ff=n_ff, width=width, B=B, q=q, t=t, v=v, o=o, flat=flat, h0=hs[0], z=zs[0])


def find_exact_layer_case():
    for seed in range(1000):
        c = exact_layer_case(seed)
        if c is not None:
            return seed, c
    raise AssertionError("no exact case in 1000 seeds")


def test_exact_layer_case_is_exact():
    """The case's construction holds in the reference: features are 0 or +-1 (to FP64
    rounding), z lies on the 2^-10 grid, and no value the layer rounds to bf16 sits near
    a rounding boundary."""
    _, c = find_exact_layer_case()
    h0 = c["h0"]
    assert np.all((np.abs(h0) < 1e-13) | (np.abs(np.abs(h0) - 1) < 1e-13))
    assert np.allclose(c["z"] * 1024, np.round(c["z"] * 1024), atol=1e-9)


# ------------------------------------------------------------------ GPU vs reference
def _setup(gpu_ok, n_ff, width, depth, n, seed):
    import torch
    from paper_2408_06765_amd import surrogate as S
    box = W.SurrogateBox()
    lo, hi = S.lohi(box)
    B = S.fourier_matrix(n_ff, (12.0, 8.0, 3.0, 3.0, 3.0), seed)
    params = S.glorot_params(n_ff, width, depth, seed + 1)
    rng = np.random.default_rng(seed + 2)
    q = np.stack([rng.uniform(lo[c], hi[c], n) for c in range(5)], 1).astype(np.float32)
    t = rng.standard_normal((n, 2)).astype(np.float32)
    net = S.MLP(n_ff, width, depth, B, lo, hi, max(n, 64))
    net.set_params(params)
    # the reference sees the same float32 inputs and parameters
    v = MO.normalise(q.astype(np.float64), lo, hi)
    o = _oracle_from_flat(B, params, n_ff, width, depth)
    return net, o, torch.as_tensor(q, device="cuda"), torch.as_tensor(t, device="cuda"), v, t, params


def _oracle_from_flat(B, p, n_ff, width, depth, noise=None):
    Ws, bs, o, fan = [], [], 0, 2 * n_ff
    p = p.astype(np.float64)
    for _ in range(depth):
        Ws.append(p[o:o + width * fan].reshape(width, fan))
        o += width * fan
        bs.append(p[o:o + width])
        o += width
        fan = width
    Wo = p[o:o + 2 * width].reshape(2, width)
    o += 2 * width
    return MO.MLPOracle(B.astype(np.float64), Ws, bs, Wo, p[o:o + 2], noise=noise)


def flip_tolerance(B, params, n_ff, width, depth, v, t, what):
    """Parity bar for a bf16 network: 1e-3, or 3x the drift between the reference and the
    same reference with FP32-sized perturbations (2^-24 sqrt(fan-in)) before each bf16
    rounding, whichever is larger -- deep networks amplify rounding-boundary flips."""
    a = _oracle_from_flat(B, params, n_ff, width, depth)
    b = _oracle_from_flat(B, params, n_ff, width, depth,
                          noise=(np.random.default_rng(123), 2.0 ** -24 * math.sqrt(width)))
    if what == "y":
        d = rel(b.forward(v)[0], a.forward(v)[0])
    else:
        ga = a.flat_grads(a.loss_and_grads(v, t)[2])
        d = rel(b.flat_grads(b.loss_and_grads(v, t)[2]), ga)
    return max(1e-3, 3.0 * d)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


SHAPES = [(32, 64, 3, 300), (128, 256, 5, 1000)]


@pytest.mark.gpu
@pytest.mark.parametrize("n_ff,width,depth,n", SHAPES)
def test_mlp_forward_matches_reference(gpu, n_ff, width, depth, n):
    net, o, q, t, v, tn, params = _setup(gpu, n_ff, width, depth, n, 3)
    y = net.forward(q).cpu().numpy()
    yr, _ = o.forward(v)
    tol = flip_tolerance(net.B, params, n_ff, width, depth, v, tn.astype(np.float64), "y")
    assert rel(y, yr) <= tol, (rel(y, yr), tol)
    net.destroy()


@pytest.mark.gpu
@pytest.mark.parametrize("n_ff,width,depth,n", SHAPES + [(64, 128, 4, 129), (64, 256, 5, 65537), (32, 64, 1, 1),
                                                      (32, 128, 2, 7)])
def test_mlp_fused_forward_equals_layerwise(gpu, n_ff, width, depth, n, monkeypatch):
    """The fused inference kernel (one launch, activations in LDS) gives the bits of the
    layer-by-layer path (features, one GEMM per layer, head), ragged row counts included."""
    net, o, q, t, v, tn, params = _setup(gpu, n_ff, width, depth, n, 7)
    y_fused = net.forward(q).cpu().numpy()
    monkeypatch.setenv("RSI_MLP_FUSED", "0")
    y_layer = net.forward(q).cpu().numpy()
    assert np.array_equal(y_fused.view(np.uint32), y_layer.view(np.uint32))
    net.destroy()


@pytest.mark.gpu
@pytest.mark.parametrize("rows", ["32", "64", "128"])
@pytest.mark.parametrize("n_ff,width,depth,n", [(64, 256, 5, 1000), (32, 128, 2, 7), (32, 64, 3, 300)])
def test_mlp_fused_row_tiles_equal_layerwise(gpu, n_ff, width, depth, n, rows, monkeypatch):
    """Each row tile of the fused kernel (forced; by default the call's size picks it)
    gives the bits of the layer-by-layer path."""
    net, o, q, t, v, tn, params = _setup(gpu, n_ff, width, depth, n, 11)
    monkeypatch.setenv("RSI_MLP_FUSED_ROWS", rows)
    y_fused = net.forward(q).cpu().numpy()
    monkeypatch.setenv("RSI_MLP_FUSED", "0")
    y_layer = net.forward(q).cpu().numpy()
    assert np.array_equal(y_fused.view(np.uint32), y_layer.view(np.uint32))
    net.destroy()


# the weight-gradient kernel's four tile shapes: 64 x 64, 128 x 128 (SHAPES), 128 x 64 (first
# layer of width 256 on 64 features), 64 x 128 (first layer of width 64 on 128 features)
GRAD_SHAPES = SHAPES + [(32, 256, 2, 500), (64, 64, 2, 300)]


@pytest.mark.gpu
@pytest.mark.parametrize("n_ff,width,depth,n", GRAD_SHAPES)
def test_mlp_gradients_match_reference(gpu, n_ff, width, depth, n):
    net, o, q, t, v, tn, params = _setup(gpu, n_ff, width, depth, n, 4)
    g, loss = net.gradients(q, t)
    lr_, _, gr = o.loss_and_grads(v, tn.astype(np.float64))
    g = g.cpu().numpy()
    flat = o.flat_grads(gr)
    assert abs(float(loss.cpu()) / lr_ - 1) < 1e-3
    tol = flip_tolerance(net.B, params, n_ff, width, depth, v, tn.astype(np.float64), "g")
    assert rel(g, flat) <= tol, (rel(g, flat), tol)
    # every weight matrix on its own
    off = 0
    for l, Wl in enumerate(gr["Ws"]):
        assert rel(g[off:off + Wl.size], Wl.ravel()) <= tol, (l, rel(g[off:off + Wl.size], Wl.ravel()), tol)
        off += Wl.size + gr["bs"][l].size
    net.destroy()


@pytest.mark.gpu
def test_mlp_train_step_is_adam(gpu):
    net, o, q, t, v, tn, p0 = _setup(gpu, 32, 64, 3, 500, 5)
    net.train_step(q, t, 1e-3)
    p1 = net.get_params().astype(np.float64)
    _, _, gr = o.loss_and_grads(v, tn.astype(np.float64))
    g = o.flat_grads(gr)
    pr, _, _ = MO.adam_step(p0.astype(np.float64), g, 0.0, 0.0, 1, 1e-3)
    d_gpu, d_ref = p1 - p0, pr - p0
    # the first bias-corrected step is lr * g / (|g| + eps): a sign step, so compare where
    # the reference gradient clearly exceeds the GPU-vs-reference gradient error
    clear = np.abs(g) > 1e-2 * np.sqrt(np.mean(g * g))
    assert clear.mean() > 0.9
    assert rel(d_gpu[clear], d_ref[clear]) <= 1e-4
    assert np.max(np.abs(d_gpu)) <= 1e-3 * (1 + 1e-5)
    net.destroy()


@pytest.mark.gpu
def test_mlp_adam_steps_match_reference(gpu):
    """Four Adam steps on the GPU against the reference's Adam fed the same gradients (the
    GPU's own, read before each step with rsi_mlp_gradients, whose sums the training step's
    fused update reproduces bit for bit): the bias correction and both moment recursions
    past step 1."""
    net, o, q, t, v, tn, p0 = _setup(gpu, 32, 64, 3, 500, 5)
    p, m, vv = p0.astype(np.float64), 0.0, 0.0
    for k in range(1, 5):
        g, _ = net.gradients(q, t)
        g = g.cpu().numpy().astype(np.float64)
        net.train_step(q, t, 1e-3)
        p, m, vv = MO.adam_step(p, g, m, vv, k, 1e-3)
        got = net.get_params().astype(np.float64)
        assert rel(got - p0, p - p0) <= 2e-5, (k, rel(got - p0, p - p0))
    net.destroy()


@pytest.mark.gpu
@pytest.mark.parametrize("fused", ["1", "0"])
def test_mlp_one_layer_exact_operands(gpu, fused, monkeypatch):
    """One hidden layer (features -> bf16 MFMA GEMM + bias + SiLU -> head) on inputs whose
    bf16 operands are the same on both sides (see exact_layer_case): the forward output
    and every gradient block match the FP64 reference to 1e-5 -- the MFMA path held to
    FP32 accumulation error, without the rounding-flip allowance of deep networks."""
    import torch
    from paper_2408_06765_amd import surrogate as S
    monkeypatch.setenv("RSI_MLP_FUSED", fused)
    _, c = find_exact_layer_case()
    net = S.MLP(c["n_ff"], c["width"], 1, c["B"], np.zeros(5), np.ones(5), 64)
    net.set_params(c["flat"])
    qd = torch.as_tensor(c["q"].astype(np.float32), device="cuda")
    td = torch.as_tensor(c["t"].astype(np.float32), device="cuda")
    y = net.forward(qd).cpu().numpy()
    yr, _ = c["o"].forward(c["v"])
    assert rel(y, yr) <= 1e-5, rel(y, yr)
    g, loss = net.gradients(qd, td)
    lr_, _, gr = c["o"].loss_and_grads(c["v"], c["t"])
    g = g.cpu().numpy()
    assert abs(float(loss.cpu()) / lr_ - 1) <= 1e-5
    W, F = c["width"], 2 * c["n_ff"]
    blocks = [("W1", 0, W * F, gr["Ws"][0]), ("b1", W * F, W, gr["bs"][0]),
              ("Wo", W * F + W, 2 * W, gr["Wo"]), ("bo", W * F + 3 * W, 2, gr["bo"])]
    for name, off, size, ref in blocks:
        assert rel(g[off:off + size], np.ravel(ref)) <= 1e-5, (name, rel(g[off:off + size], np.ravel(ref)))
    net.destroy()


@pytest.mark.gpu
@pytest.mark.parametrize("n_ff,width,depth,n", [(32, 64, 3, 500), (128, 256, 3, 1000)])
def test_mlp_fused_adam_equals_separate_launches(gpu, n_ff, width, depth, n, monkeypatch):
    """The training step's Adam update, fused with the reductions that finish the gradients
    and with the bf16 weight casts, equals the separate launches (column sums, Adam, casts;
    RSI_MLP_ADAM_FUSED=0) bit for bit: the parameters after three steps, and what reads the
    three bf16 weight copies -- the fused and the layer-by-layer forward, and the gradients."""
    a, _, q, t, _, _, _ = _setup(gpu, n_ff, width, depth, n, 7)
    b, _, _, _, _, _, _ = _setup(gpu, n_ff, width, depth, n, 7)
    for _ in range(3):
        monkeypatch.setenv("RSI_MLP_ADAM_FUSED", "1")
        a.train_step(q, t, 1e-3)
        monkeypatch.setenv("RSI_MLP_ADAM_FUSED", "0")
        b.train_step(q, t, 1e-3)
    pa, pb = a.get_params(), b.get_params()
    assert np.array_equal(pa.view(np.uint32), pb.view(np.uint32))
    for mode in ("1", "0"):
        monkeypatch.setenv("RSI_MLP_FUSED", mode)
        ya, yb = a.forward(q).cpu().numpy(), b.forward(q).cpu().numpy()
        assert np.array_equal(ya.view(np.uint32), yb.view(np.uint32)), mode
    ga, gb = a.gradients(q, t)[0].cpu().numpy(), b.gradients(q, t)[0].cpu().numpy()
    assert np.array_equal(ga.view(np.uint32), gb.view(np.uint32))
    a.destroy()
    b.destroy()


@pytest.mark.gpu
def test_mlp_checkpoint_resume_is_exact(gpu):
    import torch
    from paper_2408_06765_amd import surrogate as S
    net, o, q, t, v, tn, p0 = _setup(gpu, 32, 64, 3, 640, 6)
    for _ in range(6):
        net.train_step(q, t, 1e-3)
    straight = net.get_params()
    net.set_params(p0)
    for _ in range(3):
        net.train_step(q, t, 1e-3)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ckpt.bin")
        net.save(path)
        box = W.SurrogateBox()
        lo, hi = S.lohi(box)
        net2 = S.MLP(32, 64, 3, net.B, lo, hi, 640)
        net2.load(path)
        for _ in range(3):
            net2.train_step(q, t, 1e-3)
        resumed = net2.get_params()
        net2.destroy()
    assert np.array_equal(straight.view(np.uint32), resumed.view(np.uint32))
    net.destroy()


@pytest.mark.gpu
def test_carrier_phase_and_inverse(gpu):
    """The carrier is the refracted plane wave of the tilted piston: its phase gradient is
    (2 pi f sin(tilt)/c1) along x and (2 pi f cos(a2)/c2) along z below the interface,
    with sin(a2) = (c2/c1) sin(tilt) (Snell, eq. 15); modulate o demodulate = identity."""
    import torch
    from paper_2408_06765_amd import surrogate as S
    m1, m2 = W.WATER, W.STEEL_5900
    rng = np.random.default_rng(9)
    n, h = 64, 1e-6
    base = np.stack([rng.uniform(-0.01, 0.04, n), rng.uniform(0.002, 0.03, n), rng.uniform(1e6, 1e7, n),
                     rng.uniform(0.03, 0.07, n), rng.uniform(0.0, math.radians(14.0), n)], 1)
    qs = [base.copy(), base.copy(), base.copy()]
    qs[1][:, 0] += h
    qs[2][:, 1] += h
    one = torch.ones(n, dtype=torch.complex64, device="cuda")
    env = [S.rsi_surrogate_carrier(torch.as_tensor(q.astype(np.float32), device="cuda"), m1, m2, 0, one)
           .cpu().numpy().astype(np.complex128) for q in qs]
    qf = [q.astype(np.float32).astype(np.float64) for q in qs]
    for i in range(n):
        f, tilt = qf[0][i, 2], qf[0][i, 4]
        kx = 2 * math.pi * f * math.sin(tilt) / m1[0]
        s2 = m2[0] / m1[0] * math.sin(tilt)
        kz = 2 * math.pi * f * math.sqrt(1 - s2 * s2) / m2[0]
        # demodulation multiplies by e^{-i psi}: the phase decreases by k dx
        dpx = -np.angle(env[1][i] / env[0][i]) / (qf[1][i, 0] - qf[0][i, 0])
        dpz = -np.angle(env[2][i] / env[0][i]) / (qf[2][i, 1] - qf[0][i, 1])
        assert abs(dpx - kx) < 2e-3 * (abs(kx) + 1e3)
        assert abs(dpz - kz) < 2e-3 * kz
        assert abs(abs(env[0][i]) * m1[0] * m1[1] - 1) < 1e-6
    x = torch.as_tensor((rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64), device="cuda")
    qd = torch.as_tensor(base.astype(np.float32), device="cuda")
    back = S.rsi_surrogate_carrier(qd, m1, m2, 1, S.rsi_surrogate_carrier(qd, m1, m2, 0, x))
    assert rel(back.cpu().numpy(), x.cpu().numpy()) < 1e-6

"""Pins for the FP64 MLP reference: central finite differences of its backward
pass, torch's FP64 autograd (an independent library) on the same network,
bfloat16 rounding against torch's conversion, GELU special values, and Adam
against torch.optim.Adam."""
import math

import numpy as np
import torch

import oracle.mlp as om


def _data(rng, M=8):
    x = rng.normal(size=(M, 64))
    t = rng.normal(size=(M, 256))
    return x, t


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    theta = om.init_params(1) + rng.normal(scale=0.01, size=om.N_PARAMS)
    x, t = _data(rng)
    _, g = om.loss_and_grad(theta, x, t, bf16=False)
    idx = rng.choice(om.N_PARAMS, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(om.N_PARAMS)
        e[i] = h
        lp, _ = om.loss_and_grad(theta + e, x, t, bf16=False)
        lm, _ = om.loss_and_grad(theta - e, x, t, bf16=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_matches_torch_fp64_autograd():
    rng = np.random.default_rng(1)
    theta = om.init_params(2)
    x, t = _data(rng, 16)
    loss, g = om.loss_and_grad(theta, x, t, bf16=False)
    tt = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    parts, at = [], 0
    for o, i in om.SIZES:
        W = tt[at:at + o * i].view(o, i)
        at += o * i
        b = tt[at:at + o]
        at += o
        parts.append((W, b))
    a = torch.tensor(x, dtype=torch.float64)
    for li, (W, b) in enumerate(parts):
        a = a @ W.T + b
        if li < 3:
            a = torch.nn.functional.gelu(a)
    L = ((a - torch.tensor(t, dtype=torch.float64)) ** 2).mean()
    L.backward()
    assert abs(L.item() - loss) < 1e-12
    assert np.abs(tt.grad.numpy() - g).max() < 1e-12


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(2)
    v = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-5, 5, 5000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0]])
    ours = om.bf16_round(v)
    ref = torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)
    assert om.bf16_round(np.array([1.0 + 2 ** -8]))[0] == 1.0  # tie to even


def test_gelu_values():
    assert om.gelu(np.array([0.0]))[0] == 0.0
    assert abs(om.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15
    z = np.linspace(-6, 6, 101)
    ref = torch.nn.functional.gelu(torch.tensor(z)).numpy()
    assert np.abs(om.gelu(z) - ref).max() < 1e-12
    # derivative by central differences of the closed form
    h = 1e-6
    fd = (om.gelu(z + h) - om.gelu(z - h)) / (2 * h)
    assert np.abs(fd - om.gelu_grad(z)).max() < 1e-8
    assert abs(om.gelu(np.array([10.0]))[0] - 10.0) < 1e-12


def test_adam_matches_torch():
    rng = np.random.default_rng(3)
    theta = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    p = torch.tensor(theta.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        g = rng.normal(size=50)
        theta, m, v = om.adam_step(theta, m, v, g, step)
        p.grad = torch.tensor(g)
        opt.step()
    assert np.abs(p.detach().numpy() - theta).max() < 1e-12


def test_bf16_path_close_to_fp64_path():
    rng = np.random.default_rng(4)
    theta = om.init_params(5)
    x, t = _data(rng, 32)
    l1, g1 = om.loss_and_grad(theta, x, t, bf16=True)
    l0, g0 = om.loss_and_grad(theta, x, t, bf16=False)
    assert abs(l1 - l0) / l0 < 2e-2
    assert np.linalg.norm(g1 - g0) / np.linalg.norm(g0) < 5e-2
    assert math.isfinite(l1)


def _fp32_forward(theta, x):
    """An FP32 evaluation of the BF16 network written independently of the
    reference: float32 matrix products (BLAS sgemm accumulation order),
    float32 erf, BF16 rounding by torch's own conversion."""
    def bf(v):
        return torch.tensor(np.asarray(v, np.float32)).to(torch.bfloat16).to(torch.float32).numpy()
    from scipy.special import erf
    a = bf(x)
    at = 0
    for li, (o, i) in enumerate(om.SIZES):
        W = bf(theta[at:at + o * i].reshape(o, i))
        at += o * i
        b = np.asarray(theta[at:at + o], np.float32)
        at += o
        z = (a @ W.T + b).astype(np.float32)
        if li == 3:
            return z
        g = (np.float32(0.5) * z * (np.float32(1) + erf(z * np.float32(0.70710678)).astype(np.float32))).astype(np.float32)
        a = bf(g)


def test_forward_tolerance_holds_an_fp32_evaluation():
    """The element-wise bar of the GPU forward pass: one BF16 step at the
    output's scale, 2^-7 rms(y), per element.  Both sides round every hidden
    activation to BF16 at the same points; where an FP32 and the FP64 value
    straddle a rounding boundary the two round apart by one BF16 step, which
    moves the outputs by |w| ulp(a), far below the bar.  An independent FP32
    evaluation lands inside it on every element; a planted error of a few
    steps on one element does not."""
    rng = np.random.default_rng(7)
    for seed in (3, 4, 5):
        theta = om.init_params(seed) + rng.normal(scale=0.02, size=om.N_PARAMS)
        x = om.bf16_round(rng.normal(size=(256, 64)))
        y, _ = om.forward(theta, x, bf16=True)
        y32 = _fp32_forward(theta, x).astype(np.float64)
        tol = 2.0 ** -7 * float(np.sqrt(np.mean(y * y)))
        assert (np.abs(y32 - y) <= tol).all(), float(np.abs(y32 - y).max() / tol)
        bad = y32.copy()
        bad[3, 17] += 3 * tol
        assert (np.abs(bad - y) > tol).sum() == 1

"""Pins of the learned-closure oracle against independent library routines and closed forms."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp as M


def test_param_count():
    assert M.N_PARAMS == 9670
    p = M.init_params(7)
    assert p.shape == (9670,) and p.dtype == np.float32
    assert np.allclose(M.pack(M.unpack(p)), p)


def test_bf16_round_matches_torch_cast():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        # exact ties: 1 + 2^-8 rounds to 1, 1 + 3*2^-8 rounds to 1 + 2^-6
                        np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 0.0, -0.0])])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16_round(x32), ref)
    assert M.bf16_round(np.float32(1 + 2.0 ** -8)) == 1.0
    assert M.bf16_round(np.float32(1 + 3 * 2.0 ** -8)) == 1 + 2.0 ** -6
    assert np.isnan(M.bf16_round(np.float32(np.nan)))


def test_gelu_matches_torch():
    x = np.linspace(-8, 8, 1001)
    t = torch.from_numpy(x).requires_grad_(True)
    y = torch.nn.functional.gelu(t, approximate="tanh")
    y.sum().backward()
    assert np.allclose(M.gelu(x), y.detach().numpy(), rtol=1e-14, atol=1e-15)
    assert np.allclose(M.gelu_grad(x), t.grad.numpy(), rtol=1e-12, atol=1e-14)


def _torch_loss(params, x, y):
    layers = []
    o = 0
    for l in range(4):
        fi, fo = M.SIZES[l], M.SIZES[l + 1]
        W = params[o:o + fi * fo].view(fo, fi)
        o += fi * fo
        b = params[o:o + fo]
        o += fo
        layers.append((W, b))
    a = x
    for l, (W, b) in enumerate(layers):
        a = a @ W.T + b
        if l < 3:
            a = torch.nn.functional.gelu(a, approximate="tanh")
    return torch.mean((a - y) ** 2)


def test_backward_matches_autograd_fp64():
    rng = np.random.default_rng(4)
    p = M.init_params(3).astype(np.float64)
    x = rng.standard_normal((37, 14))
    y = rng.standard_normal((37, 6))
    loss, g = M.loss_and_grads(p, x, y, bf16=False)
    tp = torch.from_numpy(p.copy()).requires_grad_(True)
    tl = _torch_loss(tp, torch.from_numpy(x), torch.from_numpy(y))
    tl.backward()
    assert abs(loss - float(tl)) < 1e-14 * abs(loss)
    assert np.allclose(g, tp.grad.numpy(), rtol=1e-10, atol=1e-15)


def test_backward_central_differences():
    rng = np.random.default_rng(5)
    p = M.init_params(11).astype(np.float64)
    x = rng.standard_normal((16, 14))
    y = rng.standard_normal((16, 6))
    _, g = M.loss_and_grads(p, x, y, bf16=False)
    for idx in rng.choice(M.N_PARAMS, 40, replace=False):
        e = 1e-6
        pp = p.copy(); pp[idx] += e
        pm = p.copy(); pm[idx] -= e
        fd = (M.loss_and_grads(pp, x, y, bf16=False)[0] - M.loss_and_grads(pm, x, y, bf16=False)[0]) / (2 * e)
        assert abs(fd - g[idx]) <= 1e-6 * max(1e-3, abs(g[idx])) + 1e-10


def test_bf16_forward_quantisation_points():
    # With BF16 rounding the first layer equals the exact product of rounded operands.
    p = M.init_params(2).astype(np.float64)
    x = np.random.default_rng(0).standard_normal((5, 14))
    _, cache = M.forward(p, x)
    W1, b1 = M.unpack(p)[0]
    z1 = M.bf16_round(x) @ M.bf16_round(W1).T + b1
    assert np.allclose(cache["z"][0], z1, rtol=0, atol=0)
    assert np.array_equal(cache["a"][1], M.bf16_round(M.gelu(z1)))
    y_ex, _ = M.forward(p, x, bf16=False)
    y_bf, _ = M.forward(p, x)
    assert 0 < np.max(np.abs(y_bf - y_ex)) < 0.05


def test_adam_matches_torch():
    rng = np.random.default_rng(8)
    p0 = rng.standard_normal(50)
    grads = [rng.standard_normal(50) for _ in range(4)]
    tp = torch.nn.Parameter(torch.from_numpy(p0.copy()))
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for s, g in enumerate(grads, start=1):
        tp.grad = torch.from_numpy(g.copy())
        opt.step()
        p, m, v = M.adam(p, g, m, v, s)
    assert np.allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_feature_invariants():
    # pure strain g = diag(a, b, c): tr s^2 = a^2+b^2+c^2, tr s^3 = a^3+b^3+c^3, rotation terms 0
    a, b, c = 0.3, -0.1, -0.2
    f = M.features_from_grad(np.diag([a, b, c]), 1.0)
    assert np.allclose(f[:9], np.diag([a, b, c]).ravel())
    assert np.allclose(f[9:], [a * a + b * b + c * c, 0, a ** 3 + b ** 3 + c ** 3, 0, 0], atol=1e-16)
    # pure rotation about z with rate w: tr r^2 = -2 w^2
    w = 0.4
    g = np.array([[0, -w, 0], [w, 0, 0], [0, 0, 0]])
    f = M.features_from_grad(g, 2.0)
    assert np.allclose(f[9:], [0, -2 * (2 * w) ** 2, 0, 0, 0], atol=1e-15)
    # invariants are unchanged under a rotation of the frame g -> Q g Q^T
    rng = np.random.default_rng(1)
    g = rng.standard_normal((3, 3))
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    f1 = M.features_from_grad(g, 0.7)
    f2 = M.features_from_grad(Q @ g @ Q.T, 0.7)
    assert np.allclose(f1[9:], f2[9:], rtol=1e-12)
    # s r^2 mixes both parts: check one value by hand
    s = 0.5 * (g + g.T) * 0.7
    r = 0.5 * (g - g.T) * 0.7
    assert abs(f1[12] - np.trace(s @ r @ r)) < 1e-14
    assert abs(f1[13] - np.trace(s @ s @ r @ r)) < 1e-14


def test_infer_fallback():
    p = M.init_params(5)
    rng = np.random.default_rng(2)
    feats = rng.standard_normal((10, 14))
    feats[3, 2] = 50.0   # out of envelope
    feats[7, 0] = np.nan  # non-finite
    mu, sd = np.zeros(14), np.ones(14)
    lo, hi = -5 * np.ones(14), 5 * np.ones(14)
    tau_gm = rng.standard_normal((10, 6))
    rho = 1.0 + 0.1 * rng.random(10)
    tau, flag = M.infer(p, feats, rho, tau_gm, mu, sd, np.zeros(6), np.ones(6), lo, hi)
    assert flag.tolist() == [i in (3, 7) for i in range(10)]
    assert np.array_equal(tau[3], tau_gm[3]) and np.array_equal(tau[7], tau_gm[7])
    y, _ = M.forward(p, feats[:1])
    assert np.allclose(tau[0], rho[0] * y[0])


def test_norm_stats_population_std():
    """Column means and POPULATION standard deviations: the column 1, 2, 3, 4 has mean 5/2
    and std sqrt(5/4) (the sample std would be sqrt(5/3)); a constant column has std 0."""
    X = np.array([[1.0, 7.0], [2.0, 7.0], [3.0, 7.0], [4.0, 7.0]])
    mu, sd = M.norm_stats(X)
    assert mu[0] == 2.5 and mu[1] == 7.0
    assert abs(sd[0] - math.sqrt(1.25)) < 1e-15 and sd[1] == 0.0

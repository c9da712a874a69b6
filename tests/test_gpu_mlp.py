"""GPU parity of the learned closure (BF16 MFMA forward/backward, Adam, inference) against the
BF16-emulating FP64 oracle, through the C ABI; training gain over the gradient model.

Tolerances: the GPU accumulates in FP32 and the oracle in FP64, so an activation lying within
~1e-6 of a BF16 rounding boundary can round to the neighbouring BF16 value on one side only;
such flips change single activations by one BF16 step (2^-8 relative). Gradients are compared
per tensor as ||gpu - oracle||_F / ||oracle||_F <= 1e-3 (the gradient check of the
specification); outputs as max|gpu - oracle| / max|oracle| <= 1e-2, the worst single point,
where one flipped activation can shift an output by a few 1e-3, together with the RMS
relative error <= 1e-3; the exact-input Adam update to 1e-6. Every assertion carries the
measured error.
"""
import math
import os
import sys
import tempfile

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import fields as F  # noqa: E402
from oracle import mlp as M  # noqa: E402
from paper_2605_19796_amd import kcf, learned, synth  # noqa: E402

pytestmark = pytest.mark.gpu
TOL_OUT = 1e-2
TOL_GRAD = 1e-3
TOL_RMS = 1e-3
LAYERS = [("W1", 0, 896), ("b1", 896, 960), ("W2", 960, 5056), ("b2", 5056, 5120),
          ("W3", 5120, 9216), ("b3", 9216, 9280), ("W4", 9280, 9664), ("b4", 9664, 9670)]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = kcf.Context(0)
    yield c
    c.close()


def std32(x, mu, sd):
    """The GPU's float32 standardisation (x - mu) * (1/sd), reproduced exactly."""
    x = np.asarray(x, dtype=np.float32)
    inv = (np.float32(1.0) / np.asarray(sd, dtype=np.float32)).astype(np.float32)
    return ((x - np.asarray(mu, dtype=np.float32)).astype(np.float32) * inv).astype(np.float32)


def random_dataset(n, seed):
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal((n, 14)) * rng.uniform(0.1, 3.0, 14) + rng.uniform(-1, 1, 14)).astype(np.float32)
    y = (rng.standard_normal((n, 6)) * 0.5 + 0.2).astype(np.float32)
    return x, y


def make_mlp(ctx, seed, x, y):
    m = kcf.MLP(ctx)
    m.set_params(M.init_params(seed))
    m.fit_norm(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    return m


def test_norm_matches_host(ctx):
    say("[gpu] normalisation statistics")
    x, y = random_dataset(5000, 1)
    m = make_mlp(ctx, 1, x, y)
    nm = m.get_norm()
    mu, sd = M.norm_stats(x)
    assert np.allclose(nm[:14], mu, rtol=1e-6, atol=1e-7)
    assert np.allclose(nm[14:28], sd, rtol=1e-5)
    ymu, ysd = M.norm_stats(y)
    assert np.allclose(nm[28:34], ymu, rtol=1e-5, atol=1e-7) and np.allclose(nm[34:40], ysd, rtol=1e-5)
    assert np.allclose(nm[40:54], (x.min(0) - mu) / sd, rtol=1e-5)
    assert np.allclose(nm[54:68], (x.max(0) - mu) / sd, rtol=1e-5)
    m.close()


def test_forward_matches_oracle(ctx):
    say("[gpu] forward (predict) vs BF16-emulating oracle")
    x, y = random_dataset(4096 + 7, 2)
    m = make_mlp(ctx, 3, x, y)
    nm = m.get_norm()
    yg = m.predict(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    xs = std32(x, nm[:14], nm[14:28])
    yo, _ = M.forward(M.init_params(3), xs)
    err = np.max(np.abs(yg - yo)) / np.max(np.abs(yo))
    rms = np.sqrt(np.mean((yg - yo) ** 2) / np.mean(yo ** 2))
    say(f"[gpu]   forward rel err max {err:.2e} rms {rms:.2e}")
    assert err <= TOL_OUT, f"max relative error {err:.3e}"
    assert rms <= TOL_RMS, f"rms relative error {rms:.3e}"
    m.close()


@pytest.mark.parametrize("batch", [32, 96, 256, 4096, 65536])
def test_gradients_match_oracle(ctx, batch):
    say(f"[gpu] gradients vs oracle, batch {batch}")
    n = 3 * batch
    x, y = random_dataset(n, 4)
    m = make_mlp(ctx, 5, x, y)
    nm = m.get_norm()
    rng = np.random.default_rng(6)
    idx = rng.choice(n, batch, replace=False).astype(np.int32)
    loss, g = m.grads(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(),
                      torch.from_numpy(idx).cuda(), batch)
    xs = std32(x[idx], nm[:14], nm[14:28])
    ys = std32(y[idx], nm[28:34], nm[34:40])
    lo, go = M.loss_and_grads(M.init_params(5), xs, ys)
    assert abs(loss - lo) <= 1e-3 * lo, f"loss {loss} vs oracle {lo}"
    errs = {}
    for name, a, b in LAYERS:
        errs[name] = np.linalg.norm(g[a:b] - go[a:b]) / np.linalg.norm(go[a:b])
    say("[gpu]   rel Frobenius errors " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    m.close()
    for name, e in errs.items():
        assert e <= TOL_GRAD, f"batch {batch}: {name} relative Frobenius error {e:.3e}"


def test_grads_smaller_batch_more_partials(ctx):
    """A batch of 65 504 after one of 65 536 on the same network: its split-K pass has 2 047
    partials (the chunk is the largest power of two dividing the batch) against 256, so the
    training scratch must grow although the batch is smaller. Same gradients, bit for bit, as
    a network that only saw the smaller batch."""
    say("[gpu] gradient scratch: batch 65504 after 65536")
    n = 3 * 65536
    x, y = random_dataset(n, 11)
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    rng = np.random.default_rng(12)
    big = torch.from_numpy(rng.choice(n, 65536, replace=False).astype(np.int32)).cuda()
    small = torch.from_numpy(rng.choice(n, 65504, replace=False).astype(np.int32)).cuda()
    m1 = make_mlp(ctx, 5, x, y)
    m1.grads(xt, yt, big, 65536)
    l1, g1 = m1.grads(xt, yt, small, 65504)
    m2 = make_mlp(ctx, 5, x, y)
    l2, g2 = m2.grads(xt, yt, small, 65504)
    m1.close()
    m2.close()
    assert l1 == l2 and np.array_equal(g1, g2)


def test_out_of_memory_reported(ctx):
    """KCF_ENOMEM: with all but 1 GiB of device memory held by the caller, the training
    scratch of a batch of 2^22 (3.5 GB) cannot be allocated; the call returns KCF_ENOMEM
    and the network works as before once the memory is released."""
    say("[gpu] out-of-memory error path")
    n = 4096
    x, y = random_dataset(n, 13)
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    big = 1 << 22
    idx = torch.from_numpy(np.random.default_rng(14).integers(0, n, big).astype(np.int32)).cuda()
    m = make_mlp(ctx, 5, x, y)
    l0, g0 = m.grads(xt, yt, idx[:4096].contiguous(), 4096)
    torch.cuda.synchronize()
    free, _ = torch.cuda.mem_get_info()
    hold = torch.empty(free - (1 << 30), dtype=torch.uint8, device="cuda")
    try:
        with pytest.raises(kcf.KcfError) as e:
            m.grads(xt, yt, idx, big)
        assert e.value.code == -2, e.value  # KCF_ENOMEM
    finally:
        del hold
        torch.cuda.empty_cache()
    l1, g1 = m.grads(xt, yt, idx[:4096].contiguous(), 4096)
    m.close()
    assert l1 == l0 and np.array_equal(g1, g0)


def test_adam_step(ctx):
    say("[gpu] Adam update")
    x, y = random_dataset(1024, 7)
    m = make_mlp(ctx, 8, x, y)
    X, Y = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    p0 = m.get_params().astype(np.float64)
    _, g = m.grads(X, Y, None, 512)
    loss_buf = torch.zeros(1, device="cuda")
    m.train_step(X, Y, None, 512, 1e-3, loss_buf)
    torch.cuda.synchronize()
    p1 = m.get_params().astype(np.float64)
    po, mo, vo = M.adam(p0, g.astype(np.float64), np.zeros_like(p0), np.zeros_like(p0), 1, lr=1e-3)
    assert np.max(np.abs(p1 - po)) <= 1e-6 * max(1.0, np.max(np.abs(p0)))
    assert m.step_count() == 1
    assert float(loss_buf.item()) > 0
    # a second step: moments carried over
    _, g2 = m.grads(X, Y, None, 512)
    m.train_step(X, Y, None, 512, 1e-3)
    torch.cuda.synchronize()
    p2 = m.get_params().astype(np.float64)
    po2, _, _ = M.adam(po, g2.astype(np.float64), mo, vo, 2, lr=1e-3)
    assert np.max(np.abs(p2 - po2)) <= 2e-6 * max(1.0, np.max(np.abs(p0)))
    m.close()


def test_training_step_repacks_operands(ctx):
    """A training step rewrites the BF16 operand entries of every updated weight in its Adam
    launch: after a few steps the network predicts exactly what a network packed afresh from
    the same parameters and normalisation predicts."""
    say("[gpu] BF16 operands after training steps equal a fresh packing")
    x, y = random_dataset(4096, 21)
    X, Y = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    m1 = make_mlp(ctx, 22, x, y)
    for _ in range(3):
        m1.train_step(X, Y, None, 2048, 3e-3)
    torch.cuda.synchronize()
    m2 = kcf.MLP(ctx)
    m2.set_params(m1.get_params())
    m2.set_norm(m1.get_norm())
    p1 = m1.predict(X[:1024]).cpu().numpy()
    p2 = m2.predict(X[:1024]).cpu().numpy()
    m1.close()
    m2.close()
    assert np.array_equal(p1, p2)


def test_checkpoint_resume(ctx):
    say("[gpu] checkpoint save / load / resume")
    x, y = random_dataset(2048, 9)
    X, Y = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    m = make_mlp(ctx, 10, x, y)
    for _ in range(3):
        m.train_step(X, Y, None, 1024, 1e-3)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ck.bin")
        m.save(path)
        m2 = kcf.MLP(ctx)
        m2.load(path)
        assert np.array_equal(m.get_params(), m2.get_params())
        assert np.array_equal(m.get_norm(), m2.get_norm())
        assert m2.step_count() == 3
        m.train_step(X, Y, None, 1024, 1e-3)
        m2.train_step(X, Y, None, 1024, 1e-3)
        torch.cuda.synchronize()
        assert np.array_equal(m.get_params(), m2.get_params())
        raw = open(path, "rb").read()
        bad = bytearray(raw)
        bad[100] ^= 0x40
        open(path, "wb").write(bytes(bad))
        with pytest.raises(kcf.KcfError) as e:
            m2.load(path)
        assert e.value.code == kcf.EIO
        open(path, "wb").write(raw[:-10])
        with pytest.raises(kcf.KcfError) as e:
            m2.load(path)
        assert e.value.code == kcf.EIO
        with pytest.raises(kcf.KcfError) as e:
            m2.load(os.path.join(d, "missing.bin"))
        assert e.value.code == kcf.EIO
        m2.close()
    m.close()


def test_features_match_oracle(ctx):
    say("[gpu] feature builder vs oracle")
    n = 24
    h = 2 * math.pi / n
    rho, u = synth.workload_fields("c256_gauss8", n=n)
    o, st = learned.filtered_fields(ctx, rho.cuda(), u.cuda(), h, kcf.GAUSS, 4)
    X, Y = kcf.mlp_features(ctx, o["rho_bar"], o["ut"], o["tau"], h, 4 * h)
    ut = o["ut"].cpu().numpy().astype(np.float64)
    G = np.moveaxis(F.grad2(ut, h), (0, 1), (-2, -1)).reshape(-1, 3, 3)
    fo = M.features_from_grad(G, 4 * h)
    fg = X.cpu().numpy().astype(np.float64)
    for k in range(14):
        e = np.max(np.abs(fg[:, k] - fo[:, k])) / np.max(np.abs(fo[:, k]))
        assert e <= 1e-5, (k, e)
    tau = o["tau"].cpu().numpy().reshape(6, -1).T.astype(np.float64)
    yo = M.targets_from_tau(tau, o["rho_bar"].cpu().numpy().reshape(-1))
    assert np.max(np.abs(Y.cpu().numpy() - yo)) <= 1e-6 * np.max(np.abs(yo))


def test_inference_matches_oracle_and_fallback(ctx):
    say("[gpu] field inference vs oracle, with fallback")
    n = 32
    h = 2 * math.pi / n
    rho, u = synth.workload_fields("c256_gauss8", n=n)
    o, st = learned.filtered_fields(ctx, rho.cuda(), u.cuda(), h, kcf.GAUSS, 4,
                                    fields=("rho_bar", "ut", "tau", "tau_gm"))
    X, Y = kcf.mlp_features(ctx, o["rho_bar"], o["ut"], o["tau"], h, 4 * h)
    m = kcf.MLP(ctx)
    params = M.init_params(11)
    m.set_params(params)
    m.fit_norm(X, Y)
    nm = m.get_norm().copy()
    # shrink the envelope so that a good share of points falls back
    nm[40:54] = np.maximum(nm[40:54], -1.5)
    nm[54:68] = np.minimum(nm[54:68], 1.5)
    m.set_norm(nm)
    mask = torch.zeros((n ** 3 + 15) // 16, dtype=torch.int16, device="cuda")
    tau_l, nfb = m.infer_field(o["rho_bar"], o["ut"], h, 4 * h, st["m2"], mask_out=mask)
    torch.cuda.synchronize()
    ut = o["ut"].cpu().numpy().astype(np.float64)
    G = np.moveaxis(F.grad2(ut, h), (0, 1), (-2, -1)).reshape(-1, 3, 3)
    feats = X.cpu().numpy()  # the GPU's float32 features (pinned above against the oracle)
    xs = std32(feats, nm[:14], nm[14:28]).astype(np.float64)
    flag_o = ~np.all(np.isfinite(xs) & (xs >= nm[40:54]) & (xs <= nm[54:68]), axis=1)
    rb = o["rho_bar"].cpu().numpy().reshape(-1).astype(np.float64)
    gm = np.stack([rb * st["m2"] * np.einsum("pk,pk->p", G[:, i, :], G[:, j, :]) for (i, j) in F.PAIRS], 1)
    yo, _ = M.forward(params, np.where(np.isfinite(xs), xs, 0.0))
    tau_o = rb[:, None] * (nm[28:34] + nm[34:40] * yo)
    tau_o = np.where(flag_o[:, None], gm, tau_o)
    bits = mask.cpu().numpy().view(np.uint16)
    flag_g = ((bits[:, None] >> np.arange(16)) & 1).astype(bool).reshape(-1)[: n ** 3]
    assert nfb == int(flag_g.sum())
    assert 0.05 < flag_g.mean() < 0.95
    assert np.mean(flag_g != flag_o) <= 1e-4
    tg = tau_l.cpu().numpy().reshape(6, -1).T.astype(np.float64)
    same = flag_g == flag_o
    for c in range(6):
        e = np.max(np.abs(tg[same, c] - tau_o[same, c])) / np.max(np.abs(tau_o[:, c]))
        assert e <= TOL_OUT, (c, e)
        # fallback points carry the gradient model exactly (float32 evaluation)
        fb = same & flag_g
        assert np.max(np.abs(tg[fb, c] - gm[fb, c])) <= 1e-5 * np.max(np.abs(gm[:, c]))
    m.close()


def test_training_beats_gradient_model(ctx):
    say("[gpu] training on filtered fields; learned vs gradient model on a held-out field")
    n = 128
    h = 2 * math.pi / n
    train_fields = [tuple(t.cuda() for t in synth.workload_fields("c256_gauss8", n=n))]
    X, Y = learned.build_dataset(ctx, train_fields, h, widths=(4, 8))
    m = kcf.MLP(ctx)
    m.set_params(learned.init_params(7))
    m.fit_norm(X, Y)
    hist = learned.train(m, X, Y, steps=3000, batch=8192, lr=2e-3, lr_final=5e-5, seed=7,
                         loss_every=500)
    say(f"[gpu]   loss history {hist}")
    assert hist[-1][1] < 0.5 * hist[0][1]
    rho_t, u_t = (t.cuda() for t in synth.workload_fields("c256_heldout", n=n))
    res = learned.evaluate(ctx, m, rho_t, u_t, h, 8)
    say(f"[gpu]   held-out: r learned {res['r_learned_mean']:.4f} gm {res['r_gm_mean']:.4f}; "
        f"nrmse learned {res['nrmse_learned_mean']:.4f} gm {res['nrmse_gm_mean']:.4f}; "
        f"fallback {res['fallback']}/{res['n']}")
    assert res["r_learned_mean"] >= 0.9
    assert res["nrmse_learned_mean"] < res["nrmse_gm_mean"]
    # precision of the BF16 MFMA inference: the same trained network in FP64 without BF16
    # rounding (oracle), on held-out points inside the envelope, per tau component
    o, st = learned.filtered_fields(ctx, rho_t, u_t, h, kcf.GAUSS, 8)
    Xt, _ = kcf.mlp_features(ctx, o["rho_bar"], o["ut"], o["tau"], h, 8 * h)
    mask = torch.zeros((n ** 3 + 15) // 16, dtype=torch.int16, device="cuda")
    tau_l, _ = m.infer_field(o["rho_bar"], o["ut"], h, 8 * h, st["m2"], mask_out=mask)
    bits = mask.cpu().numpy().view(np.uint16)
    flag = ((bits[:, None] >> np.arange(16)) & 1).astype(bool).reshape(-1)[: n ** 3]
    rng = np.random.default_rng(5)
    idx = rng.choice(np.flatnonzero(~flag), 50000, replace=False)
    nm = m.get_norm()
    xs = std32(Xt.cpu().numpy()[idx], nm[:14], nm[14:28]).astype(np.float64)
    y64, _ = M.forward(m.get_params().astype(np.float64), xs, bf16=False)
    rb = o["rho_bar"].cpu().numpy().reshape(-1)[idx].astype(np.float64)
    t64 = rb[:, None] * (nm[28:34] + nm[34:40] * y64)
    tg = tau_l.cpu().numpy().reshape(6, -1)[:, idx].T.astype(np.float64)
    emax = np.max(np.abs(tg - t64), 0) / np.max(np.abs(t64), 0)
    erms = np.sqrt(np.mean((tg - t64) ** 2, 0) / np.mean(t64 ** 2, 0))
    say("[gpu]   BF16 inference vs FP64 network, per component (xx xy xz yy yz zz): max "
        + " ".join(f"{v:.2e}" for v in emax) + "; rms " + " ".join(f"{v:.2e}" for v in erms))
    assert np.all(erms <= 1e-2) and np.all(emax <= 2e-2)
    m.close()


def test_mlp_error_paths(ctx):
    say("[gpu] learned-closure error paths")
    m = kcf.MLP(ctx)
    X = torch.zeros((64, 14), device="cuda")
    Y = torch.zeros((64, 6), device="cuda")
    with pytest.raises(kcf.KcfError) as e:
        m.train_step(X, Y, None, 48, 1e-3)  # not a multiple of 32
    assert e.value.code == kcf.EINVAL
    with pytest.raises(kcf.KcfError) as e:
        m.train_step(X, Y, None, 32, -1.0)
    assert e.value.code == kcf.EINVAL
    bad = np.zeros(68, dtype=np.float32)
    with pytest.raises(kcf.KcfError) as e:
        m.set_norm(bad)  # zero scales
    assert e.value.code == kcf.EINVAL
    p = np.zeros(9670, dtype=np.float32)
    p[5] = np.nan
    with pytest.raises(kcf.KcfError) as e:
        m.set_params(p)
    assert e.value.code == kcf.EINVAL
    m.close()


def test_c1024_inference_sampled(ctx):
    """Learned inference over a 1024^3 field, the launch of the learned-vs-plain race
    (rho_bar, ut -> tau with the envelope fallback to the gradient model), against the oracle
    network at sampled points. The inputs are the synthetic 1024^3 density and velocity fields
    themselves (the network does not need them to be filtered), so nothing the oracle sees
    comes from the GPU: features, standardisation, envelope test and fallback at the sampled
    points come from the oracle's own central differences of the input velocity."""
    say("[gpu] 1024^3 learned inference: sampled parity")
    n = 1024
    h = 2 * math.pi / n
    delta = 8 * h
    w, _ = F.filter_weights(F.GAUSS, 8)
    m2 = F.second_moment(w, h)
    rho, u = synth.workload_fields("c1024_learned", device="cuda")
    rng = np.random.default_rng(21)
    pts = np.concatenate([np.array([[0, 0, 0], [n - 1, n - 1, n - 1], [n // 2, 7, n - 1]]),
                          rng.integers(0, n, (253, 3))])

    def grad_at(p):
        """(npts, 3, 3) central-difference gradients G[a, b] = d_b u_a at points p (k, j, i)."""
        k, j, i = (torch.as_tensor(p[:, c], device="cuda") for c in range(3))
        G = np.empty((len(p), 3, 3))
        for b, (dk, dj, di) in enumerate(((0, 0, 1), (0, 1, 0), (1, 0, 0))):
            kp, jp, ip = (k + dk) % n, (j + dj) % n, (i + di) % n
            km, jm, im = (k - dk) % n, (j - dj) % n, (i - di) % n
            up = u[:, kp, jp, ip].cpu().numpy().astype(np.float64)
            um = u[:, km, jm, im].cpu().numpy().astype(np.float64)
            G[:, :, b] = ((up - um) / (2 * h)).T
        return G

    # normalisation from oracle features of 20 000 random points; a +-3 envelope
    sample = rng.integers(0, n, (20000, 3))
    fs = M.features_from_grad(grad_at(sample), delta)
    mu, sd = M.norm_stats(fs)
    nm = np.concatenate([mu, sd, np.full(6, 2e-3), np.full(6, 1e-3), np.full(14, -3.0),
                         np.full(14, 3.0)]).astype(np.float32)
    params = M.init_params(11)
    m = kcf.MLP(ctx)
    m.set_params(params)
    m.set_norm(nm)
    mask = torch.zeros((n ** 3 + 15) // 16, dtype=torch.int16, device="cuda")
    tau, nfb = m.infer_field(rho, u, h, delta, m2, mask_out=mask)
    torch.cuda.synchronize()
    G = grad_at(pts)
    feats = M.features_from_grad(G, delta).astype(np.float32)
    xs = std32(feats, nm[:14], nm[14:28]).astype(np.float64)
    flag_o = ~np.all(np.isfinite(xs) & (xs >= nm[40:54]) & (xs <= nm[54:68]), axis=1)
    idx = torch.as_tensor(pts, device="cuda", dtype=torch.long)
    rb = rho[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy().astype(np.float64)
    gm = np.stack([rb * m2 * np.einsum("pk,pk->p", G[:, a, :], G[:, b, :]) for (a, b) in F.PAIRS], 1)
    yo, _ = M.forward(params, np.where(np.isfinite(xs), xs, 0.0))
    tau_o = np.where(flag_o[:, None], gm, rb[:, None] * (nm[28:34] + nm[34:40] * yo))
    flat = (idx[:, 0] * n + idx[:, 1]) * n + idx[:, 2]
    bits = mask.view(torch.int16).cpu().numpy().view(np.uint16)
    fl = flat.cpu().numpy()
    flag_g = ((bits[fl // 16] >> (fl % 16)) & 1).astype(bool)
    tg = tau[:, idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy().T.astype(np.float64)
    say(f"[gpu]   fallback points {nfb} of {n ** 3}; sampled flags differ at "
        f"{int(np.sum(flag_g != flag_o))} of {len(pts)}")
    assert 0 < nfb < n ** 3
    assert np.sum(flag_g != flag_o) <= 2
    same = flag_g == flag_o
    for c in range(6):
        e = np.max(np.abs(tg[same, c] - tau_o[same, c])) / np.max(np.abs(tau_o[same, c]))
        assert e <= TOL_OUT, f"component {c}: max relative error {e:.3e}"
    m.close()
    del rho, u, tau, mask
    torch.cuda.empty_cache()

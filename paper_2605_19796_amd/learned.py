"""Driver of the learned closure: dataset from filtered fields, training loop, evaluation.

Orchestration only: every arithmetic step (filtering, features, statistics, forward and
backward passes, Adam, inference) runs in libkcf. Random numbers the training draws are
handed to the library as inputs: the initial parameters come from a seeded numpy generator
on the host, the per-epoch sample order from a seeded torch generator on the device.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import kcf

N_PARAMS = 9670


def init_params(seed: int) -> np.ndarray:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases, layer by layer."""
    rng = np.random.default_rng(seed)
    sizes = (14, 64, 64, 64, 6)
    parts = []
    for l in range(4):
        fi, fo = sizes[l], sizes[l + 1]
        b = 1.0 / math.sqrt(fi)
        parts.append(rng.uniform(-b, b, (fo, fi)).ravel())
        parts.append(rng.uniform(-b, b, fo))
    return np.concatenate(parts).astype(np.float32)


def filtered_fields(ctx, rho, u, h, kind, n_delta, fields=("rho_bar", "ut", "tau")):
    n = rho.shape
    outs = [kcf.alloc_outputs(n, rho.device, fields)]
    st = ctx.filter_favre(rho, u, h, [(kind, n_delta)], outs)
    return outs[0], st[0]


def build_dataset(ctx, field_pairs, h, widths, kind=kcf.GAUSS):
    """Inputs and targets of every grid point of every field at every width (device)."""
    xs, ys = [], []
    for rho, u in field_pairs:
        for nd in widths:
            o, _ = filtered_fields(ctx, rho, u, h, kind, nd)
            x, y = kcf.mlp_features(ctx, o["rho_bar"], o["ut"], o["tau"], h, nd * h)
            xs.append(x)
            ys.append(y)
            del o
    return torch.cat(xs), torch.cat(ys)


def train(mlp, X, Y, steps, batch=65536, lr=1e-3, lr_final=1e-4, seed=7, loss_every=50,
          on_loss=None):
    """Minibatch Adam over the dataset; epochs draw a fresh permutation. Returns the loss
    history (step, loss) read back every `loss_every` steps."""
    n = X.shape[0]
    dev = X.device
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    losses = torch.zeros(steps, dtype=torch.float32, device=dev)
    per_epoch = max(n // batch, 1)
    perm = None
    hist = []
    for s in range(steps):
        e = s % per_epoch
        if e == 0:
            perm = torch.randperm(n, generator=gen, device=dev)[: per_epoch * batch].to(torch.int32)
        idx = perm[e * batch:(e + 1) * batch]
        frac = s / max(steps - 1, 1)
        cur = lr * (lr_final / lr) ** frac
        mlp.train_step(X, Y, idx, batch, cur, losses[s:s + 1])
        if s == 0 or (s + 1) % loss_every == 0 or s == steps - 1:
            v = float(losses[s].item())
            hist.append((s + 1, v))
            if on_loss:
                on_loss(s + 1, v)
    return hist


def pearson_gpu(ctx, a, b):
    """Pearson r of two device arrays via the library's FP64 reductions."""
    n = a.numel()
    sa, saa, sab = ctx.reduce_check(a.contiguous().view(-1), b.contiguous().view(-1))
    sb, sbb, _ = ctx.reduce_check(b.contiguous().view(-1))
    cov = sab - sa * sb / n
    va = saa - sa * sa / n
    vb = sbb - sb * sb / n
    return cov / math.sqrt(va * vb)


def nrmse_gpu(ctx, pred, ref):
    """sqrt(sum (pred-ref)^2 / sum (ref - mean ref)^2) with FP64 reductions."""
    d = (pred - ref).contiguous().view(-1)
    _, sdd, _ = ctx.reduce_check(d)
    sr, srr, _ = ctx.reduce_check(ref.contiguous().view(-1))
    n = ref.numel()
    return math.sqrt(sdd / (srr - sr * sr / n))


def evaluate(ctx, mlp, rho, u, h, n_delta, kind=kcf.GAUSS):
    """Per-component correlation and normalised RMSE of the learned tau and of the gradient
    model against the exact tau, on one field."""
    o, st = filtered_fields(ctx, rho, u, h, kind, n_delta,
                            fields=("rho_bar", "ut", "tau", "tau_gm"))
    m2 = st["m2"]
    tau_l, nfb = mlp.infer_field(o["rho_bar"], o["ut"], h, n_delta * h, m2)
    res = {"fallback": nfb, "n": int(rho.numel()), "r_learned": [], "r_gm": [],
           "nrmse_learned": [], "nrmse_gm": []}
    for c in range(6):
        res["r_learned"].append(pearson_gpu(ctx, tau_l[c], o["tau"][c]))
        res["r_gm"].append(pearson_gpu(ctx, o["tau_gm"][c], o["tau"][c]))
        res["nrmse_learned"].append(nrmse_gpu(ctx, tau_l[c], o["tau"][c]))
        res["nrmse_gm"].append(nrmse_gpu(ctx, o["tau_gm"][c], o["tau"][c]))
    for k in ("r_learned", "r_gm", "nrmse_learned", "nrmse_gm"):
        res[k + "_mean"] = float(np.mean(res[k]))
    return res

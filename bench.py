"""Throughput of the filtering path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: 512^3 periodic grid of synthetic spectral turbulence (u_rms 0.3, k0 16,
rho = 1 + 0.2 s), FP32 fields resident in HBM; one step = one fused pass computing four
box-filter widths (2h, 4h, 8h, 16h): products, separable periodic filter, Favre velocity,
SGS stress tau (all written), central-difference gradient, gradient-model and Smagorinsky
closures and kinetic-closure scalars (on chip), FP64 statistics per width (SGS dissipation,
tau-closure correlations) read back to the host, plus the input's E_k and enstrophy.

Prints one JSON line. `value` is grid points per second (each point filtered at all four
widths). `roofline` is for the fused filter kernel: algorithmic bytes (inputs 16 B +
outputs 4 x 40 B per point) over its HIP-event time on the stream it runs on.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_POINT = 16 + 4 * 40  # read rho,u; write rho_bar, ut, tau per width
KERNEL = "k_filter_box4"
WIDTHS = (2, 4, 8, 16)


def kernel_source_hash():
    p = os.path.join(ROOT, "paper_2605_19796_amd", "csrc", "kcf_filter.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def load_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source; otherwise None."""
    p = os.path.join(ROOT, "profiles", "k_filter_box4_512_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(rho, u, n_sub=96):
    """The FP64 oracle on a 96^3 periodic sub-cube of the same field, four widths."""
    import numpy as np
    from oracle import fields as F
    r = rho[:n_sub, :n_sub, :n_sub].cpu().numpy()
    uu = u[:, :n_sub, :n_sub, :n_sub].cpu().numpy()
    h = 2 * math.pi / rho.shape[0]
    t0 = time.perf_counter()
    for nd in WIDTHS:
        F.full_path(r, uu, F.BOX, nd, h)
    dt = time.perf_counter() - t0
    return dict(value=n_sub ** 3 / dt, unit="points/s", cores=1, kind="oracle",
                sample=f"numpy FP64 oracle, full path at 4 box widths on a {n_sub}^3 periodic "
                       f"sub-cube of the 512^3 field ({dt:.1f} s, single thread)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the filtering path here is a single-GPU build "
              "(see DESIGN.md for how it would shard); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_19796_amd import kcf, synth

    n = args.n
    h = 2 * math.pi / n
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    rho, u = synth.workload_fields("c512_box_multi", device=dev, n=n)
    filters = [(kcf.BOX, w) for w in WIDTHS]
    outs = [kcf.alloc_outputs((n, n, n), dev, ("rho_bar", "ut", "tau")) for _ in filters]
    ctx = kcf.Context(0)

    def step():
        st = ctx.filter_favre(rho, u, h, filters, outs)
        ist = ctx.input_stats(rho, u, h)
        return st, ist

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.enable_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, ist = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms, launches = ctx.kernel_ms()
    ctx.enable_timing(False)

    ms_step = (t1 - t0) * 1e3 / args.steps
    pts = float(n) ** 3
    value = pts / (ms_step * 1e-3)
    k_avg_ms = kms / max(launches, 1)
    achieved = BYTES_PER_POINT * pts / (k_avg_ms * 1e-3) / 1e9
    traffic = load_traffic()
    line = {
        "metric": "filtered grid points/s (% HBM roofline); learned vs plain closure at fixed error",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{n}^3 periodic spectral turbulence, box filter widths 2h/4h/8h/16h in one "
                        "fused pass, FP32 fields, FP64 on-GPU statistics",
            "grid": n, "filter": "box", "widths_h": list(WIDTHS), "k0": 16 * n / 512,
            "u_rms": 0.3, "rho_amp": 0.2, "seeds": [1004, 2004],
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": KERNEL, "kernel_ms": k_avg_ms, "bytes_per_point": BYTES_PER_POINT,
        },
        "stats": {
            f"{w}h": {"pi": s["pi"], "pi_gm": s["pi_gm"], "corr_tau_gm": s["corr_tau_gm"],
                      "corr_pi": s["corr_pi"]} for w, s in zip(WIDTHS, st)
        },
        "input": ist,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(rho, u)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Throughput of the filtering path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-learned]
                    [--no-carrier] [--no-lbm] [--no-c2] [--oracle-ladder]

Workload: 512^3 periodic grid of synthetic spectral turbulence (u_rms 0.3, k0 16,
rho = 1 + 0.2 s), FP32 fields resident in HBM; one step = four box-filter widths (2h, 4h,
8h, 16h) in one call, every width computing: products, separable periodic filter, Favre
velocity, SGS stress tau (all written), central-difference gradient, gradient-model and
Smagorinsky closures (on chip), FP64 statistics per width (SGS dissipation, tau-closure
correlations) read back to the host; plus the input's E_k and enstrophy.

Prints one JSON line. `value` is grid points per second (each point filtered at all four
widths). `roofline` is for the kernel with the largest share of the step: the algorithmic
bytes of the four-width step, 176 B per point (inputs 16 B once, 40 B of outputs per width),
spread over its four launches (44 B per point each), over that kernel's average HIP-event
time on the stream it runs on; `roofline.step` gives the same 176 B per point over the summed
kernel time of the step, and `stream_ceiling` the time of a plain streaming kernel that reads
4 and writes 40 fields of the same size (the practical HBM floor of the step on the device).

Further sections of the same line: `c2`, the 256^3 Gaussian-8h call with the full output set;
`carrier`, the a priori D3Q27 SGS carrier; `moment3`, the third-order SGS moment and the Favre
temperature; `kc_mp`, the a priori KC-MP SGS moment and relaxation-rate field; `lbm`, the D3Q27
collide-and-stream step of the Taylor-Green vortex with the kinetic closures; `learned`,
training and the learned-vs-plain race.

`cpu_baseline` times the FP64 oracle on the host cores on a bounded sample of the 512^3 step;
`oracle_ladder` times it at the configurations' own sizes (full path at 32^3 and 128^3,
sampled points at 512^3 and 1024^3); --oracle-ladder adds 256^3 and 2^16 sampled points
(several minutes of CPU work).

Profiling modes (for rocprofv3 runs): --profile-run times a few steps and skips the CPU
baseline and the learned section; --copy-calibration runs only a plain device copy of known
size, against which the HBM byte counters are scaled.
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
WIDTHS = (2, 4, 8, 16)
BYTES_STEP = 16 + 40 * len(WIDTHS)  # read rho, u once; write rho_bar, ut, tau per width
BYTES_PER_LAUNCH = BYTES_STEP / len(WIDTHS)  # the step's bytes spread over its four launches
# kernel instance each width launches in the timed step (radius n/2; FP64 sums up to 4h;
# Favre fields and statistics, no optional gradient-epilogue outputs)
KERNELS = {2: "k_box1<1, double, 0>", 4: "k_box1<2, double, 0>",
           8: "k_box1<4, float, 0>", 16: "k_box1<8, float, 0>"}
KERNEL_SOURCES = ("kcf_box.hip", "kcf_device.h", "kcf_internal.h")
COPY_BYTES = 1 << 31  # plain copy for counter calibration: 2 GiB read, 2 GiB written


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2605_19796_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_file(kernel):
    tag = kernel.replace("<", "_").replace(">", "").replace(", ", "_").replace(" ", "")
    return os.path.join(ROOT, "profiles", f"{tag}_512_traffic.json")


def load_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; otherwise None."""
    p = traffic_file(kernel)
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def _oracle_worker(job):
    """One process of the CPU baseline: the FP64 oracle's full path at every width on one
    periodic sub-cube (run with one numpy thread)."""
    import time as _t
    from oracle import fields as F
    r, uu, h = job
    t0 = _t.perf_counter()
    for nd in WIDTHS:
        F.full_path(r, uu, F.BOX, nd, h)
    return _t.perf_counter() - t0


def cpu_baseline(rho, u, n_sub=128):
    """The FP64 oracle on the host cores: one 128^3 periodic sub-cube of the field per process,
    every process running the full path at the four widths; points/s = processes x 128^3 /
    wall time. Processes: the host's cores, at most 16 (the CPU share of one GPU)."""
    import multiprocessing as mp
    nproc = max(1, min(os.cpu_count() or 1, 16))
    n = rho.shape[0]
    h = 2 * math.pi / n
    jobs = []
    for p in range(nproc):
        z0 = (p * n_sub) % (n - n_sub + 1)
        y0 = ((p // 4) * n_sub) % (n - n_sub + 1)
        jobs.append((rho[z0:z0 + n_sub, y0:y0 + n_sub, :n_sub].cpu().numpy().copy(),
                     u[:, z0:z0 + n_sub, y0:y0 + n_sub, :n_sub].cpu().numpy().copy(), h))
    env_old = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "1"  # inherited by the spawned workers
    try:
        ctx = mp.get_context("spawn")
        t0 = time.perf_counter()
        with ctx.Pool(nproc) as pool:
            per = pool.map(_oracle_worker, jobs)
        dt = time.perf_counter() - t0
    finally:
        if env_old is None:
            os.environ.pop("OMP_NUM_THREADS", None)
        else:
            os.environ["OMP_NUM_THREADS"] = env_old
    return dict(value=nproc * n_sub ** 3 / dt, unit="points/s", cores=nproc, kind="oracle",
                sample=f"numpy FP64 oracle, full path at the 4 box widths on one {n_sub}^3 periodic "
                       f"sub-cube of the 512^3 field per process, {nproc} processes of one thread "
                       f"({dt:.1f} s wall, {max(per):.1f} s slowest process)")


def _ladder_full_worker(job):
    """One process of the oracle ladder's full-field mode: the named workload's fields at n^3
    synthesised on the CPU (untimed), then the oracle's full path at one filter (timed, one
    thread)."""
    import time as _t
    import torch
    torch.set_num_threads(1)
    from oracle import fields as F
    from paper_2605_19796_amd import synth
    name, n, kind, nd = job
    r, uu = synth.workload_fields(name, device="cpu", n=n)
    r, uu = r.double().numpy(), uu.double().numpy()
    h = 2 * math.pi / n
    # the steps of the oracle's full path, timed together, with a line after each so that a
    # long run reports its progress
    t0 = _t.perf_counter()
    w, _ = F.filter_weights(kind, nd)
    rho_bar, ut, tau = F.filter_favre(r, uu, w)
    t1 = _t.perf_counter()
    if n >= 256:
        print(f"[bench] oracle ladder: {n}^3 filter and Favre fields in {t1 - t0:.1f} s",
              file=sys.stderr, flush=True)
    G = F.grad2(ut, h)
    cl = F.closures(rho_bar, G, tau, nd * h, F.second_moment(w, h))
    F.width_stats(rho_bar, ut, tau, G, cl["tau_gm"])
    dt = _t.perf_counter() - t0
    print(f"[bench] oracle ladder: {n}^3 full path done in {dt:.1f} s", file=sys.stderr, flush=True)
    return dt


def _ladder_sampled_worker(job):
    """One process of the oracle ladder's sampled mode: the oracle's direct 3-D sums at each
    point, given the point's periodic neighbourhood cube (2R + 3 cells wide, the point at its
    centre: the sums and the centred gradient then index the cube exactly as they would the
    whole field)."""
    import time as _t
    from oracle import fields as F
    cubes_r, cubes_u, kind, nd, h = job
    c = cubes_r.shape[1] // 2
    t0 = _t.perf_counter()
    for p in range(cubes_r.shape[0]):
        F.sampled_points(cubes_r[p], cubes_u[p], kind, nd, h, [(c, c, c)])
    return _t.perf_counter() - t0


def _neighbourhoods(rho, u, R, npts, seed):
    """npts random points of a periodic field (torch, on the GPU) and their (2R+3)^3 cubes,
    gathered on the GPU and returned as float32 numpy arrays."""
    import torch
    n = rho.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    pts = torch.randint(0, n, (npts, 3), generator=g).to(rho.device)
    offs = torch.arange(-(R + 1), R + 2, device=rho.device)
    kz = (pts[:, 0, None] + offs) % n
    jy = (pts[:, 1, None] + offs) % n
    ix = (pts[:, 2, None] + offs) % n
    flat = (kz[:, :, None, None] * n + jy[:, None, :, None]) * n + ix[:, None, None, :]
    cr = rho.reshape(-1)[flat].cpu().numpy()
    cu = torch.stack([u[a].reshape(-1)[flat] for a in range(3)], dim=1).cpu().numpy()
    return cr, cu


def oracle_ladder(full: bool):
    """The FP64 oracle timed on the host cores at the configurations' own sizes: the full-field
    path at 32^3 (box 4h), 128^3 and 256^3 (Gaussian 8h), on one process of one thread and on
    P processes of one thread each (P = host cores, at most 16), and the sampled-point mode
    (direct 3-D sums) at 512^3 (box 16h) and 1024^3 (Gaussian 8h) on random points split over
    P processes. The default run takes 32^3 and 128^3 (the latter on P processes only) and 256
    sampled points per grid; `full` adds 128^3 alone, 256^3 and 2^16 sampled points."""
    import multiprocessing as mp
    import torch
    from oracle import fields as F
    from paper_2605_19796_amd import synth
    nproc = max(1, min(os.cpu_count() or 1, 16))
    ctx = mp.get_context("spawn")
    out = []
    env_old = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "1"  # inherited by the spawned workers
    try:
        cases = [("c32_box4", 32, F.BOX, 4), ("c256_gauss8", 128, F.GAUSS, 8)]
        if full:
            cases.append(("c256_gauss8", 256, F.GAUSS, 8))
        with ctx.Pool(nproc) as pool:
            for name, n, kind, nd in cases:
                rec = dict(mode="full", grid=n, filter=f"{'box' if kind == F.BOX else 'gauss'} {nd}h")
                if full or n <= 32:  # one process alone (the default run takes the per-process
                    progress(f"oracle ladder: {n}^3 full path, 1 process")  # times below)
                    one = pool.map(_ladder_full_worker, [(name, n, kind, nd)])[0]
                    rec.update(one_process_s=one, one_process_points_per_s=n ** 3 / one)
                # the 256^3 path holds ~7 GB per process
                p = nproc if n <= 128 else min(nproc, 8)
                progress(f"oracle ladder: {n}^3 full path, {p} processes")
                t0 = time.perf_counter()
                per = pool.map(_ladder_full_worker, [(name, n, kind, nd)] * p)
                wall = time.perf_counter() - t0
                rec.update(processes=p, wall_s=wall, points_per_s=p * n ** 3 / wall,
                           slowest_process_s=max(per), fastest_process_s=min(per))
                out.append(rec)
            npts = 1 << 16 if full else 256
            for name, n, kind, nd in [("c512_box_multi", 512, F.BOX, 16),
                                      ("c1024_learned", 1024, F.GAUSS, 8)]:
                progress(f"oracle ladder: {n}^3 sampled mode, {npts} points")
                rho, u = synth.workload_fields(name, device="cuda")
                R = F.filter_weights(kind, nd)[1]
                chunk = max(1, npts // (4 * nproc))
                jobs = []
                for s in range(0, npts, chunk):
                    cr, cu = _neighbourhoods(rho, u, R, min(chunk, npts - s), seed=n + s)
                    jobs.append((cr, cu, kind, nd, 2 * math.pi / n))
                del rho, u
                torch.cuda.empty_cache()
                t0 = time.perf_counter()
                per = pool.map(_ladder_sampled_worker, jobs)
                wall = time.perf_counter() - t0
                out.append(dict(mode="sampled", grid=n, filter=f"{'box' if kind == F.BOX else 'gauss'} "
                                f"{nd}h", points=npts, processes=nproc, wall_s=wall,
                                points_per_s=npts / wall,
                                one_thread_points_per_s=npts / sum(per)))
    finally:
        if env_old is None:
            os.environ.pop("OMP_NUM_THREADS", None)
        else:
            os.environ["OMP_NUM_THREADS"] = env_old
    return dict(kind="oracle", cores=nproc, threads_per_process=1, runs=out)


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _timed(fn, reps, warm=1):
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def learned_section(ctx, args):
    """Training on 256^3 Gaussian-filtered fields (widths 4h, 8h; batch 65536), then the
    learned closure against the exact explicit-filter path on a 1024^3 field (Gaussian 8h)."""
    import torch
    from paper_2605_19796_amd import kcf, learned, synth
    dev = torch.device("cuda", 0)
    out = {}
    n_tr = 256
    h_tr = 2 * math.pi / n_tr
    progress("learned: building the 256^3 training set")
    rho, u = synth.workload_fields("c256_gauss8", device=dev)
    X, Y = learned.build_dataset(ctx, [(rho, u)], h_tr, widths=(4, 8))
    del rho, u
    mlp = kcf.MLP(ctx)
    mlp.set_params(learned.init_params(7))
    mlp.fit_norm(X, Y)
    batch = 65536
    progress(f"learned: training {args.train_steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = learned.train(mlp, X, Y, steps=args.train_steps, batch=batch, lr=2e-3, lr_final=5e-5,
                         seed=7, loss_every=max(args.train_steps // 6, 1))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    out["training"] = {
        "workload": "256^3 Gaussian-filtered fields at 4h and 8h, 33.5M samples, batch 65536, Adam",
        "samples": int(X.shape[0]), "steps": args.train_steps,
        "ms_per_step": t_train * 1e3 / args.train_steps,
        "samples_per_s": args.train_steps * batch / t_train,
        "loss_history": hist,
    }
    del X, Y
    rho_v, u_v = synth.workload_fields("c256_heldout", device=dev)
    ev = learned.evaluate(ctx, mlp, rho_v, u_v, h_tr, 8)
    out["heldout_256"] = {k: ev[k] for k in ("r_learned_mean", "r_gm_mean", "nrmse_learned_mean",
                                              "nrmse_gm_mean", "fallback", "n", "r_learned")}
    del rho_v, u_v
    torch.cuda.empty_cache()

    n = args.learned_n
    h = 2 * math.pi / n
    progress(f"learned: {n}^3 learned-vs-plain race")
    rho, u = synth.workload_fields("c1024_learned", device=dev, n=n)
    ex = kcf.alloc_outputs((n, n, n), dev, ("rho_bar", "ut", "tau"))
    st = ctx.filter_favre(rho, u, h, [(kcf.GAUSS, 8)], [ex])
    m2 = st[0]["m2"]
    tau_l = torch.empty((6, n, n, n), dtype=torch.float32, device=dev)
    tau_gm = torch.empty((6, n, n, n), dtype=torch.float32, device=dev)
    reps = 3
    # plain closure path: exact tau by explicit filtering of rho, u (statistics off)
    t_plain = _timed(lambda: ctx.filter_favre(rho, u, h, [(kcf.GAUSS, 8)], [ex], stats=False), reps)
    # learned path: tau from rho_bar, ut (features, BF16 MFMA MLP, envelope fallback)
    t_learned = _timed(lambda: mlp.infer_field(ex["rho_bar"], ex["ut"], h, 8 * h, m2, tau_out=tau_l,
                                               count=False), reps)
    # gradient-model path: tau_gm from rho_bar, ut
    t_gm = _timed(lambda: ctx.grad_closure(ex["rho_bar"], ex["ut"], None, h, 8 * h, m2,
                                           {"tau_gm": tau_gm}, stats=False), reps)
    _, nfb = mlp.infer_field(ex["rho_bar"], ex["ut"], h, 8 * h, m2, tau_out=tau_l)
    r_l = [learned.pearson_gpu(ctx, tau_l[c], ex["tau"][c]) for c in range(6)]
    r_g = [learned.pearson_gpu(ctx, tau_gm[c], ex["tau"][c]) for c in range(6)]
    nr_l = [learned.nrmse_gpu(ctx, tau_l[c], ex["tau"][c]) for c in range(6)]
    nr_g = [learned.nrmse_gpu(ctx, tau_gm[c], ex["tau"][c]) for c in range(6)]
    pts = float(n) ** 3
    out["race"] = {
        "workload": f"{n}^3 spectral turbulence (k0 {32 * n / 1024:g}), Gaussian filter 8h",
        "plain_exact_ms": t_plain, "learned_ms": t_learned, "gradient_model_ms": t_gm,
        "learned_points_per_s": pts / (t_learned * 1e-3),
        "plain_points_per_s": pts / (t_plain * 1e-3),
        "learned_speedup_vs_plain": t_plain / t_learned,
        "r_learned": r_l, "r_learned_mean": sum(r_l) / 6, "r_gm_mean": sum(r_g) / 6,
        "nrmse_learned_mean": sum(nr_l) / 6, "nrmse_gm_mean": sum(nr_g) / 6,
        "fallback_points": nfb, "points": int(pts),
        "learned_mfma_tflops": 18944 * pts / (t_learned * 1e-3) / 1e12,
    }
    mlp.close()
    return out


CARRIER_BYTES_PER_POINT = 16 + 2 * 27 * 4  # read rho, u; write f_sgs and f_h2 (27 each)


def carrier_section(ctx, rho, u, args):
    """A priori D3Q27 SGS carrier (f_sgs, its second-order Hermite reconstruction f_h2, both
    stored, and their statistics) on the 512^3 field at box 4h (FP64 sums) and 8h (FP32),
    and on the 256^3 Gaussian-8h field."""
    import torch
    from paper_2605_19796_amd import kcf, synth
    out = {}
    cases = [("box4h_512", rho, u, (kcf.BOX, 4)), ("box8h_512", rho, u, (kcf.BOX, 8))]
    r2, u2 = synth.workload_fields("c256_gauss8", device=rho.device)
    cases.append(("gauss8h_256", r2, u2, (kcf.GAUSS, 8)))
    reps = 2 if args.profile_run else 5
    for name, r, v, filt in cases:
        n = r.shape[0]
        h = 2 * math.pi / n
        fs = torch.empty((27,) + tuple(r.shape), dtype=torch.float32, device=r.device)
        fh = torch.empty_like(fs)
        progress(f"carrier {name}")
        st = ctx.sgs_carrier(r, v, h, filt, fs, fh)  # warm-up (allocates the slab buffer)
        ctx.enable_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            st = ctx.sgs_carrier(r, v, h, filt, fs, fh)
        t1 = time.perf_counter()
        kt = ctx.kernel_times()
        ctx.enable_timing(False)
        ms = (t1 - t0) * 1e3 / reps
        kz, kxy = sum(kt[0::2]) / reps, sum(kt[1::2]) / reps
        pts = float(n) ** 3
        gbs = CARRIER_BYTES_PER_POINT * pts / ((kz + kxy) * 1e-3) / 1e9
        out[name] = {
            "grid": n, "filter": ["box", "gauss"][filt[0]], "width_h": filt[1],
            "sums": "f64" if filt[1] <= 4 else "f32",
            "ms_per_call": ms, "points_per_s": pts / (ms * 1e-3),
            "kernel_ms": {"k_carrier_z": kz, "k_carrier_xy": kxy},
            "bytes_per_point": CARRIER_BYTES_PER_POINT,
            "achieved_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
            "rel_err_h2": st["rel_err"], "sgs_l2": st["sgs_l2"], "hermite_2_to_6": st["hermite"],
        }
        del fs, fh
        torch.cuda.empty_cache()
    del r2, u2
    torch.cuda.empty_cache()
    return out


MOMENT3_BYTES_PER_POINT = 20 + 11 * 4  # read rho, u, theta; write m3 (10) and theta_t


def moment3_section(ctx, rho, u, args):
    """Third-order SGS moment and Favre temperature (both stored, with statistics) on the
    512^3 field with a spectral temperature, box 4h (FP64 sums) and 8h (FP32)."""
    import torch
    from paper_2605_19796_amd import kcf, synth
    n = rho.shape[0]
    h = 2 * math.pi / n
    theta = synth.workload_temperature("c512_box_multi", device=rho.device, n=n)
    m3 = torch.empty((10,) + tuple(rho.shape), dtype=torch.float32, device=rho.device)
    tt = torch.empty_like(rho)
    out = {}
    reps = 2 if args.profile_run else 5
    for name, filt in (("box4h_512", (kcf.BOX, 4)), ("box8h_512", (kcf.BOX, 8))):
        progress(f"moment3 {name}")
        st = ctx.sgs_moment3(rho, u, h, filt, theta, m3, tt)
        ctx.enable_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            st = ctx.sgs_moment3(rho, u, h, filt, theta, m3, tt)
        t1 = time.perf_counter()
        kt = ctx.kernel_times()
        ctx.enable_timing(False)
        ms = (t1 - t0) * 1e3 / reps
        kz, kxy = sum(kt[0::2]) / reps, sum(kt[1::2]) / reps
        pts = float(n) ** 3
        gbs = MOMENT3_BYTES_PER_POINT * pts / ((kz + kxy) * 1e-3) / 1e9
        out[name] = {
            "grid": n, "width_h": filt[1], "sums": "f64" if filt[1] <= 4 else "f32",
            "ms_per_call": ms, "points_per_s": pts / (ms * 1e-3),
            "kernel_ms": {"k_moment3_z": kz, "k_moment3_xy": kxy},
            "bytes_per_point": MOMENT3_BYTES_PER_POINT,
            "achieved_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
            "rms_m3": st["rms_m3"], "mean_theta_t": st["mean_theta_t"],
        }
    del theta, m3, tt
    torch.cuda.empty_cache()
    return out


KC_BYTES_PER_POINT = 16 + 9 * 4  # read rho, u; write m_sgs (6), k_sgs, nu_t_eff, omega_sgs
# lattice units: spacing and time step 1, theta_R = 1/3, velocities u sqrt(theta_R) (the
# field's Mach numbers), nu = 1e-4 (shifted rate 1/tau_hat ~ 1.9994)
KC_PARAMS = dict(nu=1e-4, dt=1.0, theta=1.0 / 3.0, c_nu=0.035, rho_ref_one=1)


def kc_section(ctx, rho, u, args):
    """A priori KC-MP SGS moment and relaxation-rate field (all outputs stored, statistics
    against the exact tau) on the 512^3 field in lattice units, box 4h (FP64 sums) and 8h
    (FP32)."""
    import torch
    from paper_2605_19796_amd import kcf
    n = rho.shape[0]
    h = 1.0
    u = (u * math.sqrt(KC_PARAMS["theta"])).contiguous()
    m = torch.empty((6,) + tuple(rho.shape), dtype=torch.float32, device=rho.device)
    k, nue, om = (torch.empty_like(rho) for _ in range(3))
    out = {"params": KC_PARAMS, "units": "lattice (h = dt = 1, u = Mach sqrt(theta_R))"}
    reps = 2 if args.profile_run else 5
    for name, filt in (("box4h_512", (kcf.BOX, 4)), ("box8h_512", (kcf.BOX, 8))):
        progress(f"kc-mp {name}")
        call = lambda: ctx.kc_mp(rho, u, h, filt, m_sgs=m, k_sgs=k, nu_t_eff=nue, omega_sgs=om,
                                 **KC_PARAMS)
        st = call()
        ctx.enable_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            st = call()
        t1 = time.perf_counter()
        kt = ctx.kernel_times()
        ctx.enable_timing(False)
        per = len(kt) // reps  # filter launch, then z and x-y per slab
        ms = (t1 - t0) * 1e3 / reps
        pts = float(n) ** 3
        out[name] = {
            "grid": n, "width_h": filt[1], "ms_per_call": ms, "points_per_s": pts / (ms * 1e-3),
            "kernel_ms": {"filter_path": sum(kt[0::per]) / reps,
                          "k_kc_z": sum(sum(kt[i::per]) for i in range(1, per, 2)) / reps,
                          "k_kc_xy": sum(sum(kt[i::per]) for i in range(2, per, 2)) / reps},
            "bytes_per_point": KC_BYTES_PER_POINT,
            "call_gbs": KC_BYTES_PER_POINT * pts / (ms * 1e-3) / 1e9,
            "corr_m_tau": st["corr"], "rel_err": st["rel_err"],
            "mean_k": st["mean_k"], "mean_k_exact": st["mean_k_exact"],
            "mean_omega": st["mean_omega"], "mean_omega_exact": st["mean_omega_exact"],
            "clip": st["clip"], "clip_exact": st["clip_exact"],
        }
    del m, k, nue, om, u
    torch.cuda.empty_cache()
    return out


C2_BYTES_PER_POINT = 16 + 100  # read rho, u; write rho_bar, ut, tau, grad, tau_gm (25 floats)


def c2_section(ctx, args):
    """256^3 Gaussian filter 8h with the full output set (rho_bar, ut, tau, grad, tau_gm) and
    the FP64 statistics: the x-y pass into the slab buffer, the z pass with Favre division, then
    the gradient/closure pass, timed together as one call."""
    import torch
    from paper_2605_19796_amd import kcf, synth
    dev = torch.device("cuda", 0)
    rho, u = synth.workload_fields("c256_gauss8", device=dev)
    n = rho.shape[0]
    h = 2 * math.pi / n
    outs = [kcf.alloc_outputs((n, n, n), dev, ("rho_bar", "ut", "tau", "grad", "tau_gm"))]
    filt = [(kcf.GAUSS, 8)]
    progress("c2: 256^3 Gaussian 8h")
    ctx.filter_favre(rho, u, h, filt, outs)
    reps = 3 if args.profile_run else 10
    ctx.enable_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        st = ctx.filter_favre(rho, u, h, filt, outs)
    t1 = time.perf_counter()
    kt = ctx.kernel_times()
    ctx.enable_timing(False)
    ms_call = (t1 - t0) * 1e3 / reps
    k_ms = sum(kt) / reps
    pts = float(n) ** 3
    gbs = C2_BYTES_PER_POINT * pts / (k_ms * 1e-3) / 1e9
    out = {"workload": "256^3 spectral turbulence (k0 8, rho amplitude 0.2), Gaussian filter 8h, "
                       "outputs rho_bar, ut, tau, grad, tau_gm and FP64 statistics",
           "ms_per_call": ms_call, "kernel_ms": k_ms, "points_per_s": pts / (ms_call * 1e-3),
           "bytes_per_point": C2_BYTES_PER_POINT, "achieved_gbs": gbs,
           "hbm_frac": gbs / HBM_PEAK_GBS, "pi": st[0]["pi"], "corr_tau_gm": st[0]["corr_tau_gm"]}
    del rho, u, outs
    torch.cuda.empty_cache()
    return out


LBM_BYTES_PER_NODE = 2 * 27 * 4  # read and write the 27 FP32 populations


def lbm_section(ctx, args):
    """D3Q27 collide-and-stream of the Taylor-Green vortex (Re 1600, Ma 0.2: u0 = 0.2 c_s,
    nu = u0 (N / 2 pi) / 1600) on a 256^3 lattice, one timed kernel per step, for the resolved
    BGK step and the kinetic closures (C_nu 0.02 for KC-RB and KC-RR, 0.035 for KC-MP)."""
    import torch
    from paper_2605_19796_amd import kcf, synth
    n = args.lbm_n
    u0 = 0.2 / math.sqrt(3.0)
    nu = u0 * (n / (2 * math.pi)) / 1600.0
    rho_np, u_np = synth.taylor_green(n, u0=u0, rho_fluct=3.0 * u0 * u0 / 16.0)
    dev = torch.device("cuda", 0)
    rho = torch.from_numpy(rho_np).to(dev)
    u = torch.from_numpy(u_np).to(dev)
    f0 = ctx.lbm_equilibrium(rho, u)
    a = torch.empty_like(f0)
    b = torch.empty_like(f0)
    del rho, u
    steps = 4 if args.profile_run else 20
    out = {"workload": f"Taylor-Green vortex on a {n}^3 lattice, Re 1600, Ma 0.2 (lattice units, "
                       f"nu {nu:.5g})", "bytes_per_node": LBM_BYTES_PER_NODE}
    nodes = float(n) ** 3
    for model, c_nu in (("bgk", 0.0), ("kcrb_raw", 0.02), ("kcmp", 0.035), ("kcrr", 0.02)):
        progress(f"lbm {model}")
        a.copy_(f0)
        st0 = ctx.lbm_step(a, b, model, nu, c_nu)
        a, b = b, a
        ctx.enable_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.lbm_step(a, b, model, nu, c_nu, stats=False)
            a, b = b, a
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kt = ctx.kernel_times()
        ctx.enable_timing(False)
        st1 = ctx.lbm_step(a, b, model, nu, c_nu)
        k_ms = sum(kt) / len(kt)
        gbs = LBM_BYTES_PER_NODE * nodes / (k_ms * 1e-3) / 1e9
        out[model] = {
            "c_nu": c_nu, "ms_per_step": (t1 - t0) * 1e3 / steps, "kernel_ms": k_ms,
            "lattice_updates_per_s": nodes / (k_ms * 1e-3), "achieved_gbs": gbs,
            "hbm_frac": gbs / HBM_PEAK_GBS,
            "relative_mass_drift": (st1["mass"] - st0["mass"]) / st0["mass"],
            "kinetic_energy_ratio": st1["kinetic_energy"] / st0["kinetic_energy"],
            "mean_omega_sgs": st1["mean_omega_sgs"], "clip_fraction": st1["clip_fraction"],
        }
    del a, b, f0
    torch.cuda.empty_cache()
    return out


def stream_ceiling(ctx, n):
    """Time of kcf_stream_probe reading 4 and writing 40 fields of n^3 floats: the bytes of
    the four-width step moved by a kernel that does nothing else."""
    import torch
    inp = torch.ones((4, n, n, n), dtype=torch.float32, device="cuda")
    out = torch.empty((40, n, n, n), dtype=torch.float32, device="cuda")
    ctx.stream_probe(inp, out)
    ctx.enable_timing(True)
    for _ in range(5):
        ctx.stream_probe(inp, out)
    kt = ctx.kernel_times()
    ctx.enable_timing(False)
    ms = sum(kt) / len(kt)
    del inp, out
    torch.cuda.empty_cache()
    gbs = BYTES_STEP * float(n) ** 3 / (ms * 1e-3) / 1e9
    return {"kernel": "kcf_stream_probe (4 fields in, 40 out)", "ms": ms, "gbs": gbs,
            "frac_of_peak": gbs / HBM_PEAK_GBS}


def copy_calibration():
    """One plain device-to-device copy of COPY_BYTES, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = COPY_BYTES // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU baseline and the oracle ladder")
    ap.add_argument("--oracle-ladder", action="store_true",
                    help="the full oracle ladder (256^3 full path, 2^16 sampled points; minutes)")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-carrier", action="store_true",
                    help="skip the carrier, third-order moment and KC-MP sections")
    ap.add_argument("--profile-run", action="store_true",
                    help="a few steps only (no CPU baseline, no learned section)")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--learned-n", type=int, default=1024, help="grid of the learned-vs-plain race")
    ap.add_argument("--train-steps", type=int, default=3000)
    ap.add_argument("--no-lbm", action="store_true")
    ap.add_argument("--no-c2", action="store_true")
    ap.add_argument("--lbm-n", type=int, default=256, help="lattice of the lbm section")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the filtering path here is a single-GPU build; "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.profile_run:
        args.no_cpu_baseline = args.no_learned = True

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

    progress(f"{n}^3 4-width pass: warmup")
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
    times = ctx.kernel_times()
    ctx.enable_timing(False)
    progress(f"timed {args.steps} steps")

    ms_step = (t1 - t0) * 1e3 / args.steps
    pts = float(n) ** 3
    value = pts / (ms_step * 1e-3)
    # the timed launches are the filter kernels, one per width per step, in width order
    assert len(times) == len(WIDTHS) * args.steps, (len(times), args.steps)
    per_width = {w: times[i::len(WIDTHS)] for i, w in enumerate(WIDTHS)}
    avg = {w: sum(v) / len(v) for w, v in per_width.items()}
    dom = max(WIDTHS, key=lambda w: avg[w])
    kernel = KERNELS[dom]
    bytes_launch = BYTES_PER_LAUNCH * pts
    achieved = bytes_launch / (avg[dom] * 1e-3) / 1e9
    step_kernel_ms = sum(avg.values())
    step_gbs = BYTES_STEP * pts / (step_kernel_ms * 1e-3) / 1e9
    traffic = load_traffic(kernel)
    progress("streaming ceiling")
    ceiling = stream_ceiling(ctx, n)
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
            "workload": f"{n}^3 periodic spectral turbulence, box filter widths 2h/4h/8h/16h, "
                        "FP32 fields, FP64 on-GPU statistics",
            "grid": n, "filter": "box", "widths_h": list(WIDTHS), "k0": 16 * n / 512,
            "u_rms": 0.3, "rho_amp": 0.2, "seeds": [1004, 2004],
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": kernel, "width_h": dom, "kernel_ms": avg[dom],
            "bytes_per_launch": bytes_launch, "bytes_per_point": BYTES_PER_LAUNCH,
            "kernel_ms_by_width": {f"{w}h": avg[w] for w in WIDTHS},
            "step": {"bytes_per_point": BYTES_STEP, "kernel_ms": step_kernel_ms,
                     "achieved": step_gbs, "frac": step_gbs / HBM_PEAK_GBS,
                     "frac_by_ms_per_step": BYTES_STEP * pts / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS},
        },
        "stream_ceiling": ceiling,
        "stats": {
            f"{w}h": {"pi": s["pi"], "pi_gm": s["pi_gm"], "corr_tau_gm": s["corr_tau_gm"],
                      "corr_pi": s["corr_pi"]} for w, s in zip(WIDTHS, st)
        },
        "input": ist,
    }
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(rho, u)
    del outs
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        line["oracle_ladder"] = oracle_ladder(args.oracle_ladder)
    if not args.no_c2:
        line["c2"] = c2_section(ctx, args)
    if not args.no_carrier:
        line["carrier"] = carrier_section(ctx, rho, u, args)
        line["moment3"] = moment3_section(ctx, rho, u, args)
        line["kc_mp"] = kc_section(ctx, rho, u, args)
    if not args.no_lbm:
        line["lbm"] = lbm_section(ctx, args)
    if not args.no_learned:
        del rho, u
        torch.cuda.empty_cache()
        line["learned"] = learned_section(ctx, args)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""GPU parity of the D3Q27 SGS carrier (kcf_sgs_carrier) against the FP64 oracle, through the
C ABI.

Tolerance: per population i, max_x |gpu_i - oracle_i| / max_x |oracle_i| <= 1e-5 for f_sgs
and f_h2 on the same float32 inputs. Statistics: the GPU sums a point's 27 populations in FP32
and the points in FP64; against host FP64 sums of the GPU's own float outputs that agrees to
2e-6 relative (27 FP32 additions), against the oracle's statistics to the field tolerance. The moment identities of the carrier (vanishing zeroth and
first moments, second moment = tau) are checked on the GPU output against tau of the filter
path, a separate set of kernels.
"""
import math
import sys
import zlib

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import carrier as K  # noqa: E402
from oracle import fields as F  # noqa: E402
from paper_2605_19796_amd import kcf, synth  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-5
HOST_TOL = 2e-6  # device sums vs host FP64 sums of the device's outputs


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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def rel(g, o):
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    m = np.max(np.abs(o))
    return float(np.max(np.abs(g - o)) / m) if m > 0 else float(np.max(np.abs(g)))


def seed_of(name):
    return zlib.crc32(name.encode()) & 0xFFFF


def run(ctx, rho, u, h, filt, stats=True):
    nz, ny, nx = rho.shape
    fs = torch.empty((27, nz, ny, nx), dtype=torch.float32, device="cuda")
    fh = torch.empty_like(fs)
    st = ctx.sgs_carrier(rho, u, h, filt, fs, fh, stats)
    torch.cuda.synchronize()
    return fs, fh, st


def host_sums(fs, fh):
    """FP64 sums of the device's float outputs (over all points and populations)."""
    s1 = s2 = 0.0
    for i in range(27):
        a = fs[i].double()
        b = fh[i].double()
        s1 += float((a * a).sum())
        s2 += float(((a - b) ** 2).sum())
    return s1, s2


# ------------------------------------------------------------------ full fields, small grids
CASES = [
    ("box4_auto", (20, 36, 40), (F.BOX, 4, 0)),      # FP64, R = 2
    ("box2_auto", (17, 33, 18), (F.BOX, 2, 0)),      # FP64, R = 1
    ("gauss2_auto", (24, 20, 35), (F.GAUSS, 2, 0)),  # FP64, R = 3
    ("box8_fp32", (19, 34, 37), (F.BOX, 8, 1)),      # FP32, R = 4
    ("gauss4_fp32", (30, 33, 40), (F.GAUSS, 4, 1)),  # FP32, R = 6
    ("gauss8_fp32", (28, 36, 40), (F.GAUSS, 8, 1)),  # FP32, R = 12 (the Gaussian 8h taps)
    ("gauss8_fp64", (26, 26, 25), (F.GAUSS, 8, 2)),  # FP64, R = 12: three monomials per round
    ("tiny_box4", (5, 6, 7), (F.BOX, 4, 0)),          # 2R + 1 = n along z, one partial tile
    ("thin_box2", (3, 70, 3), (F.BOX, 2, 1)),         # FP32, three cells in x and z
]


@pytest.mark.parametrize("name,shape,filt", CASES, ids=[c[0] for c in CASES])
def test_full_field_parity(ctx, name, shape, filt):
    say(f"[gpu] carrier {name} {shape} filter {filt}")
    rho_h, u_h = synth.random_fields(shape, seed=seed_of(name), rho_amp=0.2)
    h = 2 * math.pi / shape[2]
    fs, fh, st = run(ctx, dev(rho_h), dev(u_h), h, filt)
    o = K.carrier(rho_h, u_h, filt[0], filt[1])
    gs, gh = fs.cpu().numpy(), fh.cpu().numpy()
    for i in range(27):
        assert rel(gs[i], o["f_sgs"][i]) <= TOL, (i, rel(gs[i], o["f_sgs"][i]))
        assert rel(gh[i], o["f_h2"][i]) <= TOL, (i, rel(gh[i], o["f_h2"][i]))
    n = int(np.prod(shape))
    assert st["n_points"] == n and st["n_nonfinite"] == 0
    s1, s2 = host_sums(fs, fh)
    assert abs(st["raw"][1] - s1) <= HOST_TOL * s1
    assert abs(st["raw"][2] - s2) <= HOST_TOL * s2
    os_ = K.carrier_stats(o["f_sgs"], o["f_h2"])
    assert abs(st["sgs_l2"] - os_["sgs_l2"]) <= TOL * os_["sgs_l2"]
    assert abs(st["err_l2"] - os_["err_l2"]) <= 10 * TOL * os_["err_l2"]
    assert abs(st["rel_err"] - os_["rel_err"]) <= 10 * TOL * os_["rel_err"]
    # Hermite energies: relative to the total, order by order
    tot = float(np.sum(os_["hermite"]))
    for k in range(5):
        assert abs(st["hermite"][k] - os_["hermite"][k + 2]) <= TOL * tot, (k, st["hermite"], os_["hermite"])


def test_moments_match_filter_path_tau(ctx):
    """sum_i f_sgs = 0, sum_i xh f_sgs = 0, sum_i xh xh f_sgs = tau of kcf_filter_favre."""
    shape = (24, 32, 40)
    rho_h, u_h = synth.random_fields(shape, seed=11, rho_amp=0.2)
    rho, u = dev(rho_h), dev(u_h)
    h = 2 * math.pi / shape[2]
    for filt in [(F.BOX, 4, 0), (F.GAUSS, 4, 1)]:
        fs, fh, _ = run(ctx, rho, u, h, filt, stats=False)
        outs = [kcf.alloc_outputs(shape, "cuda", ("tau",))]
        ctx.filter_favre(rho, u, h, [filt], outs, stats=False)
        torch.cuda.synchronize()
        tau = outs[0]["tau"].cpu().numpy().astype(np.float64)
        m0, m1, m2 = K.moments(fs.cpu().numpy().astype(np.float64))
        scale = np.max(np.abs(tau))
        assert np.max(np.abs(m0)) <= TOL * scale
        assert np.max(np.abs(m1)) <= TOL * scale
        for c, (a, b) in enumerate(F.PAIRS):
            assert rel(m2[a, b], tau[c]) <= TOL, (filt, a, b, rel(m2[a, b], tau[c]))
        # the reconstruction has exactly these three moments
        h0, h1, h2 = K.moments(fh.cpu().numpy().astype(np.float64))
        assert np.max(np.abs(h0)) <= TOL * scale and np.max(np.abs(h1)) <= TOL * scale
        for c, (a, b) in enumerate(F.PAIRS):
            assert rel(h2[a, b], tau[c]) <= TOL


def test_vanishing_cases(ctx):
    """Constant fields and a uniform velocity with variable density give f_sgs = 0."""
    shape = (16, 20, 18)
    h = 2 * math.pi / 18
    rho_h, _ = synth.random_fields(shape, seed=12, rho_amp=0.3)
    u_h = np.zeros((3,) + shape, dtype=np.float32)
    u_h[0], u_h[1], u_h[2] = 0.2, -0.1, 0.05
    for filt in [(F.BOX, 4, 0), (F.GAUSS, 2, 1)]:
        fs, fh, st = run(ctx, dev(rho_h), dev(u_h), h, filt)
        # relative to the size of the equilibrium (about w_i rho), rounding only
        assert float(fs.abs().max()) < 1e-6 and float(fh.abs().max()) < 1e-6
        assert st["n_points"] == int(np.prod(shape))


def test_outputs_optional_and_bit_identical(ctx):
    """Any subset of outputs; each output is bit-identical across subsets; repeated calls are
    bit-identical (statistics included)."""
    shape = (20, 24, 30)
    rho_h, u_h = synth.random_fields(shape, seed=13, rho_amp=0.2)
    rho, u = dev(rho_h), dev(u_h)
    h = 2 * math.pi / 30
    filt = (F.GAUSS, 3, 0)
    fs, fh, st = run(ctx, rho, u, h, filt)
    fs2 = torch.empty_like(fs)
    assert ctx.sgs_carrier(rho, u, h, filt, fs2, None, False) is None
    fh2 = torch.empty_like(fh)
    st2 = ctx.sgs_carrier(rho, u, h, filt, None, fh2, True)
    st3 = ctx.sgs_carrier(rho, u, h, filt, None, None, True)
    torch.cuda.synchronize()
    assert torch.equal(fs, fs2) and torch.equal(fh, fh2)
    assert st["raw"] == st2["raw"] == st3["raw"]


def test_nonfinite_points_counted(ctx):
    shape = (12, 16, 16)
    rho_h, u_h = synth.random_fields(shape, seed=14)
    rho_h[5, 7, 3] = np.nan
    _, _, st = run(ctx, dev(rho_h), dev(u_h), 2 * math.pi / 16, (F.BOX, 2, 0))
    assert st["n_nonfinite"] > 0 and st["n_points"] + st["n_nonfinite"] == 12 * 16 * 16


def test_error_paths(ctx):
    shape = (12, 12, 12)
    rho_h, u_h = synth.random_fields(shape, seed=15)
    rho, u = dev(rho_h), dev(u_h)
    h = 2 * math.pi / 12
    with pytest.raises(kcf.KcfError) as e:
        ctx.sgs_carrier(rho, u, h, (F.BOX, 4, 0), None, None, False)
    assert e.value.code == kcf.EINVAL
    with pytest.raises(kcf.KcfError) as e:
        ctx.sgs_carrier(rho, u, h, (F.BOX, 3, 0))
    assert e.value.code == kcf.EINVAL
    with pytest.raises(kcf.KcfError) as e:  # 2R+1 = 13 > 12
        ctx.sgs_carrier(rho, u, h, (F.GAUSS, 4, 0))
    assert e.value.code == kcf.EUNSUPPORTED
    with pytest.raises(kcf.KcfError) as e:
        ctx.sgs_carrier(rho, u, h, (F.BOX, 4, 3))
    assert e.value.code == kcf.EINVAL


# ------------------------------------------------------------------ full sizes, sampled points
def sample_points(n, k, seed):
    rng = np.random.default_rng(seed)
    pts = [(0, 0, 0), (n - 1, n - 1, n - 1), (n // 2, 15, 16), (n // 2 + 1, 16, 15)]
    pts += [tuple(int(v) for v in p) for p in rng.integers(0, n, (k, 3))]
    return np.array(pts)


def check_sampled(ctx, name, n, filt, k, seed):
    h = 2 * math.pi / n
    rho_d, u_d = synth.workload_fields(name, device="cuda")
    fs, fh, st = run(ctx, rho_d, u_d, h, filt)
    assert st["n_points"] == n ** 3 and st["n_nonfinite"] == 0
    s1, s2 = host_sums(fs, fh)
    assert abs(st["raw"][1] - s1) <= HOST_TOL * s1
    assert abs(st["raw"][2] - s2) <= HOST_TOL * s2
    pts = sample_points(n, k, seed)
    say(f"[gpu]   {len(pts)} sampled points")
    rf, rh = K.carrier_at(rho_d.cpu().numpy(), u_d.cpu().numpy(), filt[0], filt[1], pts)
    idx = torch.as_tensor(pts, device="cuda", dtype=torch.long)
    gs = fs[:, idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy().T
    gh = fh[:, idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy().T
    for i in range(27):
        assert rel(gs[:, i], rf[:, i]) <= TOL, (i, rel(gs[:, i], rf[:, i]))
        assert rel(gh[:, i], rh[:, i]) <= TOL, (i, rel(gh[:, i], rh[:, i]))
    return st


def test_c256_gauss8_sampled(ctx):
    say("[gpu] carrier 256^3 gaussian delta=8h (FP32): sampled-point parity")
    check_sampled(ctx, "c256_gauss8", 256, (F.GAUSS, 8, 0), 10, 1)


def test_c512_box4_fp64_slabs_sampled(ctx):
    """512^3 at FP64 holds 27 monomials in z slabs of the 8 GiB buffer (four slabs)."""
    say("[gpu] carrier 512^3 box delta=4h (FP64, z slabs): sampled-point parity")
    check_sampled(ctx, "c512_box_multi", 512, (F.BOX, 4, 0), 16, 2)

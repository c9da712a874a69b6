"""GPU parity of the a priori KC-MP evaluation (kcf_kc_mp) against the FP64 oracle, through
the C ABI.

Tolerance: per component or field, max_x |gpu - oracle| / max_x |oracle| <= 1e-5 on the same
float32 inputs. Statistics: the GPU's FP64 sums of its own float outputs agree with host FP64
sums of those outputs to 1e-10 relative; against the oracle's statistics to the field
tolerance, except the fractions of clipped points, where a point within rounding of the
threshold may fall either way.
"""
import math
import sys
import zlib

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import fields as F  # noqa: E402
from oracle import kc_mp as KC  # noqa: E402
from paper_2605_19796_amd import kcf, synth  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-5


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


def run(ctx, rho, u, h, filt, p, stats=True, m_ce=None):
    nz, ny, nx = rho.shape
    m = torch.empty((6, nz, ny, nx), dtype=torch.float32, device="cuda")
    k, nue, om = (torch.empty((nz, ny, nx), dtype=torch.float32, device="cuda") for _ in range(3))
    st = ctx.kc_mp(rho, u, h, filt, m_sgs=m, m_ce=m_ce, k_sgs=k, nu_t_eff=nue, omega_sgs=om,
                   stats=stats, **p)
    torch.cuda.synchronize()
    return m, k, nue, om, st


P1 = dict(nu=0.002, dt=0.5, theta=1.0 / 3.0, c_nu=0.035, rho_ref_one=1)
P2 = dict(nu=0.004, dt=0.0, theta=1.0, c_nu=0.02, rho_ref_one=0)
CASES = [
    ("box4_auto", (20, 36, 40), (F.BOX, 4, 0), P1),      # FP64, R = 2
    ("box2_auto", (17, 33, 18), (F.BOX, 2, 0), P2),      # FP64, R = 1
    ("gauss3_auto", (24, 20, 35), (F.GAUSS, 3, 0), P1),  # FP64, R = 5 (general-tap filter path)
    ("box8_fp32", (19, 34, 37), (F.BOX, 8, 1), P2),      # FP32, R = 4
    ("gauss8_fp32", (28, 36, 40), (F.GAUSS, 8, 1), P1),  # FP32, R = 12
    ("tiny_box4", (5, 6, 7), (F.BOX, 4, 0), P2),         # 2R + 1 = n along z
    ("thin_box2", (3, 70, 3), (F.BOX, 2, 1), P1),        # FP32, three cells in x and z
]


@pytest.mark.parametrize("name,shape,filt,p", CASES, ids=[c[0] for c in CASES])
def test_full_field_parity(ctx, name, shape, filt, p):
    say(f"[gpu] kc-mp {name} {shape} filter {filt}")
    rho_h, u_h = synth.random_fields(shape, seed=seed_of(name), rho_amp=0.2)
    h = 2 * math.pi / shape[2]
    mce = torch.empty((6,) + shape, dtype=torch.float32, device="cuda")
    m, k, nue, om, st = run(ctx, dev(rho_h), dev(u_h), h, filt, p, m_ce=mce)
    o = KC.kc_mp(rho_h, u_h, filt[0], filt[1], h, p["nu"], p["dt"], p["theta"], p["c_nu"],
                 bool(p["rho_ref_one"]))
    g = m.cpu().numpy()
    gce = mce.cpu().numpy()
    for c, (i, j) in enumerate(F.PAIRS):
        assert rel(g[c], o["m_sgs"][i, j]) <= TOL, (c, rel(g[c], o["m_sgs"][i, j]))
        assert rel(gce[c], o["m_ce"][i, j]) <= TOL, (c, rel(gce[c], o["m_ce"][i, j]))
    for got, key in ((k, "k_sgs"), (nue, "nu_t_eff"), (om, "omega_sgs")):
        assert rel(got.cpu().numpy(), o[key]) <= TOL, (key, rel(got.cpu().numpy(), o[key]))
    n = int(np.prod(shape))
    assert st["n_points"] == n and st["n_nonfinite"] == 0
    # device sums of the device's outputs
    assert abs(st["raw"][33] - float(k.double().sum())) <= 1e-10 * float(k.double().sum())
    assert abs(st["raw"][35] - float(om.double().sum())) <= 1e-10 * float(om.double().sum())
    os_ = KC.kc_mp_stats(o, p["nu"])
    for c in range(6):
        assert abs(st["corr"][c] - os_["corr"][c]) <= 1e-4, (c, st["corr"], os_["corr"])
    assert abs(st["rel_err"] - os_["rel_err"]) <= 1e-4 * os_["rel_err"] + 1e-6
    for a, b in (("mean_k", "mean_k"), ("mean_k_exact", "mean_k_exact"),
                 ("mean_omega", "mean_omega"), ("mean_omega_exact", "mean_omega_exact")):
        assert abs(st[a] - os_[b]) <= TOL * abs(os_[b]), (a, st[a], os_[b])
    assert abs(st["clip"] - os_["clip"]) <= 5.0 / n
    assert abs(st["clip_exact"] - os_["clip_exact"]) <= 5.0 / n


def test_constant_density_gives_tau(ctx):
    """At constant density the discrete filter commutes with the differences, so the KC-MP
    moment is the exact tau of the filter path."""
    shape = (16, 24, 20)
    _, u_h = synth.random_fields(shape, seed=51)
    rho_h = np.full(shape, 1.2, dtype=np.float32)
    h = 2 * math.pi / 20
    filt = (F.BOX, 4, 0)
    rho, u = dev(rho_h), dev(u_h)
    m, _, _, _, st = run(ctx, rho, u, h, filt, P1)
    outs = [kcf.alloc_outputs(shape, "cuda", ("tau",))]
    ctx.filter_favre(rho, u, h, [filt], outs, stats=False)
    torch.cuda.synchronize()
    tau = outs[0]["tau"].cpu().numpy()
    assert rel(m.cpu().numpy(), tau) <= 1e-6
    assert st["rel_err"] <= 1e-6 and min(st["corr"]) > 0.999999


def test_outputs_optional_and_bit_identical(ctx):
    shape = (20, 24, 30)
    rho_h, u_h = synth.random_fields(shape, seed=52, rho_amp=0.2)
    rho, u = dev(rho_h), dev(u_h)
    h = 2 * math.pi / 30
    filt = (F.GAUSS, 2, 0)
    m, k, nue, om, st = run(ctx, rho, u, h, filt, P1)
    m2 = torch.empty_like(m)
    assert ctx.kc_mp(rho, u, h, filt, m_sgs=m2, stats=False, **P1) is None
    st2 = ctx.kc_mp(rho, u, h, filt, stats=True, **P1)
    om2 = torch.empty_like(om)
    ctx.kc_mp(rho, u, h, filt, omega_sgs=om2, stats=False, **P1)
    torch.cuda.synchronize()
    assert torch.equal(m, m2) and torch.equal(om, om2) and st["raw"] == st2["raw"]


def test_error_paths(ctx):
    shape = (12, 12, 12)
    rho_h, u_h = synth.random_fields(shape, seed=53)
    rho, u = dev(rho_h), dev(u_h)
    h = 2 * math.pi / 12
    with pytest.raises(kcf.KcfError) as e:
        ctx.kc_mp(rho, u, h, (F.BOX, 4, 0), stats=False, **P1)
    assert e.value.code == kcf.EINVAL
    bad = dict(P1, theta=0.0)
    with pytest.raises(kcf.KcfError) as e:
        ctx.kc_mp(rho, u, h, (F.BOX, 4, 0), **bad)
    assert e.value.code == kcf.EINVAL
    with pytest.raises(kcf.KcfError) as e:
        ctx.kc_mp(rho, u, h, (F.GAUSS, 4, 0), **P1)
    assert e.value.code == kcf.EUNSUPPORTED


def test_c256_gauss8_sampled(ctx):
    say("[gpu] kc-mp 256^3 gaussian delta=8h: sampled-point parity")
    n = 256
    h = 2 * math.pi / n
    rho_d, u_d = synth.workload_fields("c256_gauss8", device="cuda")
    p = dict(nu=1e-3, dt=0.0, theta=1.0, c_nu=0.035, rho_ref_one=1)
    m, k, nue, om, st = run(ctx, rho_d, u_d, h, (F.GAUSS, 8, 0), p)
    assert st["n_points"] == n ** 3 and st["n_nonfinite"] == 0
    rng = np.random.default_rng(6)
    pts = np.concatenate([np.array([(0, 0, 0), (n - 1, n - 1, n - 1), (9, 15, 16)]),
                          rng.integers(0, n, (8, 3))])
    rm, rk, rnue, rom = KC.kc_mp_at(rho_d.cpu().numpy(), u_d.cpu().numpy(), F.GAUSS, 8, h,
                                    p["nu"], p["dt"], p["theta"], p["c_nu"], True, pts)
    idx = torch.as_tensor(pts, device="cuda", dtype=torch.long)
    gm = m[:, idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy().T
    for c, (i, j) in enumerate(F.PAIRS):
        assert rel(gm[:, c], rm[:, i, j]) <= TOL, (c, rel(gm[:, c], rm[:, i, j]))
    for got, ref in ((k, rk), (om, rom)):
        assert rel(got[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy(), ref) <= TOL

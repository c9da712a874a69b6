"""GPU parity of the third-order SGS moment and the Favre temperature (kcf_sgs_moment3)
against the FP64 oracle, through the C ABI.

Tolerance: per component c, max_x |gpu_c - oracle_c| / max_x |oracle_c| <= 1e-5 on the same
float32 inputs. Statistics: the GPU forms a point's values in FP32 and sums points in FP64;
against host FP64 sums of the GPU's own float outputs that agrees to 1e-6 relative (the
squares are FP32 products), against the oracle's means to the field tolerance.
"""
import math
import sys
import zlib

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import fields as F  # noqa: E402
from oracle import moment3 as M  # noqa: E402
from paper_2605_19796_amd import kcf, synth  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-5
HOST_TOL = 1e-6


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


def run(ctx, rho, u, h, filt, theta=None, stats=True):
    nz, ny, nx = rho.shape
    m3 = torch.empty((10, nz, ny, nx), dtype=torch.float32, device="cuda")
    tt = torch.empty((nz, ny, nx), dtype=torch.float32, device="cuda") if theta is not None else None
    st = ctx.sgs_moment3(rho, u, h, filt, theta, m3, tt, stats)
    torch.cuda.synchronize()
    return m3, tt, st


CASES = [
    ("box4_auto", (20, 36, 40), (F.BOX, 4, 0)),      # FP64, R = 2
    ("box2_auto", (17, 33, 18), (F.BOX, 2, 0)),      # FP64, R = 1
    ("gauss3_auto", (24, 20, 35), (F.GAUSS, 3, 0)),  # FP64, R = 5
    ("box8_fp32", (19, 34, 37), (F.BOX, 8, 1)),      # FP32, R = 4
    ("gauss8_fp32", (28, 36, 40), (F.GAUSS, 8, 1)),  # FP32, R = 12
    ("gauss8_fp64", (26, 26, 25), (F.GAUSS, 8, 2)),  # FP64, R = 12
    ("tiny_box4", (5, 6, 7), (F.BOX, 4, 0)),          # 2R + 1 = n along z, one partial tile
    ("thin_box2", (3, 70, 3), (F.BOX, 2, 1)),         # FP32, three cells in x and z
]


@pytest.mark.parametrize("name,shape,filt", CASES, ids=[c[0] for c in CASES])
def test_full_field_parity(ctx, name, shape, filt):
    say(f"[gpu] moment3 {name} {shape} filter {filt}")
    rho_h, u_h = synth.random_fields(shape, seed=seed_of(name), rho_amp=0.2)
    th_h, _ = synth.random_fields(shape, seed=seed_of(name) + 1, rho_amp=0.15)
    h = 2 * math.pi / shape[2]
    m3, tt, st = run(ctx, dev(rho_h), dev(u_h), h, filt, theta=dev(th_h))
    o = M.moment3(rho_h, u_h, filt[0], filt[1])
    ot = M.favre_temperature(rho_h, th_h, filt[0], filt[1])
    g = m3.cpu().numpy()
    for c in range(10):
        assert rel(g[c], o["m3"][c]) <= TOL, (c, rel(g[c], o["m3"][c]))
    assert rel(tt.cpu().numpy(), ot) <= TOL
    n = int(np.prod(shape))
    assert st["n_points"] == n and st["n_nonfinite"] == 0
    gd = m3.double()
    for c in range(10):
        s1 = float(gd[c].sum())
        s2 = float((gd[c] ** 2).sum())
        assert abs(st["raw"][1 + c] - s1) <= HOST_TOL * float(gd[c].abs().sum())
        assert abs(st["raw"][11 + c] - s2) <= HOST_TOL * s2
        scale = np.max(np.abs(o["m3"][c]))
        assert abs(st["mean_m3"][c] - float(np.mean(o["m3"][c]))) <= TOL * scale
        assert abs(st["rms_m3"][c] - math.sqrt(float(np.mean(o["m3"][c] ** 2)))) <= TOL * scale
    assert abs(st["mean_theta_t"] - float(np.mean(ot))) <= TOL * np.max(np.abs(ot))


def test_without_temperature_and_bit_identical(ctx):
    """The moment does not depend on whether a temperature is filtered alongside; outputs are
    optional; repeated calls are bit-identical."""
    shape = (20, 24, 30)
    rho_h, u_h = synth.random_fields(shape, seed=31, rho_amp=0.2)
    th_h, _ = synth.random_fields(shape, seed=32, rho_amp=0.1)
    rho, u = dev(rho_h), dev(u_h)
    h = 2 * math.pi / 30
    filt = (F.GAUSS, 3, 0)
    a, _, sa = run(ctx, rho, u, h, filt, theta=dev(th_h))
    b, _, sb = run(ctx, rho, u, h, filt)
    assert torch.equal(a, b)
    assert sb["mean_theta_t"] == 1.0 and sa["raw"][:21] == sb["raw"][:21]
    c = torch.empty_like(a)
    assert ctx.sgs_moment3(rho, u, h, filt, None, c, None, False) is None
    s3 = ctx.sgs_moment3(rho, u, h, filt, None, None, None, True)
    torch.cuda.synchronize()
    assert torch.equal(a, c) and s3["raw"] == sb["raw"]


def test_galilean_shift_rule_on_gpu(ctx):
    """m3(u + U) - m3(u) = U_i tau_jk + U_j tau_ik + U_k tau_ij, tau from kcf_filter_favre."""
    shape = (16, 24, 20)
    rho_h, u_h = synth.random_fields(shape, seed=33, rho_amp=0.2)
    U = np.array([0.25, -0.15, 0.1], dtype=np.float32)
    h = 2 * math.pi / 20
    filt = (F.BOX, 4, 0)
    rho = dev(rho_h)
    a, _, _ = run(ctx, rho, dev(u_h), h, filt, stats=False)
    b, _, _ = run(ctx, rho, dev(u_h + U[:, None, None, None]), h, filt, stats=False)
    outs = [kcf.alloc_outputs(shape, "cuda", ("tau",))]
    ctx.filter_favre(rho, dev(u_h), h, [filt], outs, stats=False)
    torch.cuda.synchronize()
    tau6 = outs[0]["tau"].cpu().numpy().astype(np.float64)
    T = np.empty((3, 3) + shape)
    for c, (i, j) in enumerate(F.PAIRS):
        T[i, j] = T[j, i] = tau6[c]
    d = (b - a).cpu().numpy().astype(np.float64)
    for c, (i, j, k) in enumerate(M.TRIPLES):
        shift = U[i] * T[j, k] + U[j] * T[i, k] + U[k] * T[i, j]
        # the shift is O(U tau); each side carries its own 1e-5 relative error
        assert rel(d[c], shift) <= 1e-4, (i, j, k, rel(d[c], shift))


def test_error_paths(ctx):
    shape = (12, 12, 12)
    rho_h, u_h = synth.random_fields(shape, seed=34)
    rho, u = dev(rho_h), dev(u_h)
    h = 2 * math.pi / 12
    with pytest.raises(kcf.KcfError) as e:
        ctx.sgs_moment3(rho, u, h, (F.BOX, 4, 0), None, None, None, False)
    assert e.value.code == kcf.EINVAL
    tt = torch.empty_like(rho)
    with pytest.raises(kcf.KcfError) as e:  # theta_t without theta
        ctx.sgs_moment3(rho, u, h, (F.BOX, 4, 0), None, None, tt, True)
    assert e.value.code == kcf.EINVAL
    with pytest.raises(kcf.KcfError) as e:
        ctx.sgs_moment3(rho, u, h, (F.GAUSS, 4, 0))
    assert e.value.code == kcf.EUNSUPPORTED


def test_c512_box4_sampled(ctx):
    """512^3 box 4h (FP64 sums, the field's z slabs fit the buffer) at sampled points."""
    say("[gpu] moment3 512^3 box delta=4h: sampled-point parity")
    n = 512
    h = 2 * math.pi / n
    rho_d, u_d = synth.workload_fields("c512_box_multi", device="cuda")
    m3, _, st = run(ctx, rho_d, u_d, h, (F.BOX, 4, 0))
    assert st["n_points"] == n ** 3 and st["n_nonfinite"] == 0
    rng = np.random.default_rng(5)
    pts = np.concatenate([np.array([(0, 0, 0), (n - 1, n - 1, n - 1), (7, 15, 16)]),
                          rng.integers(0, n, (16, 3))])
    ref, _ = M.moment3_at(rho_d.cpu().numpy(), u_d.cpu().numpy(), None, F.BOX, 4, pts)
    idx = torch.as_tensor(pts, device="cuda", dtype=torch.long)
    got = m3[:, idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy().T
    for c in range(10):
        assert rel(got[:, c], ref[:, c]) <= TOL, (c, rel(got[:, c], ref[:, c]))

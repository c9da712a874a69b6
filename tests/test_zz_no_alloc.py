"""The no-allocation entry point kcf_filter_favre_noalloc against kcf_filter_favre, through the
C ABI: two calls in a row (the second on a smaller grid, so the shared scratch holds the first
call's records when the second starts), outputs and statistics compared bit for bit (the same
kernels, launch geometry and fixed-order reductions run on both paths), plus its limits."""
import ctypes as C
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2605_19796_amd import kcf, synth  # noqa: E402

pytestmark = pytest.mark.gpu
FIELDS = ("rho_bar", "ut", "tau", "grad", "tau_gm")
# (box 2h at precision 2: the exact-statistics kernel; 4h: the float32 fold)
FILTERS = [(kcf.BOX, 2, 2), (kcf.BOX, 4), (kcf.BOX, 8), (kcf.BOX, 16)]


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


def run_both(ctx, shape, seed):
    rho, u = synth.random_fields(shape, seed=seed, rho_amp=0.2)
    rho, u = torch.from_numpy(rho).float().cuda(), torch.from_numpy(u).float().cuda()
    h = 2 * math.pi / shape[2]
    nz, ny, nx = shape
    filt = [f for f in FILTERS if 2 * (f[1] // 2) + 1 <= min(shape)]
    ref_out = [kcf.alloc_outputs(shape, "cuda", FIELDS) for _ in filt]
    na_out = [kcf.alloc_outputs(shape, "cuda", FIELDS) for _ in filt]
    for o in na_out:
        for t in o.values():
            t.fill_(float("nan"))
    st_ref = ctx.filter_favre(rho, u, h, filt, ref_out)
    st_na = kcf.filter_favre_noalloc(rho, u, h, filt, na_out)
    torch.cuda.synchronize()
    return filt, ref_out, na_out, st_ref, st_na


@pytest.mark.parametrize("shapes", [((40, 36, 44), (20, 18, 22))])
def test_noalloc_matches_filter_favre(ctx, shapes):
    for i, shape in enumerate(shapes):
        say(f"[gpu] no-allocation entry point, call {i + 1}, grid {shape}")
        filt, ref_out, na_out, st_ref, st_na = run_both(ctx, shape, 900 + i)
        for f, (a, b) in enumerate(zip(ref_out, na_out)):
            for k in FIELDS:
                assert torch.equal(a[k], b[k]), (shape, filt[f], k)
        for f, (a, b) in enumerate(zip(st_ref, st_na)):
            assert a["raw"] == b["raw"], (shape, filt[f])
            assert a["n_points"] == math.prod(shape) and b["n_points"] == a["n_points"]
            assert a["pi"] == b["pi"] and a["corr_tau_gm"] == b["corr_tau_gm"]


def test_noalloc_without_stats_and_limits(ctx):
    say("[gpu] no-allocation entry point: no statistics, rejected requests")
    shape = (24, 24, 24)
    rho, u = synth.random_fields(shape, seed=77, rho_amp=0.2)
    rho, u = torch.from_numpy(rho).float().cuda(), torch.from_numpy(u).float().cuda()
    h = 2 * math.pi / 24
    o1 = [kcf.alloc_outputs(shape, "cuda", ("rho_bar", "ut", "tau"))]
    o2 = [kcf.alloc_outputs(shape, "cuda", ("rho_bar", "ut", "tau"))]
    ctx.filter_favre(rho, u, h, [(kcf.BOX, 4)], o1, stats=False)
    assert kcf.filter_favre_noalloc(rho, u, h, [(kcf.BOX, 4)], o2, stats=False) is None
    torch.cuda.synchronize()
    for k in o1[0]:
        assert torch.equal(o1[0][k], o2[0][k])
    with pytest.raises(kcf.KcfError) as e:  # Gaussian: not on the box path
        kcf.filter_favre_noalloc(rho, u, h, [(kcf.GAUSS, 2)], o2)
    assert e.value.code == kcf.EUNSUPPORTED
    # a 1024^3 grid at 2h has more statistics records than the scratch holds: rejected by
    # the size check before any launch (the small tensors are never touched)
    L = kcf.lib()
    g = kcf.Grid(1024, 1024, 1024, 2 * math.pi / 1024)
    fa = (kcf.Filter * 1)(kcf.Filter(kcf.BOX, 2, 0))
    oa = (kcf.Outputs * 1)()
    st = (kcf.WidthStats * 1)()
    rc = L.kcf_filter_favre_noalloc(C.byref(g), fa, 1, kcf._ptr(rho), kcf._ptr(u), oa, None, st,
                                    0, None)
    assert rc == kcf.EUNSUPPORTED and b"scratch" in L.kcf_last_error()
    assert L.kcf_filter_favre_noalloc(C.byref(g), fa, 1, kcf._ptr(rho), kcf._ptr(u), oa, None,
                                      st, 99, None) in (kcf.EINVAL, kcf.EUNSUPPORTED)

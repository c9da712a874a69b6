"""C-ABI checks that need no GPU: the library loads, exports every declared symbol, and its
host-side logic (filter taps, argument checks) agrees with the oracle's definitions."""
import ctypes as C
import glob
import os
import re

import numpy as np
import pytest

from oracle import fields as F
from paper_2605_19796_amd import kcf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for hdr in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(hdr).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(kcf_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(kcf.LIB_PATH):
        pytest.skip("libkcf.so not built")
    return kcf.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/ but not exported"
    # the binding covers every declared function
    assert set(names) <= set(kcf.exported_symbols())


def test_version(L):
    assert L.kcf_version() >= 100


@pytest.mark.parametrize("kind,n", [(F.BOX, 2), (F.BOX, 4), (F.BOX, 8), (F.BOX, 16),
                                    (F.GAUSS, 1), (F.GAUSS, 2), (F.GAUSS, 4), (F.GAUSS, 8)])
def test_taps_match_oracle(L, kind, n):
    h = 2 * np.pi / 64
    w, R, m2 = kcf.filter_taps(kind, n, h)
    wo, Ro = F.filter_weights(kind, n)
    assert R == Ro
    assert np.array_equal(np.array(w, dtype=np.float32), wo.astype(np.float32))
    assert abs(m2 - F.second_moment(wo, h)) <= 1e-14 * F.second_moment(wo, h)


def test_taps_errors(L):
    buf = (C.c_float * 129)()
    R = C.c_int()
    m2 = C.c_double()
    assert L.kcf_filter_taps(kcf.BOX, 3, 0.1, buf, 129, C.byref(R), C.byref(m2)) == kcf.EINVAL
    assert L.kcf_filter_taps(kcf.BOX, 0, 0.1, buf, 129, C.byref(R), C.byref(m2)) == kcf.EINVAL
    assert L.kcf_filter_taps(kcf.GAUSS, 0, 0.1, buf, 129, C.byref(R), C.byref(m2)) == kcf.EINVAL
    assert L.kcf_filter_taps(7, 2, 0.1, buf, 129, C.byref(R), C.byref(m2)) == kcf.EINVAL
    assert L.kcf_filter_taps(kcf.BOX, 2, -1.0, buf, 129, C.byref(R), C.byref(m2)) == kcf.EINVAL
    assert L.kcf_filter_taps(kcf.GAUSS, 8, 0.1, buf, 5, C.byref(R), C.byref(m2)) == kcf.EINVAL
    assert b"small" in L.kcf_last_error()
    assert L.kcf_filter_taps(kcf.BOX, 2, 0.1, None, 129, C.byref(R), C.byref(m2)) == kcf.EINVAL


def test_null_context_is_rejected(L):
    g = kcf.Grid(8, 8, 8, 0.1)
    f = (kcf.Filter * 1)(kcf.Filter(kcf.BOX, 2))
    o = (kcf.Outputs * 1)()
    assert L.kcf_filter_favre(None, C.byref(g), f, 1, None, None, o, None, None) == kcf.EINVAL
    assert L.kcf_grad_closure(None, C.byref(g), None, None, None, 1.0, 0.1, None, None, None) == kcf.EINVAL
    assert L.kcf_input_stats(None, C.byref(g), None, None, None) == kcf.EINVAL
    assert L.kcf_ctx_set_stream(None, None) == kcf.EINVAL
    L.kcf_ctx_destroy(None)

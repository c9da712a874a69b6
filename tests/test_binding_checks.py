"""Argument checks of the Python binding, on the CPU: every wrapper checks tensor sizes against
the grid before anything reaches the library, so a mismatched buffer raises ValueError and no
kernel is launched. The context and network below are shells without a library handle; any
call into the library would fail with AttributeError instead of the ValueError expected."""
import pytest
import torch

from paper_2605_19796_amd import kcf


def shell_ctx():
    c = object.__new__(kcf.Context)
    c._lib = None
    c.handle = None
    c._children = []
    return c


def shell_mlp():
    m = object.__new__(kcf.MLP)
    m._lib = None
    m.handle = None
    return m


N = (4, 5, 6)
n = 4 * 5 * 6


def f(*shape):
    return torch.zeros(shape, dtype=torch.float32)


SIZE = "expected .* elements|expected an|expected a \\("


def test_filter_favre_sizes():
    c = shell_ctx()
    good = {"rho_bar": f(1, *N), "tau": f(6, *N)}
    with pytest.raises(ValueError, match="2 output sets"):
        c.filter_favre(f(*N), f(3, *N), 0.1, [(kcf.BOX, 2), (kcf.BOX, 4), (kcf.BOX, 8)],
                       [good, good])
    with pytest.raises(ValueError, match="1 to 4 filters"):
        c.filter_favre(f(*N), f(3, *N), 0.1, [(kcf.BOX, 2)] * 5, [good] * 5)
    with pytest.raises(ValueError, match=SIZE):
        c.filter_favre(f(*N), f(2, *N), 0.1, [(kcf.BOX, 2)], [good])  # u has 2 components
    with pytest.raises(ValueError, match=SIZE):
        c.filter_favre(f(*N), f(3, *N), 0.1, [(kcf.BOX, 2)], [{"tau": f(5, *N)}])
    with pytest.raises(ValueError, match=SIZE):
        c.filter_favre(f(*N), f(3, *N), 0.1, [(kcf.BOX, 2)], [{"grad": f(6, *N)}])
    with pytest.raises(ValueError, match="unknown output"):
        c.filter_favre(f(*N), f(3, *N), 0.1, [(kcf.BOX, 2)], [{"tau2": f(6, *N)}])
    with pytest.raises(ValueError, match="expected a \\(nz, ny, nx\\)"):
        c.filter_favre(f(n), f(3, *N), 0.1, [(kcf.BOX, 2)], [good])


def test_other_field_calls_sizes():
    c = shell_ctx()
    with pytest.raises(ValueError, match=SIZE):
        c.grad_closure(f(*N), f(3, *N), f(3, *N), 0.1, 0.4, 0.01, {})  # tau needs 6
    with pytest.raises(ValueError, match=SIZE):
        c.sgs_carrier(f(*N), f(3, *N), 0.1, (kcf.BOX, 2), f_sgs=f(26, *N))
    with pytest.raises(ValueError, match=SIZE):
        c.sgs_moment3(f(*N), f(3, *N), 0.1, (kcf.BOX, 2), m3=f(9, *N))
    with pytest.raises(ValueError, match=SIZE):
        c.sgs_moment3(f(*N), f(3, *N), 0.1, (kcf.BOX, 2), theta=f(2, *N))
    with pytest.raises(ValueError, match=SIZE):
        c.kc_mp(f(*N), f(3, *N), 0.1, (kcf.BOX, 2), 1e-3, m_sgs=f(9, *N))
    with pytest.raises(ValueError, match=SIZE):
        c.kc_mp(f(*N), f(3, *N), 0.1, (kcf.BOX, 2), 1e-3, omega_sgs=f(2, *N))
    with pytest.raises(ValueError, match=SIZE):
        c.input_stats(f(*N), f(1, *N), 0.1)
    with pytest.raises(ValueError, match=SIZE):
        c.reduce_check(f(10), f(11))


def test_mlp_sizes():
    m = shell_mlp()
    with pytest.raises(ValueError, match=SIZE):
        m.fit_norm(f(64, 13), f(64, 6))
    with pytest.raises(ValueError, match=SIZE):
        m.fit_norm(f(64, 14), f(63, 6))
    with pytest.raises(ValueError, match="batch"):
        m.train_step(f(64, 14), f(64, 6), None, 96, 1e-3)
    with pytest.raises(ValueError, match="indices"):
        m.grads(f(64, 14), f(64, 6), torch.zeros(16, dtype=torch.int32), 32)
    with pytest.raises(ValueError, match=SIZE):
        m.predict(f(64, 6))
    with pytest.raises(ValueError, match=SIZE):
        m.infer_field(f(*N), f(3, *N), 0.1, 0.4, 0.01, tau_out=f(5, *N))
    with pytest.raises(ValueError, match=SIZE):
        m.infer_field(f(*N), f(3, *N), 0.1, 0.4, 0.01, tau_out=f(6, *N),
                      mask_out=torch.zeros(n // 16, dtype=torch.int16))  # needs ceil(n/16)
    with pytest.raises(ValueError, match=SIZE):
        kcf.mlp_features(shell_ctx(), f(*N), f(3, *N), f(5, *N), 0.1, 0.4)
    with pytest.raises(ValueError, match="ncol"):
        kcf.column_stats(shell_ctx(), f(10, 40))

"""Pins of the D3Q27 SGS-carrier oracle (CPU)."""
import math

import numpy as np
import pytest

from oracle import carrier as K
from oracle import fields as F
from paper_2605_19796_amd import synth


def test_lattice_weights_and_quadrature():
    xi, xh, w = K.lattice()
    assert xi.shape == (27, 3) and abs(w.sum() - 1.0) < 1e-15
    # D1Q3 Gauss-Hermite: the weights integrate 1, xh_a xh_b = delta_ab, xh^4 = 3 per direction
    assert np.allclose(np.einsum("i,ia,ib->ab", w, xh, xh), np.eye(3), atol=1e-15)
    assert np.allclose(np.einsum("i,ia->a", w, xh ** 4), 3.0, atol=1e-14)


def test_equilibrium_is_the_lattice_formula():
    """The normalised form equals eq. discrete_equilibrium in lattice units (xi in {-1, 0, 1},
    theta_R = 1/3) for velocities given in units of sqrt(theta_R)."""
    rng = np.random.default_rng(1)
    rho = 1 + 0.2 * rng.standard_normal(50)
    u = 0.3 * rng.standard_normal((3, 50))
    xi, _, w = K.lattice()
    th = 1.0 / 3.0
    ul = u * math.sqrt(th)
    ref = np.empty((27, 50))
    for i in range(27):
        f = w[i] * rho
        for a in range(3):
            c = xi[i, a]
            f = f * (1 + c * ul[a] / th + (c * c - th) * ul[a] ** 2 / (2 * th * th))
        ref[i] = f
    assert np.max(np.abs(K.equilibrium(rho, u) - ref)) < 1e-15
    m0, m1, m2 = K.moments(ref)
    assert np.allclose(m0, rho, rtol=1e-14)
    assert np.allclose(m1, rho * u, atol=1e-14)
    assert np.allclose(m2, rho * (np.eye(3)[:, :, None] + u[:, None] * u[None]), atol=1e-14)


@pytest.mark.parametrize("kind,nd", [(F.BOX, 4), (F.GAUSS, 2)])
def test_carrier_moments_are_conserved_and_tau(kind, nd):
    """Zeroth and first moments of f_sgs vanish, the second moment is tau (computed by the
    field oracle from the filtered products, independently of the populations)."""
    rho, u = synth.random_fields((12, 10, 14), seed=3, rho_amp=0.2)
    r = K.carrier(rho, u, kind, nd)
    m0, m1, m2 = K.moments(r["f_sgs"])
    scale = np.max(np.abs(r["tau"]))
    assert np.max(np.abs(m0)) < 1e-13 * scale
    assert np.max(np.abs(m1)) < 1e-13 * scale
    _, _, tau = F.filter_favre(rho, u, F.filter_weights(kind, nd)[0])
    assert np.max(np.abs(m2 - tau)) < 1e-12 * scale
    # the second-order reconstruction carries the same three moments, but not the rest
    h0, h1, h2 = K.moments(r["f_h2"])
    assert np.max(np.abs(h0)) < 1e-15 and np.max(np.abs(h1)) < 1e-15
    assert np.max(np.abs(h2 - tau)) < 1e-12 * scale
    st = K.carrier_stats(r["f_sgs"], r["f_h2"])
    assert 1e-6 < st["rel_err"] < 1.0


def test_carrier_vanishes_without_subgrid_variation():
    rho = np.full((8, 8, 8), 1.3)
    u = np.zeros((3, 8, 8, 8))
    u[0], u[1], u[2] = 0.2, -0.1, 0.05
    assert np.max(np.abs(K.carrier(rho, u, F.BOX, 4)["f_sgs"])) < 1e-15
    # uniform velocity, variable density: bar(rho g(U)) = rho_bar g(U)
    rho2, _ = synth.random_fields((8, 8, 8), seed=4, rho_amp=0.3)
    assert np.max(np.abs(K.carrier(rho2, u, F.GAUSS, 2)["f_sgs"])) < 1e-15


def test_reconstruction_exact_for_one_component_velocity():
    """rho = 1 and u = (u_x, 0, 0): the equilibrium is quadratic in u_x, so the carrier has no
    moment above the second and the Hermite reconstruction is exact."""
    n = 16
    X, Y, Z = synth.grid_coords(n)
    rho = np.ones((n, n, n))
    u = np.zeros((3, n, n, n))
    u[0] = 0.3 * np.cos(X + 2 * Y - Z + 0.4)
    r = K.carrier(rho, u, F.BOX, 4)
    assert np.max(np.abs(r["f_sgs"])) > 1e-4
    assert np.max(np.abs(r["f_sgs"] - r["f_h2"])) < 1e-15


def test_carrier_separable_equals_direct():
    rho, u = synth.random_fields((8, 8, 8), seed=5, rho_amp=0.2)
    a = K.carrier(rho, u, F.BOX, 2)["f_sgs"]
    b = K.carrier(rho, u, F.BOX, 2, separable=False)["f_sgs"]
    assert np.max(np.abs(a - b)) < 1e-15


def test_hermite_energies_of_basis_functions():
    """A single basis term w_i P_a P_b P_c has all its energy n_a n_b n_c in order a + b + c."""
    _, xh, w = K.lattice()
    P = [np.ones(27), None, None]
    nrm = [1.0, 1.0, 0.5]
    for a, b, c in [(0, 0, 0), (1, 0, 0), (0, 2, 0), (1, 1, 1), (2, 0, 2), (2, 2, 2)]:
        fac = []
        for deg, dim in zip((a, b, c), range(3)):
            x = xh[:, dim]
            fac.append([np.ones(27), x, 0.5 * (x * x - 1.0)][deg])
        f = (w * fac[0] * fac[1] * fac[2])[:, None]
        e = K.hermite_energies(f)
        expect = np.zeros(7)
        expect[a + b + c] = nrm[a] * nrm[b] * nrm[c]
        assert np.allclose(e, expect, atol=1e-14), (a, b, c, e)


def test_hermite_energies_of_the_carrier():
    """Parseval under the lattice weights; no energy in orders 0 and 1 (vanishing zeroth and
    first moments); order 2 carries sum_a tau_aa^2 / 2 + sum_{a<b} tau_ab^2 with tau from the
    field oracle; the reconstruction holds exactly the order-2 part."""
    rho, u = synth.random_fields((10, 12, 8), seed=6, rho_amp=0.2)
    r = K.carrier(rho, u, F.GAUSS, 2)
    _, _, w = K.lattice()
    e = K.hermite_energies(r["f_sgs"])
    total = float(np.mean(np.sum(r["f_sgs"] ** 2 / w[:, None, None, None], 0)))
    assert abs(e.sum() - total) < 1e-13 * total
    assert e[0] < 1e-25 * total and e[1] < 1e-25 * total
    _, _, tau = F.filter_favre(rho, u, F.filter_weights(F.GAUSS, 2)[0])
    e2 = float(np.mean(0.5 * (tau[0, 0] ** 2 + tau[1, 1] ** 2 + tau[2, 2] ** 2)
                       + tau[0, 1] ** 2 + tau[0, 2] ** 2 + tau[1, 2] ** 2))
    assert abs(e[2] - e2) < 1e-12 * e2
    assert min(e[3], e[4]) > 0
    h = K.hermite_energies(r["f_h2"])
    assert abs(h[2] - e[2]) < 1e-12 * e[2] and h.sum() - h[2] < 1e-25 * total
    d = K.hermite_energies(r["f_sgs"] - r["f_h2"])
    assert abs(d.sum() - e[3:].sum()) < 1e-12 * total and d[2] < 1e-25 * total


def test_pointwise_carrier_equals_field_carrier():
    """Direct 3-D sums at sampled points agree with the separable full-field carrier."""
    rho, u = synth.random_fields((9, 11, 10), seed=7, rho_amp=0.2)
    r = K.carrier(rho, u, F.GAUSS, 2)
    pts = np.array([(0, 0, 0), (8, 10, 9), (4, 5, 3), (2, 9, 7)])
    fs, fh = K.carrier_at(rho, u, F.GAUSS, 2, pts)
    for n, (k, j, i) in enumerate(pts):
        assert np.max(np.abs(fs[n] - r["f_sgs"][:, k, j, i])) < 1e-15
        assert np.max(np.abs(fh[n] - r["f_h2"][:, k, j, i])) < 1e-15


def test_carrier_stats_on_literal_populations():
    """carrier_stats on hand-built populations: <sum_i f_i^2> is a mean over points of the
    sum over the 27 populations (two points with 27 values 1 and 27 values 3 give
    (27 + 243) / 2 = 135); err_l2 = 0 when f_h2 = f_sgs, rel_err = 1 when f_h2 = 0,
    rel_err = 1/2 when f_h2 = f_sgs / 2, and err_l2 = 27 * (1^2 + 2^2) / 2 for f_h2 = 0 and 1
    on the two points."""
    f = np.empty((27, 2))
    f[:, 0], f[:, 1] = 1.0, 3.0
    st = K.carrier_stats(f, f.copy())
    assert st["sgs_l2"] == 135.0 and st["err_l2"] == 0.0 and st["rel_err"] == 0.0
    assert K.carrier_stats(f, np.zeros_like(f))["rel_err"] == 1.0
    assert abs(K.carrier_stats(f, 0.5 * f)["rel_err"] - 0.5) < 1e-15
    fh = np.empty_like(f)
    fh[:, 0], fh[:, 1] = 0.0, 1.0
    assert K.carrier_stats(f, fh)["err_l2"] == 27 * (1.0 + 4.0) / 2
    assert K.carrier_stats(np.zeros_like(f), np.zeros_like(f))["rel_err"] == 0.0

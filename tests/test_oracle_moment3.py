"""Pins of the third-order SGS moment and Favre temperature oracle (CPU)."""
import numpy as np
import pytest

from oracle import carrier as K
from oracle import fields as F
from oracle import moment3 as M
from paper_2605_19796_amd import synth


@pytest.mark.parametrize("kind,nd", [(F.BOX, 4), (F.GAUSS, 2)])
def test_single_mode_closed_form(kind, nd):
    """rho = 1, u_x = a cos(k x + phi): cos^3 = (3 cos + cos 3)/4 through the transfer
    function G gives m3_xxx = a^3/4 [3 (G(k) - G(k)^3) cos + (G(3k) - G(k)^3) cos 3(.)]; every
    other component vanishes."""
    n = 24
    X, Y, Z = synth.grid_coords(n)
    h = 2 * np.pi / n
    a, k, phi = 0.4, 2, 0.3
    rho = np.ones((n, n, n))
    u = np.zeros((3, n, n, n))
    u[0] = a * np.cos(k * X + phi) + 0 * Y + 0 * Z
    m3 = M.moment3(rho, u, kind, nd)["m3"]
    g1, g3 = F.transfer(kind, nd, k * h), F.transfer(kind, nd, 3 * k * h)
    c1 = np.cos(k * X + phi) + 0 * Y + 0 * Z
    c3 = np.cos(3 * (k * X + phi)) + 0 * Y + 0 * Z
    ref = a ** 3 / 4 * (3 * (g1 - g1 ** 3) * c1 + (g3 - g1 ** 3) * c3)
    assert np.max(np.abs(m3[0] - ref)) < 1e-15
    assert np.max(np.abs(m3[1:])) < 1e-15


def test_galilean_shift_rule():
    rho, u = synth.random_fields((10, 12, 14), seed=21, rho_amp=0.2)
    U = np.array([0.3, -0.2, 0.15])
    a = M.moment3(rho, u, F.BOX, 4)["m3"]
    b = M.moment3(rho, u + U[:, None, None, None], F.BOX, 4)["m3"]
    _, _, tau = F.filter_favre(rho, u, F.filter_weights(F.BOX, 4)[0])
    for c, (i, j, k) in enumerate(M.TRIPLES):
        shift = U[i] * tau[j, k] + U[j] * tau[i, k] + U[k] * tau[i, j]
        assert np.max(np.abs(b[c] - a[c] - shift)) < 1e-14, (i, j, k)


def test_uniform_velocity_gives_zero():
    rho, _ = synth.random_fields((8, 10, 9), seed=22, rho_amp=0.3)
    u = np.zeros((3,) + rho.shape)
    u[0], u[1], u[2] = 0.3, -0.1, 0.2
    assert np.max(np.abs(M.moment3(rho, u, F.GAUSS, 2)["m3"])) < 1e-15


def test_mixed_components_are_the_carrier_order3_coefficients():
    """The order-3 Hermite coefficients of the carrier oracle's f_sgs (filtered equilibria,
    projected by lattice quadrature) are the mixed components of m3."""
    rho, u = synth.random_fields((9, 10, 11), seed=23, rho_amp=0.2)
    m3 = M.moment3(rho, u, F.GAUSS, 2)["m3"]
    d = K.hermite_coefficients(K.carrier(rho, u, F.GAUSS, 2)["f_sgs"])
    # exponents (a, b, c) of x, y, z for each mixed triple
    for c, (i, j, k) in enumerate(M.TRIPLES):
        e = [0, 0, 0]
        for idx in (i, j, k):
            e[idx] += 1
        if max(e) > 2:
            continue  # xxx, yyy, zzz are outside the D3Q27 product basis
        ref = d[e[0], e[1], e[2]]
        assert np.max(np.abs(ref - m3[c])) < 1e-13 * np.max(np.abs(m3[c])), (i, j, k)


def test_favre_temperature_cases():
    rho, _ = synth.random_fields((8, 9, 10), seed=24, rho_amp=0.3)
    rho = rho.astype(np.float64)
    th = np.full(rho.shape, 1.7)
    assert np.max(np.abs(M.favre_temperature(rho, th, F.BOX, 4) - 1.7)) < 1e-14
    # rho theta constant: theta_t = c / rho_bar
    tt = M.favre_temperature(rho, 2.0 / rho, F.GAUSS, 2)
    rb = F.filter_separable(rho, F.filter_weights(F.GAUSS, 2)[0])
    assert np.max(np.abs(tt - 2.0 / rb)) < 1e-14
    th2, _ = synth.random_fields((8, 9, 10), seed=25, rho_amp=0.2)
    a = M.favre_temperature(rho, th2, F.BOX, 2)
    b = M.favre_temperature(rho, th2, F.BOX, 2, separable=False)
    assert np.max(np.abs(a - b)) < 1e-14


def test_pointwise_equals_field():
    rho, u = synth.random_fields((9, 11, 10), seed=26, rho_amp=0.2)
    th, _ = synth.random_fields((9, 11, 10), seed=27, rho_amp=0.1)
    r = M.moment3(rho, u, F.BOX, 4)
    tt = M.favre_temperature(rho, th, F.BOX, 4)
    pts = np.array([(0, 0, 0), (8, 10, 9), (3, 4, 5)])
    m3, t = M.moment3_at(rho, u, th, F.BOX, 4, pts)
    for n, (k, j, i) in enumerate(pts):
        assert np.max(np.abs(m3[n] - r["m3"][:, k, j, i])) < 1e-15
        assert abs(t[n] - tt[k, j, i]) < 1e-15

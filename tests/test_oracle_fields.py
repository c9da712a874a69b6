"""Pins of the FP64 field oracle against facts fixed by the paper and by mathematics.

Each test is chosen so that a plausible slip in the oracle (a wrong tap weight, a
dropped rho_bar, a sign, a transposed gradient, a wrong FD offset) fails one of them.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import fields as F
from paper_2605_19796_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def box_transfer_closed(n, theta):
    """sin(n theta/2) / (n tan(theta/2)), with the theta -> 0 limit 1."""
    theta = np.asarray(theta, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        v = np.sin(n * theta / 2.0) / (n * np.tan(theta / 2.0))
    return np.where(np.abs(theta) < 1e-300, 1.0, v)


# ------------------------------------------------------------------ weights
@pytest.mark.parametrize("n", [2, 4, 8, 16])
def test_box_weights_and_moment(n):
    w, R = F.filter_weights(F.BOX, n)
    assert R == n // 2 and len(w) == n + 1
    assert abs(w.sum() - 1.0) < 1e-15
    assert w[0] == w[-1] == 0.5 / n and np.all(w[1:-1] == 1.0 / n)
    h = 0.3
    # trapezoidal top-hat: M2 = Delta^2/12 + h^2/6
    assert abs(F.second_moment(w, h) - ((n * h) ** 2 / 12 + h * h / 6)) < 1e-14


def test_box_transfer_closed_form():
    theta = np.linspace(0.0, math.pi, 41)
    for n in (2, 4, 8, 16):
        assert np.allclose(F.transfer(F.BOX, n, theta), box_transfer_closed(n, theta), atol=1e-14)


def test_gauss_weights_and_moment():
    # sampled exp(-6 m^2/n^2), R = ceil(1.5 n); M2/h^2 = 0.3212, 4/3, 16/3, 64/3 for n = 2, 4, 8, 16
    expect = {2: 0.3212, 4: 4.0 / 3.0, 8: 16.0 / 3.0, 16: 64.0 / 3.0}
    for n, m2 in expect.items():
        w, R = F.filter_weights(F.GAUSS, n)
        assert R == math.ceil(1.5 * n)
        assert abs(w.sum() - 1.0) < 1e-15
        m = np.arange(-R, R + 1)
        ratio = w / w[R]
        assert np.allclose(ratio, np.exp(-6.0 * m * m / n ** 2), rtol=1e-13)
        tol = 5e-5 if n == 2 else 1e-5
        assert abs(F.second_moment(w, 1.0) - m2) < tol * m2


def test_weights_reject():
    with pytest.raises(ValueError):
        F.filter_weights(F.BOX, 3)
    with pytest.raises(ValueError):
        F.filter_weights(F.BOX, 0)


# ------------------------------------------------------------------ brute force vs separable
@pytest.mark.parametrize("shape,kind,n", [((8, 8, 8), F.BOX, 4), ((8, 8, 8), F.GAUSS, 2),
                                          ((12, 12, 12), F.BOX, 8), ((12, 12, 12), F.GAUSS, 4),
                                          ((6, 10, 8), F.BOX, 2), ((8, 8, 8), F.BOX, 16)])
def test_direct_equals_separable(shape, kind, n):
    rng = np.random.default_rng(7)
    a = rng.standard_normal(shape)
    w, R = F.filter_weights(kind, n)
    d = F.filter_direct(a, w)
    s = F.filter_separable(a, w)
    assert np.max(np.abs(d - s)) <= 1e-13 * np.max(np.abs(d))


def test_filter_is_circular_convolution():
    # The separable pass must equal the product of transfer functions in Fourier space.
    rng = np.random.default_rng(3)
    a = rng.standard_normal((8, 12, 10))
    w, R = F.filter_weights(F.GAUSS, 2)
    out = F.filter_separable(a, w)
    spec = np.fft.fftn(a)
    for ax, nn in zip((0, 1, 2), a.shape):
        theta = 2 * np.pi * np.fft.fftfreq(nn)
        g = np.sum(w[None, :] * np.cos(np.outer(theta, np.arange(-R, R + 1))), axis=1)
        shape = [1, 1, 1]
        shape[ax] = nn
        spec = spec * g.reshape(shape)
    assert np.allclose(np.fft.ifftn(spec).real, out, atol=1e-13)


# ------------------------------------------------------------------ invariants
def test_constant_field():
    rho = np.full((8, 8, 8), 1.7)
    u = np.stack([np.full((8, 8, 8), c) for c in (0.3, -0.1, 0.25)])
    for kind, n in ((F.BOX, 4), (F.GAUSS, 2)):
        out = F.full_path(rho, u, kind, n, 2 * np.pi / 8)
        assert np.allclose(out["rho_bar"], 1.7, rtol=1e-14)
        for i, c in enumerate((0.3, -0.1, 0.25)):
            assert np.allclose(out["ut"][i], c, rtol=1e-13)
        for key in ("tau", "G", "tau_gm", "tau_smag", "k_sgs"):
            assert np.max(np.abs(out[key])) < 1e-14
        # nu_t = C_nu Delta sqrt(k_sgs): the square root lifts round-off to ~1e-8
        assert np.max(out["nu_t"]) < 0.02 * out["delta"] * 1e-7


def test_uniform_velocity_variable_density():
    rho, _ = synth.random_fields((8, 8, 8), seed=11, rho_amp=0.3, dtype=np.float64)
    U = (0.2, -0.05, 0.1)
    u = np.stack([np.full((8, 8, 8), c) for c in U])
    w, _ = F.filter_weights(F.GAUSS, 2)
    rho_bar, ut, tau = F.filter_favre(rho, u, w)
    for i, c in enumerate(U):
        assert np.allclose(ut[i], c, rtol=1e-13)
    assert np.max(np.abs(tau)) < 1e-15
    # bar(rho u_i) = rho_bar ut_i
    assert np.allclose(F.filter_separable(rho * u[0], w), rho_bar * ut[0], rtol=1e-14)


def test_tau_symmetric_psd_galilean():
    rho, u = synth.random_fields((10, 12, 8), seed=5, rho_amp=0.5, dtype=np.float64)
    h = 0.2
    for kind, n in ((F.BOX, 4), (F.GAUSS, 4), (F.BOX, 2)):
        w, _ = F.filter_weights(kind, n)
        rho_bar, ut, tau = F.filter_favre(rho, u, w)
        assert np.max(np.abs(tau - np.swapaxes(tau, 0, 1))) < 1e-15
        # positive weights and rho > 0 make tau = sum w rho (u - ut)(u - ut)^T semidefinite
        ev = np.linalg.eigvalsh(np.moveaxis(tau, (0, 1), (-2, -1)))
        assert ev.min() > -1e-15 * ev.max()
        assert np.all(np.trace(tau) > 0)
        U = np.array([0.7, -0.4, 0.3])
        rho_b2, ut2, tau2 = F.filter_favre(rho, u + U[:, None, None, None], w)
        assert np.max(np.abs(tau2 - tau)) < 1e-13
        G1 = F.grad2(ut, h)
        G2 = F.grad2(ut2, h)
        assert np.max(np.abs(G2 - G1)) < 1e-12


def test_favre_weighting_is_by_density():
    # rho concentrated where u is large: the Favre velocity differs from the plain filtered u.
    n = 8
    rho, u = synth.single_mode(n, (1, 0, 0), (0.0, 0.5, 0.0), rho_b=0.5, qvec=(1, 0, 0))
    w, _ = F.filter_weights(F.BOX, 2)
    _, ut, _ = F.filter_favre(rho, u, w)
    # ut_y = bar(rho u_y)/rho_bar; check at one point by hand
    k, j, i = 0, 0, 0
    xs = [(i - 1) % n, i, (i + 1) % n]
    ws = [0.25, 0.5, 0.25]
    num = sum(wx * rho[k, j, x] * u[1, k, j, x] for wx, x in zip(ws, xs))
    den = sum(wx * rho[k, j, x] for wx, x in zip(ws, xs))
    assert abs(ut[1, k, j, i] - num / den) < 1e-15


# ------------------------------------------------------------------ closed forms
@pytest.mark.parametrize("kind,nd", [(F.BOX, 4), (F.GAUSS, 2), (F.BOX, 2)])
def test_single_mode_closed_form(kind, nd):
    n = 16
    h = 2 * np.pi / n
    kv = np.array([1, 2, 3])
    av = np.array([0.3, -0.2, 0.1])
    qv = np.array([2, -1, 1])
    b = 0.3
    rho, u = synth.single_mode(n, kv, av, phase=0.4, rho_b=b, qvec=qv, rho_phase=-0.7)
    out = F.full_path(rho, u, kind, nd, h)

    def T(kvec):
        kvec = np.asarray(kvec)
        if kind == F.BOX:
            return float(np.prod(box_transfer_closed(nd, kvec * h)))
        return float(np.prod(F.transfer(kind, nd, kvec * h)))

    X, Y, Z = synth.grid_coords(n)
    phi = kv[0] * X + kv[1] * Y + kv[2] * Z + 0.4
    psi = qv[0] * X + qv[1] * Y + qv[2] * Z - 0.7
    rho_bar = 1 + b * T(qv) * np.cos(psi)
    m = [av[i] * (T(kv) * np.cos(phi) + 0.5 * b * (T(qv + kv) * np.cos(psi + phi)
                                                   + T(qv - kv) * np.cos(psi - phi))) for i in range(3)]
    for i in range(3):
        for j in range(3):
            p = av[i] * av[j] * (0.5 + 0.5 * T(2 * kv) * np.cos(2 * phi) + 0.5 * b * T(qv) * np.cos(psi)
                                 + 0.25 * b * (T(qv + 2 * kv) * np.cos(psi + 2 * phi)
                                               + T(qv - 2 * kv) * np.cos(psi - 2 * phi)))
            tau = p - m[i] * m[j] / rho_bar
            assert np.max(np.abs(out["tau"][i, j] - tau)) < 1e-14
    assert np.max(np.abs(out["rho_bar"] - rho_bar)) < 1e-14
    for i in range(3):
        assert np.max(np.abs(out["ut"][i] - m[i] / rho_bar)) < 1e-14


def test_single_mode_gradient_closed_form():
    # rho = 1: ut_i = a_i T(k) cos(phi), G_ij = -a_i T(k) sin(phi) sin(k_j h)/h (eq. fd).
    n = 16
    h = 2 * np.pi / n
    kv = np.array([1, -2, 3])
    av = np.array([0.2, 0.1, -0.3])
    rho, u = synth.single_mode(n, kv, av, phase=0.2)
    out = F.full_path(rho, u, F.BOX, 4, h)
    Tk = float(np.prod(box_transfer_closed(4, kv * h)))
    X, Y, Z = synth.grid_coords(n)
    phi = kv[0] * X + kv[1] * Y + kv[2] * Z + 0.2
    for i in range(3):
        for j in range(3):
            g = -av[i] * Tk * np.sin(phi) * np.sin(kv[j] * h) / h
            assert np.max(np.abs(out["G"][i, j] - g)) < 1e-14


def test_taylor_green_closed_form():
    gold = json.load(open(os.path.join(GOLD, "tgv_closed_form.json")))
    n, u0, nd = 32, 0.1, 4
    h = 2 * np.pi / n
    rho, u = synth.taylor_green(n, u0, dtype=np.float64)
    st = F.input_stats(rho, u, h)
    assert abs(st["ek"] - gold["ek_over_u0sq"] * u0 ** 2) < 1e-9 * u0 ** 2
    # sixth-order FD on wavenumber-1 modes scales each derivative by the modified wavenumber
    th = h
    kmod = (45 * np.sin(th) - 9 * np.sin(2 * th) + np.sin(3 * th)) / (30 * h)
    assert abs(st["enstrophy"] - gold["enstrophy_over_u0sq_continuum"] * u0 ** 2 * kmod ** 2) < 1e-9 * u0 ** 2
    assert abs(kmod - 1.0) < 1e-6
    out = F.full_path(rho, u, F.BOX, nd, h)
    g1 = float(box_transfer_closed(nd, h))
    g2 = float(box_transfer_closed(nd, 2 * h))
    X, Y, Z = synth.grid_coords(n)
    ux = u0 * np.sin(X) * np.cos(Y) * np.cos(Z)
    uy = -u0 * np.cos(X) * np.sin(Y) * np.cos(Z)
    pxx = u0 ** 2 / 8 * (1 - g2 * np.cos(2 * X)) * (1 + g2 * np.cos(2 * Y)) * (1 + g2 * np.cos(2 * Z))
    pyy = u0 ** 2 / 8 * (1 + g2 * np.cos(2 * X)) * (1 - g2 * np.cos(2 * Y)) * (1 + g2 * np.cos(2 * Z))
    pxy = -u0 ** 2 / 8 * g2 * g2 * np.sin(2 * X) * np.sin(2 * Y) * (1 + g2 * np.cos(2 * Z))
    g6 = g1 ** 6
    assert np.max(np.abs(out["tau"][0, 0] - (pxx - g6 * ux ** 2))) < 1e-15
    assert np.max(np.abs(out["tau"][1, 1] - (pyy - g6 * uy ** 2))) < 1e-15
    assert np.max(np.abs(out["tau"][0, 1] - (pxy - g6 * ux * uy))) < 1e-15
    assert np.max(np.abs(out["tau"][2])) < 1e-18


def test_gradient_model_taylor_limit():
    # Single shear mode u_x = cos(y): <tau_xx>/<tau_gm_xx> -> 1 with O((k h)^2) error.
    errs = []
    for n in (32, 64):
        h = 2 * np.pi / n
        rho, u = synth.single_mode(n, (0, 1, 0), (1.0, 0.0, 0.0))
        out = F.full_path(rho, u, F.BOX, 4, h)
        ratio = np.mean(out["tau"][0, 0]) / np.mean(out["tau_gm"][0, 0])
        errs.append(abs(ratio - 1))
    assert errs[0] < 0.05
    assert 3.5 < errs[0] / errs[1] < 4.5


# ------------------------------------------------------------------ closures
def test_closures_pure_shear():
    gold = json.load(open(os.path.join(GOLD, "paper_constants.json")))
    assert F.DEFAULT_PARAMS["c_s"] == gold["c_s_smagorinsky"]
    assert F.DEFAULT_PARAMS["c_nu"] == gold["c_nu_kcrb"]
    gam, rb, delta, m2 = 0.7, 1.3, 0.5, 0.03
    G = np.zeros((3, 3, 1))
    G[0, 1] = gam  # d_y u_x
    tau = np.zeros((3, 3, 1))
    tau[0, 0], tau[1, 1], tau[2, 2] = 0.02, 0.01, 0.005
    rho_bar = np.array([rb])
    c = F.closures(rho_bar, G, tau, delta, m2)
    assert abs(c["tau_gm"][0, 0, 0] - rb * m2 * gam ** 2) < 1e-15  # Taylor form: G G^T
    assert np.count_nonzero(c["tau_gm"]) == 1
    c1 = F.closures(rho_bar, G, tau, delta, m2, dict(gm_form=1))
    assert abs(c1["tau_gm"][1, 1, 0] - rb * m2 * gam ** 2) < 1e-15  # printed form: G^T G
    c2 = F.closures(rho_bar, G, tau, delta, m2, dict(m2_mode=1))
    assert abs(c2["tau_gm"][0, 0, 0] - rb * delta ** 2 / 12 * gam ** 2) < 1e-15
    cs = 0.11
    assert abs(c["tau_smag"][0, 1, 0] + rb * (cs * delta) ** 2 * abs(gam) * gam) < 1e-15
    assert abs(c["tau_smag"][0, 0, 0]) < 1e-18
    k = 0.035 / (2 * rb)
    assert abs(c["k_sgs"][0] - k) < 1e-16
    assert abs(c["nu_t"][0] - 0.02 * delta * math.sqrt(k)) < 1e-16
    assert abs(c["omega_t"][0] - 1.0 / (0.02 * delta * math.sqrt(k))) < 1e-12
    # reference density rho0 = 1 of the operational form
    c3 = F.closures(rho_bar, G, tau, delta, m2, dict(ksgs_rho_ref=1))
    assert abs(c3["k_sgs"][0] - 0.035 / 2) < 1e-16
    # molecular clip and shifted rate: (max(nu, nu_t)/theta + dt/2)^-1
    c4 = F.closures(rho_bar, G, tau, delta, m2, dict(nu_mol=1.0, theta=1 / 3, dt=1.0))
    assert abs(c4["omega_t"][0] - 1.0 / (3.0 + 0.5)) < 1e-15


def test_smagorinsky_is_deviatoric_and_dissipative():
    rng = np.random.default_rng(2)
    G = rng.standard_normal((3, 3, 50))
    tau = np.zeros((3, 3, 50))
    c = F.closures(np.ones(50), G, tau, 0.3, 0.01)
    tr = c["tau_smag"][0, 0] + c["tau_smag"][1, 1] + c["tau_smag"][2, 2]
    assert np.max(np.abs(tr)) < 1e-15
    S, _ = F.strain_rotation(G)
    diss = -np.einsum("ij...,ij...->...", c["tau_smag"], S)
    assert np.all(diss >= -1e-15)


# ------------------------------------------------------------------ statistics
def test_pearson_and_dissipation():
    rng = np.random.default_rng(9)
    a = rng.standard_normal(1000)
    assert abs(F.pearson(a, a) - 1) < 1e-14
    assert abs(F.pearson(a, -2 * a + 3) + 1) < 1e-14
    b = rng.standard_normal(1000)
    assert abs(F.pearson(a, b) - np.corrcoef(a, b)[0, 1]) < 1e-13
    # tau = -alpha S gives pi = alpha <S:S>
    G = rng.standard_normal((3, 3, 4, 5, 6))
    S, _ = F.strain_rotation(G)
    st = F.width_stats(np.ones((4, 5, 6)), np.zeros((3, 4, 5, 6)), -0.5 * S, G, -0.25 * S)
    ss = np.mean(np.einsum("ij...,ij...->...", S, S))
    assert abs(st["pi"] - 0.5 * ss) < 1e-14
    assert abs(st["pi_gm"] - 0.25 * ss) < 1e-14
    assert all(abs(r - 1) < 1e-12 for r in st["corr_tau_gm"])


def test_sampled_points_match_full_field():
    rho, u = synth.random_fields((12, 10, 14), seed=21, dtype=np.float32)
    h = 0.1
    for kind, nd in ((F.BOX, 4), (F.GAUSS, 2)):
        full = F.full_path(rho, u, kind, nd, h)
        pts = np.array([[0, 0, 0], [11, 9, 13], [5, 3, 7], [6, 0, 13]])
        sp = F.sampled_points(rho, u, kind, nd, h, pts)
        for idx, (k, j, i) in enumerate(pts):
            assert abs(sp["rho_bar"][idx] - full["rho_bar"][k, j, i]) < 1e-14
            assert np.max(np.abs(sp["tau"][idx] - full["tau"][:, :, k, j, i])) < 1e-14
            assert np.max(np.abs(sp["G"][idx] - full["G"][:, :, k, j, i])) < 1e-12
            assert np.max(np.abs(sp["tau_gm"][idx] - full["tau_gm"][:, :, k, j, i])) < 1e-14
            assert abs(sp["k_sgs"][idx] - full["k_sgs"][k, j, i]) < 1e-14


def test_q_criterion_cases():
    """Solid-body rotation has Q = |W|^2 / 2 = omega^2 / 2 > 0, pure strain Q = -|S|^2 / 2,
    and in general Q = -G_ij G_ji / 2."""
    om = 0.7
    G = np.zeros((3, 3, 1))
    G[0, 1, 0], G[1, 0, 0] = -om, om  # u = omega x (0, 0, 1) x r
    assert abs(F.q_criterion(G)[0] - om * om) < 1e-15  # |W|_F^2 = 2 om^2
    Gs = np.zeros((3, 3, 1))
    Gs[0, 0, 0], Gs[1, 1, 0], Gs[2, 2, 0] = 1.0, -0.4, -0.6
    assert abs(F.q_criterion(Gs)[0] + 0.5 * (1.0 + 0.16 + 0.36)) < 1e-15
    rng = np.random.default_rng(3)
    Gr = rng.standard_normal((3, 3, 5))
    assert np.allclose(F.q_criterion(Gr), -0.5 * np.einsum("ij...,ji...->...", Gr, Gr), atol=1e-14)


def test_resolved_energy_single_mode_closed_form():
    """rho = c (constant), u_i = a_i cos(k.x): rho_bar = c and ut_i = a_i G3(k) cos(k.x), so
    <rho_bar |ut|^2 / 2> = c G3(k)^2 |a|^2 / 4 (the mean of cos^2 over whole periods is 1/2).
    A dropped 1/2, a dropped rho_bar or the unfiltered velocity all fail this."""
    n = 16
    h = 2 * np.pi / n
    X, Y, Z = synth.grid_coords(n)
    kv = np.array([2, 1, 3])
    a = np.array([0.3, -0.2, 0.1])
    phi = kv[0] * X + kv[1] * Y + kv[2] * Z
    u = np.stack([a[i] * np.cos(phi) for i in range(3)])
    c = 2.0
    rho = np.full((n, n, n), c)
    for kind, nd in ((F.BOX, 4), (F.GAUSS, 2)):
        g3 = np.prod([F.transfer(kind, nd, kk * h) for kk in kv])
        st = F.full_path(rho, u, kind, nd, h)["stats"]
        assert abs(st["ke_resolved"] - c * g3 ** 2 * np.dot(a, a) / 4) < 1e-15
        assert abs(st["mean_rho_bar"] - c) < 1e-14

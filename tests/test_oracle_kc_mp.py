"""Pins of the a priori KC-MP oracle (CPU)."""
import numpy as np
import pytest

from oracle import fields as F
from oracle import kc_mp as KC
from paper_2605_19796_amd import synth


@pytest.mark.parametrize("kind,nd", [(F.BOX, 4), (F.GAUSS, 2)])
def test_shear_wave_with_density_wave(kind, nd):
    """rho = 1 + b cos(q z), u = (a cos(k z), 0, 0): only the xz pair of rho S is nonzero;
    with s_k = sin(k h)/h and the transfer function G,
    bar(rho S_xz) = -(a s_k / 2)(G(k) sin kz + b/2 (G(k+q) sin (k+q)z + G(k-q) sin (k-q)z)),
    rho_bar = 1 + b G(q) cos qz, bar(rho u_x) = a (G(k) cos kz + b/2 (G(k+q) cos (k+q)z
    + G(k-q) cos (k-q)z)), and S_t,xz is the central difference of their ratio along z."""
    n = 24
    h = 2 * np.pi / n
    a, b, k, q = 0.3, 0.25, 3, 2
    X, Y, Z = synth.grid_coords(n)
    rho = np.broadcast_to(1.0 + b * np.cos(q * Z), (n, n, n)).copy()
    u = np.zeros((3, n, n, n))
    u[0] = a * np.cos(k * Z) + 0 * X + 0 * Y
    nu, dt, theta = 0.01, 0.5, 1.0 / 3.0
    r = KC.kc_mp(rho, u, kind, nd, h, nu, dt, theta)
    G = lambda m: F.transfer(kind, nd, m * h)
    z = Z[:, 0, 0]
    sk = np.sin(k * h) / h
    rs = -(a * sk / 2) * (G(k) * np.sin(k * z) + b / 2 * (G(k + q) * np.sin((k + q) * z)
                                                          + G(k - q) * np.sin((k - q) * z)))
    rb = lambda zz: 1.0 + b * G(q) * np.cos(q * zz)
    mx = lambda zz: a * (G(k) * np.cos(k * zz) + b / 2 * (G(k + q) * np.cos((k + q) * zz)
                                                          + G(k - q) * np.cos((k - q) * zz)))
    ut = lambda zz: mx(zz) / rb(zz)
    st = (ut(z + h) - ut(z - h)) / (4 * h)
    tau_hat = nu / theta + dt / 2
    diff = -2 * theta * tau_hat * (rs - rb(z) * st)
    got = (r["m_sgs"] - r["tau"])[0, 2][:, 0, 0]
    assert np.max(np.abs(got - diff)) < 1e-15
    assert np.max(np.abs(r["rs_bar"][0, 2][:, 0, 0] - rs)) < 1e-15
    others = r["rs_bar"].copy()
    others[0, 2] = others[2, 0] = 0
    assert np.max(np.abs(others)) < 1e-15


def test_constant_density_and_zero_tau_hat():
    _, u = synth.random_fields((10, 12, 14), seed=41)
    rho = np.full((10, 12, 14), 1.3)
    h = 2 * np.pi / 14
    r = KC.kc_mp(rho, u, F.BOX, 4, h, nu=0.01, dt=1.0)
    assert np.max(np.abs(r["m_sgs"] - r["tau"])) < 1e-14 * np.max(np.abs(r["tau"]))
    rho2, _ = synth.random_fields((10, 12, 14), seed=42, rho_amp=0.2)
    r2 = KC.kc_mp(rho2, u, F.GAUSS, 2, h, nu=0.0, dt=0.0)
    assert np.max(np.abs(r2["m_sgs"] - r2["tau"])) == 0.0
    r3 = KC.kc_mp(rho2, u, F.GAUSS, 2, h, nu=0.01, dt=0.0)
    assert np.max(np.abs(r3["m_sgs"] - r3["tau"])) > 1e-6 * np.max(np.abs(r3["tau"]))


def test_velocity_shift_invariance():
    rho, u = synth.random_fields((10, 11, 12), seed=43, rho_amp=0.2)
    h = 2 * np.pi / 12
    U = np.array([0.2, -0.3, 0.1])
    a = KC.kc_mp(rho, u, F.BOX, 2, h, nu=0.02, dt=0.5)
    b = KC.kc_mp(rho, u + U[:, None, None, None], F.BOX, 2, h, nu=0.02, dt=0.5)
    for key in ("m_sgs", "omega_sgs", "k_sgs"):
        assert np.max(np.abs(a[key] - b[key])) < 1e-12 * np.max(np.abs(a[key])), key


def test_exact_rates_match_the_closure_oracle():
    rho, u = synth.random_fields((10, 12, 9), seed=44, rho_amp=0.2)
    h = 2 * np.pi / 12
    nu, dt, theta, c_nu = 0.003, 0.5, 0.7, 0.035
    r = KC.kc_mp(rho, u, F.GAUSS, 2, h, nu, dt, theta, c_nu, rho_ref_one=True)
    w, _ = F.filter_weights(F.GAUSS, 2)
    G = F.grad2(r["ut"], h)
    cl = F.closures(r["rho_bar"], G, r["tau"], 2 * h, F.second_moment(w, h),
                    dict(c_nu=c_nu, theta=theta, nu_mol=nu, dt=dt, ksgs_rho_ref=1))
    assert np.max(np.abs(cl["k_sgs"] - r["k_exact"])) < 1e-15
    assert np.max(np.abs(cl["omega_t"] - r["omega_exact"])) < 1e-12 * np.max(r["omega_exact"])
    st = KC.kc_mp_stats(r, nu)
    assert 0.0 <= st["clip"] <= 1.0 and -1.0 <= min(st["corr"]) <= 1.0


def test_pointwise_equals_field():
    rho, u = synth.random_fields((11, 12, 13), seed=45, rho_amp=0.2)
    h = 2 * np.pi / 13
    args = dict(nu=0.003, dt=0.5, theta=0.7, c_nu=0.035, rho_ref_one=False)
    r = KC.kc_mp(rho, u, F.BOX, 4, h, **args)
    pts = np.array([(0, 0, 0), (10, 11, 12), (5, 6, 2)])
    m, k, nue, om = KC.kc_mp_at(rho, u, F.BOX, 4, h, args["nu"], args["dt"], args["theta"],
                                args["c_nu"], args["rho_ref_one"], pts)
    for n, (a, b, c) in enumerate(pts):
        assert np.max(np.abs(m[n] - r["m_sgs"][:, :, a, b, c])) < 1e-14
        assert abs(k[n] - r["k_sgs"][a, b, c]) < 1e-14
        assert abs(om[n] - r["omega_sgs"][a, b, c]) < 1e-10 * abs(om[n])


def test_kc_mp_stats_on_literal_arrays():
    """kc_mp_stats on hand-built arrays: the relative error runs over all nine pairs (a
    symmetric perturbation d of the xy pair counts twice), Pearson r is +1 for an affine
    image and -1 for a negated one, the clipped fractions count nu_t_eff <= nu (equality
    included) and the means are plain means."""
    rng = np.random.default_rng(5)
    t = rng.standard_normal((3, 3, 50))
    t = 0.5 * (t + np.swapaxes(t, 0, 1))
    d = 0.1
    m = t.copy()
    m[0, 1] += d
    m[1, 0] += d
    nu = 1e-3
    nue = np.full(50, 2e-3)
    nue[:10] = nu  # ten points exactly at the molecular viscosity: clipped
    nue_ex = np.full(50, 2e-3)
    nue_ex[:4] = 0.5 * nu
    r = dict(m_sgs=m, tau=t, k_sgs=np.arange(50.0), k_exact=np.full(50, 2.0),
             omega_sgs=np.full(50, 1.5), omega_exact=np.linspace(1.0, 2.0, 50),
             nu_t_eff=nue, nu_t_exact=nue_ex)
    st = KC.kc_mp_stats(r, nu)
    assert abs(st["rel_err"] - np.sqrt(2 * 50 * d * d / np.sum(t ** 2))) < 1e-15
    assert st["clip"] == 10 / 50 and st["clip_exact"] == 4 / 50
    assert st["mean_k"] == 24.5 and st["mean_k_exact"] == 2.0
    assert st["mean_omega"] == 1.5 and abs(st["mean_omega_exact"] - 1.5) < 1e-15
    r2 = dict(r, m_sgs=3.0 * t + 1.0)
    assert all(abs(c - 1) < 1e-14 for c in KC.kc_mp_stats(r2, nu)["corr"])
    r3 = dict(r, m_sgs=-t)
    assert all(abs(c + 1) < 1e-14 for c in KC.kc_mp_stats(r3, nu)["corr"])
    assert KC.kc_mp_stats(dict(r, m_sgs=t), nu)["rel_err"] == 0.0

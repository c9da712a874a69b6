"""Pins of the D3Q27 collide-and-stream oracle (CPU)."""
import numpy as np
import pytest

from oracle import lbm as L

TH = L.THETA


def random_state(shape, seed, amp=1e-3, u_amp=0.08):
    """Populations of a smooth-ish random flow at equilibrium plus a random nonequilibrium part
    of relative size amp."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.02 * rng.standard_normal(shape)
    u = u_amp * rng.standard_normal((3,) + shape)
    f0 = L.equilibrium(rho, u)
    return f0 * (1.0 + amp * rng.standard_normal(f0.shape))


def test_lattice_and_equilibrium_moments():
    xi, w = L.lattice()
    assert xi.shape == (27, 3) and abs(w.sum() - 1) < 1e-15
    assert list(xi[13]) == [0, 0, 0] and list(xi[9 * 2 + 3 * 1 + 0]) == [1, 0, -1]
    rng = np.random.default_rng(1)
    rho = 1 + 0.1 * rng.standard_normal(40)
    u = 0.15 * rng.standard_normal((3, 40))
    f0 = L.equilibrium(rho, u)
    x = xi.astype(float)
    assert np.allclose(f0.sum(0), rho, rtol=0, atol=1e-15)
    assert np.allclose(np.einsum("ia,i...->a...", x, f0), rho * u, rtol=0, atol=1e-15)
    m2 = np.einsum("ia,ib,i...->ab...", x, x, f0)
    ref = rho * (np.einsum("a...,b...->ab...", u, u) + TH * np.eye(3)[..., None])
    assert np.allclose(m2, ref, rtol=0, atol=1e-15)
    # product form: the mixed third moment is rho ux uy uz; a one-direction cube aliases to xi
    assert np.allclose(np.einsum("i,i...->...", x[:, 0] * x[:, 1] * x[:, 2], f0),
                       rho * u[0] * u[1] * u[2], rtol=0, atol=1e-16)
    assert np.allclose(np.einsum("i,i...->...", x[:, 0] ** 3, f0), rho * u[0], rtol=0, atol=1e-15)


def test_rates_by_hand():
    k, nue, om = L.rates(np.array([-0.08, 0.0]), nu=1e-3, c_nu=0.02)
    assert np.allclose(k, [0.04, 0.0], rtol=0, atol=1e-17)
    assert np.allclose(nue, [0.004, 1e-3], rtol=0, atol=1e-18)  # 0.02 * sqrt(0.04); clipped to nu
    assert np.allclose(om, [1.0 / (0.012 + 0.5), 1.0 / (0.003 + 0.5)], rtol=0, atol=1e-15)


@pytest.mark.parametrize("model", ["kcrb", "kcrb_raw", "kcmp", "kcrr"])
def test_every_closure_reduces_to_bgk_when_rates_coincide(model):
    """With C_nu = 0, nu_t_eff = nu and omega_sgs = omega: the two-rate update is the resolved BGK
    step (stated after eq. operational_two_rate_update)."""
    f = random_state((6, 5, 7), 3)
    nu = 0.02
    fb, _ = L.collide(f, "bgk", nu, 0.0)
    fm, info = L.collide(f, model, nu, 0.0)
    assert np.all(info["omega_sgs"] == info["omega"])
    assert np.max(np.abs(fm - fb)) < 1e-15


@pytest.mark.parametrize("model", ["kcrb", "kcmp", "kcrr"])
def test_hermite_closures_conserve_mass_and_momentum(model):
    f = random_state((6, 5, 7), 4, amp=5e-3, u_amp=0.15)
    fp, info = L.collide(f, model, 0.005, 0.3)
    assert np.any(info["omega_sgs"] != info["omega"])  # the SGS rate is active
    xi, _ = L.lattice()
    x = xi.astype(float)
    assert np.max(np.abs(fp.sum(0) - f.sum(0))) < 1e-15
    assert np.max(np.abs(np.einsum("ia,i...->a...", x, fp - f))) < 1e-15


def test_kcrb_raw_versus_hermite():
    """The raw xi xi first-order part equals the Hermite one minus w_i rho tau_hat d_a u_a
    (KC-RB appendix), so the raw collision changes the mass by (omega - omega_sgs) rho tau_hat
    tr S while the Hermite one conserves it."""
    f = random_state((6, 5, 7), 5, amp=5e-3, u_amp=0.15)
    nu, c_nu = 0.005, 0.3
    _, ih = L.collide(f, "kcrb", nu, c_nu)
    fr, ir = L.collide(f, "kcrb_raw", nu, c_nu)
    _, w = L.lattice()
    tau_hat = nu / TH + 0.5
    trS = ih["S"][0, 0] + ih["S"][1, 1] + ih["S"][2, 2]
    assert np.max(np.abs(ir["f1"] - (ih["f1"] - w[:, None, None, None] * ih["rho"] * tau_hat * trS))) < 1e-16
    dm = fr.sum(0) - f.sum(0)
    assert np.max(np.abs(dm - (ir["omega"] - ir["omega_sgs"]) * ir["rho"] * tau_hat * trS)) < 1e-15
    assert np.max(np.abs(trS)) > 1e-3  # the defect is exercised


def test_kcmp_carrier_moments():
    """The KC-MP carrier w_i / (2 theta^2) H_iab m_ab has no mass or momentum and reproduces the
    SGS second moment m_sgs = m_cneq - m_CE."""
    f = random_state((5, 6, 4), 6, amp=5e-3)
    _, info = L.collide(f, "kcmp", 0.01, 0.1)
    xi, _ = L.lattice()
    x = xi.astype(float)
    fs = info["f_sgs"]
    tol = 1e-13 * np.max(np.abs(info["m_sgs"]))
    assert np.max(np.abs(fs.sum(0))) < tol
    assert np.max(np.abs(np.einsum("ia,i...->a...", x, fs))) < tol
    assert np.max(np.abs(np.einsum("ia,ib,i...->ab...", x, x, fs) - info["m_sgs"])) < tol


def test_kcrr_reconstruction_is_complete():
    """The 6 second-order and 17 higher-order Hermite components, projected from a massless,
    momentumless f_cneq and rebuilt with the T_2 .. T_6 sums of eq.
    kcrr_operational_post_population, give f_cneq back: the reconstruction's coefficients are
    the inverse norms of the D3Q27 tensor-product basis."""
    f = random_state((4, 5, 3), 7, amp=2e-2)
    rho, u = L.moments(f)
    fneq = f - L.equilibrium(rho, u)
    xi, w = L.lattice()
    a = {c: np.einsum("i,i...->...", L.hermite_component(c), fneq) for c in L.SECOND + L.B_HIGH}
    assert np.max(np.abs(L._t_terms(w, a, 3) - fneq)) < 1e-12 * np.max(np.abs(fneq))
    # the second-order Hermite coefficient of a massless distribution is its raw moment
    x = xi.astype(float)
    tol = 1e-13 * np.max(np.abs(a["xx"]))
    assert np.max(np.abs(a["xy"] - np.einsum("i,i...->...", x[:, 0] * x[:, 1], fneq))) < tol
    assert np.max(np.abs(a["xx"] - np.einsum("i,i...->...", x[:, 0] ** 2, fneq))) < tol


def test_rr_recursion_closed_forms():
    """Expansions of the recursion by hand: a_xxy = u_y a_xx + 2 u_x a_xy,
    a_xyz = u_x a_yz + u_y a_xz + u_z a_xy, a_xxyy = u_y^2 a_xx + u_x^2 a_yy + 4 u_x u_y a_xy,
    a_xxyz = u_y u_z a_xx + 2 u_x u_z a_xy + 2 u_x u_y a_xz + u_x^2 a_yz; the result does not
    depend on the order in which a component's letters are expanded."""
    rng = np.random.default_rng(8)
    rho = 1 + 0.1 * rng.standard_normal(20)
    u = 0.2 * rng.standard_normal((3, 20))
    A = rng.standard_normal((3, 3, 20))
    A = 0.5 * (A + A.transpose(1, 0, 2))
    a2 = {(p, q): A[p, q] for p in range(3) for q in range(p, 3)}
    r = L.rr_coefficients(rho, u, a2)
    ux, uy, uz = u
    assert np.allclose(r["xxy"], uy * A[0, 0] + 2 * ux * A[0, 1], atol=1e-15, rtol=0)
    assert np.allclose(r["xyz"], ux * A[1, 2] + uy * A[0, 2] + uz * A[0, 1], atol=1e-15, rtol=0)
    assert np.allclose(r["xxyy"], uy ** 2 * A[0, 0] + ux ** 2 * A[1, 1] + 4 * ux * uy * A[0, 1],
                       atol=1e-15, rtol=0)
    assert np.allclose(r["xxyz"], uy * uz * A[0, 0] + 2 * ux * uz * A[0, 1] + 2 * ux * uy * A[0, 2]
                       + ux ** 2 * A[1, 2], atol=1e-15, rtol=0)
    # order independence: expand permuted spellings through the same recursion
    for comp in ("xxyyz", "xyyzz", "xxyyzz", "xzz"):
        perm = comp[::-1]
        saved = L.B_HIGH
        try:
            L.B_HIGH = (perm,)
            rp = L.rr_coefficients(rho, u, a2)[perm]
        finally:
            L.B_HIGH = saved
        assert np.allclose(rp, r[comp], atol=1e-15, rtol=0), comp


@pytest.mark.parametrize("model", L.MODELS)
def test_uniform_flow_is_a_fixed_point(model):
    shape = (4, 5, 6)
    rho = np.full(shape, 1.03)
    u = np.stack([np.full(shape, v) for v in (0.05, -0.02, 0.07)])
    f = L.equilibrium(rho, u)
    assert np.max(np.abs(L.step(f, model, 0.01, 0.1) - f)) < 1e-15


def test_streaming_moves_each_population_along_its_link():
    xi, _ = L.lattice()
    f = np.zeros((27, 5, 6, 7))
    f[:, 2, 3, 4] = np.arange(1, 28)
    g = L.stream(f)
    for i in range(27):
        k, j, m = (2 + xi[i, 2]) % 5, (3 + xi[i, 1]) % 6, (4 + xi[i, 0]) % 7
        assert g[i, k, j, m] == i + 1 and g[i].sum() == i + 1


def test_bgk_shear_wave_decays_at_the_lattice_viscosity():
    """u_x = A sin(2 pi y / n) at unit density decays as exp(-nu k^2 t) with the viscosity of the
    shifted rate, omega = (nu / theta + 1/2)^-1 (eq. omega_t_discrete), up to the O(k^2) lattice
    error of BGK (below 1 % of the rate at n = 32)."""
    n, A, nu, steps = 32, 1e-4, 0.05, 300
    y = np.arange(n)
    rho = np.ones((1, n, 1))
    u = np.zeros((3, 1, n, 1))
    u[0, 0, :, 0] = A * np.sin(2 * np.pi * y / n)
    f = L.equilibrium(rho, u)
    for _ in range(steps):
        f = L.step(f, "bgk", nu, 0.0)
    _, uu = L.moments(f)
    amp = 2.0 / n * np.sum(uu[0, 0, :, 0] * np.sin(2 * np.pi * y / n))
    k = 2 * np.pi / n
    rate = -np.log(amp / A) / steps
    assert abs(rate / (nu * k * k) - 1) < 1e-2
    # a wrong shift of the rate (omega = theta / nu) would decay at a different rate
    assert abs(rate / ((TH * (TH / nu) - 0.5 * TH) * k * k) - 1) > 0.5


@pytest.mark.parametrize("model", L.MODELS)
def test_step_at_equals_full_step(model):
    f = random_state((7, 6, 8), 9, amp=3e-3)
    full = L.step(f, model, 0.01, 0.15)
    pts = np.array([[0, 0, 0], [6, 5, 7], [3, 2, 4], [1, 5, 0]])
    loc = L.step_at(f, pts, model, 0.01, 0.15)
    for n, (k, j, i) in enumerate(pts):
        assert np.max(np.abs(loc[n] - full[:, k, j, i])) < 1e-16


def test_kcrb_trace_equals_the_kcmp_trace():
    """sum_i f1_i |xi_i|^2 of the Hermite first-order part is tr m_CE = -2 rho theta tau_hat tr S,
    so the KC-RB (Hermite) SGS trace equals the KC-MP one built from m_CE directly; the raw form
    adds rho tau_hat tr S (sum_i w_i |xi_i|^2 = 3 theta = 1)."""
    f = random_state((5, 6, 7), 10, amp=5e-3, u_amp=0.15)
    _, ib = L.collide(f, "kcrb", 0.01, 0.1)
    _, ir = L.collide(f, "kcrb_raw", 0.01, 0.1)
    _, im = L.collide(f, "kcmp", 0.01, 0.1)
    tol = 1e-13 * np.max(np.abs(im["m_trace"]))
    assert np.max(np.abs(ib["m_trace"] - im["m_trace"])) < tol
    tau_hat = 0.01 / TH + 0.5
    trS = ib["S"][0, 0] + ib["S"][1, 1] + ib["S"][2, 2]
    assert np.max(np.abs(ir["m_trace"] - (ib["m_trace"] + ib["rho"] * tau_hat * trS))) < tol


@pytest.mark.parametrize("model", ["kcrb", "kcmp", "kcrr"])
def test_post_collision_hermite_coefficients(model):
    """Projections of f_post - f0 on the D3Q27 Hermite components: every closure relaxes the
    second-order sector as (1 - omega) m_CE + (1 - omega_sgs)(m_cneq - m_CE); the 17 higher-order
    components relax with omega (KC-MP, whose carrier is second order), with omega_sgs (KC-RB,
    whose carrier holds all of them), or split into the RR reference at omega and the rest at
    omega_sgs (KC-RR, eqs. kcrr_operational_sgs_high and kcrr_operational_high_order_collision)."""
    f = random_state((5, 4, 6), 11, amp=5e-3, u_amp=0.15)
    nu, c_nu = 0.004, 0.25
    fp, info = L.collide(f, model, nu, c_nu)
    rho, u = info["rho"], info["u"]
    f0 = L.equilibrium(rho, u)
    om, oms = info["omega"], info["omega_sgs"]
    assert np.mean(np.abs(om - oms) > 1e-3) > 0.5  # the SGS rate differs at most nodes
    tau_hat = nu / TH + 0.5
    m_ce = -2.0 * rho * TH * tau_hat * info["S"]
    xi, _ = L.lattice()
    x = xi.astype(float)
    m_cneq = np.einsum("ia,ib,i...->ab...", x, x, f - f0)
    post2 = np.einsum("ia,ib,i...->ab...", x, x, fp - f0)
    want2 = (1 - om) * m_ce + (1 - oms) * (m_cneq - m_ce)
    assert np.max(np.abs(post2 - want2)) < 1e-12 * np.max(np.abs(m_cneq))
    a2 = {(p, q): m_ce[p, q] for p in range(3) for q in range(p, 3)}
    rr = L.rr_coefficients(rho, u, a2)
    for comp in L.B_HIGH:
        Hc = L.hermite_component(comp)
        a_cneq = np.einsum("i,i...->...", Hc, f - f0)
        a_post = np.einsum("i,i...->...", Hc, fp - f0)
        if model == "kcmp":
            want = (1 - om) * a_cneq
        elif model == "kcrb":
            want = (1 - oms) * a_cneq
        else:
            want = (1 - om) * rr[comp] + (1 - oms) * (a_cneq - rr[comp])
        assert np.max(np.abs(a_post - want)) < 1e-11 * max(np.max(np.abs(a_cneq)), 1e-12), comp

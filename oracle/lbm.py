"""FP64 oracle: one collide-and-stream step of the D3Q27 lattice-Boltzmann solver with the
kinetic closures KC-RB (Hermite and raw first-order reconstructions), KC-MP and KC-RR, and the
resolved BGK step they reduce to.

TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this module; the product path never calls it. It shares no code with the
HIP library: the steps below follow the paper's operational algorithm in population space
(the GPU kernel works on Hermite coefficients instead).

Lattice units throughout: Delta x = Delta t = 1, xi_i in {-1, 0, 1}^3, theta_R = 1/3, weights
w_i = product of the D1Q3 weights (2/3 for 0, 1/6 for +-1); population i is
xi_i = (c_x, c_y, c_z) with i = 9 (c_x + 1) + 3 (c_y + 1) + (c_z + 1). Populations are arrays
(27, nz, ny, nx) of the time-shifted populations of App. "Lattice-Boltzmann discretization".

Steps of App. "Common operational algorithm", per node:
  1. rho = sum_i f_i, rho u = sum_i f_i xi_i;
  2. f0_i(rho, u), the product equilibrium (eq. discrete_equilibrium);
  3. G_ab = d_b u_a by central differences (eq. fd), S = (G + G^T) / 2
     (eq. strain_rate_discrete), periodic;
  4. the closure's SGS trace m_aa (eq. kcrb_operational_msgstrace for KC-RB,
     eq. kcmp_operational_msgstrace for KC-MP and KC-RR);
  5. k_sgs = |m_aa| / (2 rho0), rho0 = 1, nu_t_eff = max(nu, C_nu Delta sqrt(k_sgs)) with
     Delta = Delta x = 1, omega_sgs = (nu_t_eff / theta_R + 1/2)^-1 (eq. omega_sgs_operational);
     omega = (nu / theta_R + 1/2)^-1 (eq. omega_t_discrete), tau_hat = 1 / omega;
  6. the closure's collision (eqs. kcrb_operational_collision, kcmp_operational_collision,
     kcrr_operational_second_order_collision, kcrr_operational_high_order_collision,
     kcrr_operational_post_population);
  7. streaming f_i(x + xi_i) = f_post_i(x) (eq. streaming).

Models: "bgk" (resolved BGK, f_post = f - omega (f - f0)), "kcrb" (first-order part from the
Hermite form, eq. kcrb_operational_fone), "kcrb_raw" (the raw xi xi form,
eq. kcrb_operational_raw_fone), "kcmp", "kcrr".

Parity status: pinned in tests/test_oracle_lbm.py by the equilibrium moments, the reduction of
every closure to BGK when omega_sgs = omega (C_nu = 0), mass and momentum conservation of the
Hermite-consistent collisions, the raw-versus-Hermite relation of the KC-RB appendix, the
completeness of the KC-RR Hermite reconstruction, closed forms of the RR recursion, a uniform
flow as a fixed point, and the viscous decay of a shear wave under BGK.
"""
from __future__ import annotations

import itertools

import numpy as np

THETA = 1.0 / 3.0
MODELS = ("bgk", "kcrb", "kcrb_raw", "kcmp", "kcrr")
W1 = {0: 2.0 / 3.0, 1: 1.0 / 6.0, -1: 1.0 / 6.0}
AX = "xyz"
# the 17 higher-order components of App. "Operational implementation of KC-RR"
B_HIGH = ("xxy", "xxz", "yyz", "xyy", "xzz", "yzz", "xyz",
          "xxyy", "xxzz", "yyzz", "xxyz", "xyyz", "xyzz",
          "xxyyz", "xxyzz", "xyyzz", "xxyyzz")
SECOND = ("xx", "yy", "zz", "xy", "xz", "yz")


def lattice():
    """(xi (27, 3) integers, w (27,)) in the population order above."""
    xi = np.array(list(itertools.product((-1, 0, 1), repeat=3)), dtype=np.int64)
    w = np.array([W1[a] * W1[b] * W1[c] for a, b, c in xi])
    return xi, w


def _bshape(w, ndim):
    return w.reshape((27,) + (1,) * ndim)


def moments(f):
    """rho and u (3, ...) of populations f (27, ...)."""
    xi, _ = lattice()
    f = np.asarray(f, dtype=np.float64)
    rho = f.sum(axis=0)
    j = np.einsum("ia,i...->a...", xi.astype(np.float64), f)
    return rho, j / rho


def equilibrium(rho, u):
    """f0_i = w_i rho prod_a (1 + xi_ia u_a / theta + (xi_ia^2 - theta) u_a^2 / (2 theta^2))."""
    xi, w = lattice()
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    out = np.empty((27,) + rho.shape)
    for i in range(27):
        p = w[i] * rho
        for a in range(3):
            c = xi[i, a]
            p = p * (1.0 + c * u[a] / THETA + (c * c - THETA) * u[a] ** 2 / (2.0 * THETA ** 2))
        out[i] = p
    return out


def gradient(u):
    """G[a, b] = d_b u_a, second-order central differences on the periodic lattice (eq. fd)."""
    G = np.empty((3, 3) + u.shape[1:])
    axis = {0: 2, 1: 1, 2: 0}  # direction -> axis of a (nz, ny, nx) field
    for a in range(3):
        for b in range(3):
            ax = axis[b]
            G[a, b] = 0.5 * (np.roll(u[a], -1, axis=ax) - np.roll(u[a], 1, axis=ax))
    return G


def hermite2(xi):
    """H_iab = xi_ia xi_ib - theta delta_ab (eq. discrete_second_order_hermite), (27, 3, 3)."""
    x = xi.astype(np.float64)
    return np.einsum("ia,ib->iab", x, x) - THETA * np.eye(3)[None]


def rates(m_trace, nu, c_nu, delta=1.0, rho0=1.0):
    """k_sgs, nu_t_eff and omega_sgs of eq. omega_sgs_operational from the SGS trace."""
    k = np.abs(m_trace) / (2.0 * rho0)
    nu_eff = np.maximum(nu, c_nu * delta * np.sqrt(k))
    return k, nu_eff, 1.0 / (nu_eff / THETA + 0.5)


def _h_factor(c, count):
    """Directional Hermite factor of D3Q27: 1, xi or xi^2 - theta for power 0, 1, 2."""
    return (1.0, float(c), float(c * c) - THETA)[count]


def hermite_component(comp):
    """H_i of a component given as a string over x, y, z (each letter at most twice): the product
    of the directional factors, shape (27,)."""
    xi, _ = lattice()
    cnt = [comp.count(a) for a in AX]
    return np.array([np.prod([_h_factor(xi[i, a], cnt[a]) for a in range(3)]) for i in range(27)])


def rr_coefficients(rho, u, a2):
    """RR reference coefficients of the 17 higher-order components, by the recursion of
    eq. kcrr_rr: a_(a1..an) = u_an a_(a1..an-1)
                              + (1/rho) sum_{i<n} a0_(a1..an-1 without ai) a_(ai an),
    with a0_(b1..bk) = rho u_b1 ... u_bk (isothermal equilibrium coefficients) and the
    second-order seed a2[(a, b)] (symmetric). Components are expanded in the order of their
    letters. Returns dict comp -> array."""
    idx = {c: k for k, c in enumerate(AX)}
    memo = {}

    def a0(t):
        out = rho
        for c in t:
            out = out * u[idx[c]]
        return out

    def arr(t):
        if len(t) == 2:
            return a2[tuple(sorted((idx[t[0]], idx[t[1]])))]
        if t in memo:
            return memo[t]
        n = len(t)
        v = u[idx[t[-1]]] * arr(t[:-1])
        for i in range(n - 1):
            rest = t[:i] + t[i + 1:n - 1]
            v = v + a0(rest) * arr(t[i] + t[-1]) / rho
        memo[t] = v
        return v

    return {comp: arr(comp) for comp in B_HIGH}


def _t_terms(w, a, ndim):
    """w_i sum_{m=2..6} T_m of eq. kcrr_operational_post_population for coefficients a[comp]."""
    xi, _ = lattice()
    x = [xi[:, k].astype(np.float64).reshape((27,) + (1,) * ndim) for k in range(3)]
    H = {c: x[k] for k, c in enumerate(AX)}
    H2 = {c: x[k] ** 2 - THETA for k, c in enumerate(AX)}
    t = THETA
    T2 = (H2["x"] * a["xx"] + H2["y"] * a["yy"] + H2["z"] * a["zz"]) / (2 * t ** 2) \
        + (H["x"] * H["y"] * a["xy"] + H["x"] * H["z"] * a["xz"] + H["y"] * H["z"] * a["yz"]) / t ** 2
    T3 = (H2["x"] * H["y"] * a["xxy"] + H2["x"] * H["z"] * a["xxz"] + H2["y"] * H["z"] * a["yyz"]) / (2 * t ** 3) \
        + (H["x"] * H2["y"] * a["xyy"] + H["x"] * H2["z"] * a["xzz"] + H["y"] * H2["z"] * a["yzz"]) / (2 * t ** 3) \
        + H["x"] * H["y"] * H["z"] * a["xyz"] / t ** 3
    T4 = (H2["x"] * H2["y"] * a["xxyy"] + H2["x"] * H2["z"] * a["xxzz"] + H2["y"] * H2["z"] * a["yyzz"]) / (4 * t ** 4) \
        + (H2["x"] * H["y"] * H["z"] * a["xxyz"] + H["x"] * H2["y"] * H["z"] * a["xyyz"]
           + H["x"] * H["y"] * H2["z"] * a["xyzz"]) / (2 * t ** 4)
    T5 = (H2["x"] * H2["y"] * H["z"] * a["xxyyz"] + H2["x"] * H["y"] * H2["z"] * a["xxyzz"]
          + H["x"] * H2["y"] * H2["z"] * a["xyyzz"]) / (4 * t ** 5)
    T6 = H2["x"] * H2["y"] * H2["z"] * a["xxyyzz"] / (8 * t ** 6)
    return _bshape(w, ndim) * (T2 + T3 + T4 + T5 + T6)


def collide(f, model, nu, c_nu, grad_u=None):
    """Post-collision populations of every node (step 6) and the closure fields.

    f: (27, nz, ny, nx); nu: molecular viscosity (lattice units); c_nu: closure constant.
    grad_u, if given, replaces the central differences of step 3 (used by collide_at).
    Returns (f_post, info) with info = dict(rho, u, S, m_trace, k_sgs, nu_t_eff, omega_sgs,
    omega)."""
    if model not in MODELS:
        raise ValueError(f"unknown model {model}")
    f = np.asarray(f, dtype=np.float64)
    nd = f.ndim - 1
    xi, w = lattice()
    wb = _bshape(w, nd)
    rho, u = moments(f)
    f0 = equilibrium(rho, u)
    G = gradient(u) if grad_u is None else grad_u
    S = 0.5 * (G + np.swapaxes(G, 0, 1))
    tau_hat = nu / THETA + 0.5
    omega = 1.0 / tau_hat
    H = hermite2(xi)
    xx = xi.astype(np.float64)
    fneq = f - f0
    info = dict(rho=rho, u=u, S=S, omega=omega)
    if model == "bgk":
        info.update(m_trace=np.zeros_like(rho), k_sgs=np.zeros_like(rho),
                    nu_t_eff=np.full_like(rho, nu), omega_sgs=np.full_like(rho, omega))
        return f - omega * fneq, info
    if model in ("kcrb", "kcrb_raw"):
        # step 4, KC-RB: first-order CE part, carrier estimate, trace over |xi|^2
        if model == "kcrb":
            proj = np.einsum("iab,ab...->i...", H, S)
        else:
            proj = np.einsum("ia,ib,ab...->i...", xx, xx, S)
        f1 = -wb * rho * tau_hat / THETA * proj
        f_sgs = fneq - f1
        m_trace = np.einsum("i,i...->...", (xx ** 2).sum(1), f_sgs)
        k, nue, om_s = rates(m_trace, nu, c_nu)
        info.update(m_trace=m_trace, k_sgs=k, nu_t_eff=nue, omega_sgs=om_s, f1=f1, f_sgs=f_sgs)
        return f - omega * f1 - om_s * f_sgs, info
    # KC-MP and KC-RR: second-order moments of the coarse nonequilibrium
    m_ce = -2.0 * rho * THETA * tau_hat * S
    m_cneq = np.einsum("ia,ib,i...->ab...", xx, xx, fneq)
    m_sgs = m_cneq - m_ce
    m_trace = m_sgs[0, 0] + m_sgs[1, 1] + m_sgs[2, 2]
    k, nue, om_s = rates(m_trace, nu, c_nu)
    info.update(m_trace=m_trace, k_sgs=k, nu_t_eff=nue, omega_sgs=om_s, m_sgs=m_sgs, m_ce=m_ce)
    if model == "kcmp":
        f_sgs = wb / (2.0 * THETA ** 2) * np.einsum("iab,ab...->i...", H, m_sgs)
        f1 = fneq - f_sgs
        info.update(f1=f1, f_sgs=f_sgs)
        return f - omega * f1 - om_s * f_sgs, info
    # KC-RR
    a = {}
    idx = {c: k for k, c in enumerate(AX)}
    for comp in SECOND:
        p, q = idx[comp[0]], idx[comp[1]]
        a[comp] = (1.0 - omega) * m_ce[p, q] + (1.0 - om_s) * m_sgs[p, q]
    a2 = {(p, q): m_ce[p, q] for p in range(3) for q in range(p, 3)}
    a_rr = rr_coefficients(rho, u, a2)
    for comp in B_HIGH:
        a_cneq = np.einsum("i,i...->...", hermite_component(comp), fneq)
        a_sgs = a_cneq - a_rr[comp]
        a[comp] = (1.0 - omega) * a_rr[comp] + (1.0 - om_s) * a_sgs
    info.update(a_post=a, a_rr=a_rr)
    return f0 + _t_terms(w, a, nd), info


def stream(f):
    """f_new_i(x + xi_i) = f_i(x) on the periodic lattice (eq. streaming)."""
    xi, _ = lattice()
    out = np.empty_like(f)
    for i in range(27):
        g = f[i]
        for d, ax in ((0, 2), (1, 1), (2, 0)):
            if xi[i, d]:
                g = np.roll(g, int(xi[i, d]), axis=ax)
        out[i] = g
    return out


def step(f, model, nu, c_nu):
    """One collide-and-stream step of the whole lattice."""
    f_post, _ = collide(f, model, nu, c_nu)
    return stream(f_post)


def step_at(f, pts, model, nu, c_nu):
    """Populations after one step at the nodes pts ((k, j, i) rows), each from its periodic
    5^3 neighbourhood: f_new_i(x) = f_post_i(x - xi_i), and f_post at the 27 nodes x - xi_i
    needs the velocity of their face neighbours. Returns (npts, 27)."""
    f = np.asarray(f)
    _, nz, ny, nx = f.shape
    xi, _ = lattice()
    o = np.arange(-2, 3)
    out = []
    for (k, j, i) in np.asarray(pts).reshape(-1, 3):
        blk = f[:, ((k + o) % nz)[:, None, None], ((j + o) % ny)[None, :, None],
                ((i + o) % nx)[None, None, :]].astype(np.float64)
        fp, _ = collide(blk, model, nu, c_nu)  # valid on the inner 3^3 nodes
        out.append([fp[q, 2 - xi[q, 2], 2 - xi[q, 1], 2 - xi[q, 0]] for q in range(27)])
    return np.array(out)


def tgv_populations(n, u0, dtype=np.float32):
    """Equilibrium populations of the Taylor-Green vortex of Sec. "Taylor-Green vortex" on an
    n^3 lattice: u_x = u0 sin X cos Y cos Z, u_y = -u0 cos X sin Y cos Z, u_z = 0, and the
    density of the pressure fluctuation (u0^2 / 16)(cos 2X + cos 2Y)(cos 2Z + 2) at the lattice
    temperature (rho = 1 + p / theta)."""
    X = 2 * np.pi * np.arange(n) / n
    Z3, Y3, X3 = np.meshgrid(X, X, X, indexing="ij")
    u = np.stack([u0 * np.sin(X3) * np.cos(Y3) * np.cos(Z3),
                  -u0 * np.cos(X3) * np.sin(Y3) * np.cos(Z3), np.zeros_like(X3)])
    rho = 1.0 + (u0 ** 2 / 16.0) * (np.cos(2 * X3) + np.cos(2 * Y3)) * (np.cos(2 * Z3) + 2.0) / THETA
    return equilibrium(rho, u).astype(dtype)

"""FP64 oracle: homogeneous filter, Favre filter, SGS stress, FD gradient, closures, statistics.

TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this module; the product path never calls it. It shares no code
with the HIP library: each formula below is written out from the paper's definitions.

Notation follows the paper: rho_bar = filtered density, ut = Favre velocity,
tau = m^sgs (the SGS second moment), G_ij = d_j ut_i.

Array conventions: fields are float64 numpy arrays shaped (nz, ny, nx) (x fastest);
vectors stack components first: (3, nz, ny, nx); tensors (3, 3, nz, ny, nx).
Axis of Cartesian direction d (0=x, 1=y, 2=z) is AXIS[d].

Parity status of each function is listed with its pin in the tests:
  filter_weights, filter_separable, filter_direct, products, favre, grad2, curl6,
  closures, stats: pinned (closed forms, invariants, brute force).
"""
from __future__ import annotations

import math

import numpy as np

BOX, GAUSS = 0, 1
AXIS = (2, 1, 0)  # Cartesian direction -> numpy axis of a (z, y, x) array
PAIRS = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))  # stored SGS components xx xy xz yy yz zz


# --------------------------------------------------------------------------------------
# Filter kernel
# --------------------------------------------------------------------------------------
def filter_weights(kind: int, n: int):
    """1-D taps (w_{-R}..w_{R}) of a homogeneous filter of width Delta = n h.

    The paper requires a homogeneous filter of uniform width that commutes with
    differentiation and deliberately leaves its shape open (Sec. "Filtered
    nondimensional recorrelated BGK-BE"). Two discrete kernels are used here:

    box:   trapezoidal rule applied to the top-hat of width n h (n even):
           R = n/2, w_m = 1/n for |m| < R, w_{+-R} = 1/(2n).
    gauss: exp(-6 m^2 / n^2) sampled for |m| <= ceil(1.5 n) and normalised to sum 1
           (variance Delta^2/12 for the continuous kernel).
    """
    if n < 1:
        raise ValueError("filter width must be >= 1 grid spacing")
    if kind == BOX:
        if n % 2:
            raise ValueError("box filter needs an even width in grid spacings")
        R = n // 2
        w = np.full(2 * R + 1, 1.0 / n)
        w[0] = w[-1] = 0.5 / n
        return w, R
    if kind == GAUSS:
        R = int(math.ceil(1.5 * n))
        m = np.arange(-R, R + 1, dtype=np.float64)
        g = np.exp(-6.0 * m * m / float(n * n))
        return g / g.sum(), R
    raise ValueError(f"unknown filter kind {kind}")


def second_moment(w, h: float) -> float:
    """M2 = sum_m w_m (m h)^2, the per-direction second moment of the discrete kernel."""
    R = (len(w) - 1) // 2
    m = np.arange(-R, R + 1, dtype=np.float64)
    return float(np.sum(w * (m * h) ** 2))


def transfer(kind: int, n: int, theta):
    """Discrete 1-D transfer function G(theta) = sum_m w_m cos(m theta), theta = k h."""
    w, R = filter_weights(kind, n)
    m = np.arange(-R, R + 1, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    return np.sum(w * np.cos(np.multiply.outer(theta, m)), axis=-1)


def filter_separable(a, w):
    """Periodic filter with product kernel w(x) w(y) w(z): three 1-D passes."""
    R = (len(w) - 1) // 2
    out = np.asarray(a, dtype=np.float64)
    for ax in (2, 1, 0):
        acc = np.zeros_like(out)
        for m in range(-R, R + 1):
            acc += w[m + R] * np.roll(out, -m, axis=ax)  # roll(-m)[i] = a[i + m]
        out = acc
    return out


def filter_direct(a, w):
    """Periodic filter as one direct 3-D sum over all (2R+1)^3 offsets (brute force)."""
    R = (len(w) - 1) // 2
    a = np.asarray(a, dtype=np.float64)
    out = np.zeros_like(a)
    for c in range(-R, R + 1):
        for b in range(-R, R + 1):
            for d in range(-R, R + 1):
                out += (w[c + R] * w[b + R] * w[d + R]) * np.roll(a, (-c, -b, -d), axis=(0, 1, 2))
    return out


# --------------------------------------------------------------------------------------
# Favre filter and SGS stress
# --------------------------------------------------------------------------------------
def products(rho, u):
    """The quantities that get filtered: rho, rho u_i, rho u_i u_j (full 3x3).

    Returns (rho, m (3,...), p (3,3,...)) with m_i = rho u_i and p_ij = rho u_i u_j.
    """
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    m = rho[None] * u
    p = np.empty((3, 3) + rho.shape)
    for i in range(3):
        for j in range(3):
            p[i, j] = rho * u[i] * u[j]
    return rho, m, p


def favre(rho_bar, m_bar, p_bar):
    """Favre velocity and SGS second moment.

    ut_i = bar(rho u_i) / bar(rho) (Favre fields defined after eq. f0resolved);
    tau_ij = rho_bar (~(u_i u_j) - ut_i ut_j) = bar(rho u_i u_j) - rho_bar ut_i ut_j
    (eq. m_sgs_2: the second raw moment of f_sgs).
    """
    ut = m_bar / rho_bar[None]
    tau = np.empty_like(p_bar)
    for i in range(3):
        for j in range(3):
            tau[i, j] = p_bar[i, j] - rho_bar * ut[i] * ut[j]
    return ut, tau


def filter_favre(rho, u, w, separable=True):
    """rho_bar, ut (3,...), tau (3,3,...) of a field pair (rho, u) for taps w."""
    flt = filter_separable if separable else filter_direct
    r, m, p = products(rho, u)
    rho_bar = flt(r, w)
    m_bar = np.stack([flt(m[i], w) for i in range(3)])
    p_bar = np.empty_like(p)
    for i in range(3):
        for j in range(i, 3):
            p_bar[i, j] = flt(p[i, j], w)
            if j != i:
                p_bar[j, i] = flt(p[j, i], w)
    ut, tau = favre(rho_bar, m_bar, p_bar)
    return rho_bar, ut, tau


# --------------------------------------------------------------------------------------
# Gradients
# --------------------------------------------------------------------------------------
def grad2(ut, h: float):
    """G[i, j] = d_j ut_i by second-order central differences, periodic.

    App. "Lattice-Boltzmann discretization", eq. fd:
    d_j u_i ~ (u_i(x + e_j h) - u_i(x - e_j h)) / (2 h).
    """
    G = np.empty((3, 3) + ut.shape[1:])
    for i in range(3):
        for j in range(3):
            ax = AXIS[j]
            G[i, j] = (np.roll(ut[i], -1, axis=ax) - np.roll(ut[i], 1, axis=ax)) / (2.0 * h)
    return G


def strain_rotation(G):
    """S = (G + G^T)/2 (eq. strain_rate_discrete) and W = (G - G^T)/2.

    With G_ij = d_j u_i this W matches the rotation tensor written next to eq. ansumali.
    """
    GT = np.swapaxes(G, 0, 1)
    return 0.5 * (G + GT), 0.5 * (G - GT)


def q_criterion(G):
    """Q = (|W|^2 - |S|^2) / 2 with the Frobenius norms of the antisymmetric and symmetric
    parts of the gradient (the Q-criterion the paper shows for its wake and cavity flows,
    Secs. "Flow in a lid-driven cavity" and "Flow past a circular cylinder")."""
    S, W = strain_rotation(G)
    return 0.5 * (np.einsum("ij...,ij...->...", W, W) - np.einsum("ij...,ij...->...", S, S))


def curl6(u, h: float):
    """Vorticity with sixth-order central differences (Sec. "Taylor-Green vortex":
    enstrophy diagnostics use a sixth-order centered stencil). Standard coefficients
    D f = [45 (f1 - f-1) - 9 (f2 - f-2) + (f3 - f-3)] / (60 h)."""
    def d(f, j):
        ax = AXIS[j]
        acc = np.zeros_like(f)
        for mstep, c in ((1, 45.0), (2, -9.0), (3, 1.0)):
            acc += c * (np.roll(f, -mstep, axis=ax) - np.roll(f, mstep, axis=ax))
        return acc / (60.0 * h)
    u = np.asarray(u, dtype=np.float64)
    return np.stack([d(u[2], 1) - d(u[1], 2), d(u[0], 2) - d(u[2], 0), d(u[1], 0) - d(u[0], 1)])


# --------------------------------------------------------------------------------------
# Closures
# --------------------------------------------------------------------------------------
DEFAULT_PARAMS = dict(c_s=0.11, c_nu=0.02, theta=1.0, nu_mol=0.0, dt=0.0,
                      gm_form=0, m2_mode=0, ksgs_rho_ref=0)


def closures(rho_bar, G, tau, delta: float, m2: float, params=None):
    """Plain closures evaluated from the filtered fields.

    gradient model: tau_gm_ij = rho_bar * C2 * sum_k G_ik G_jk (gm_form 0: second-order
        Taylor expansion of the filter, C2 = M2 of the kernel or Delta^2/12) or
        rho_bar * C2 * sum_k G_ki G_kj (gm_form 1: the contraction of the tensor-
        diffusivity term of eq. ansumali as printed, using the rotation tensor defined
        there). Coefficient Kn/12 of that equation is read as Delta^2/12 (m2_mode 1).
    eddy viscosity (Boussinesq row of the FNSE/FRBGK comparison table, Smagorinsky
        coefficient C_s of Sec. "Test cases"): tau_sm_ij = -2 rho_bar (C_s Delta)^2 |S| S^d_ij,
        |S| = sqrt(2 S:S), S^d the deviatoric strain.
    kinetic closure scalars (Sec. "Turbulent relaxation frequency", eqs.
        ksgs_sharp_trace, nu_t_sharp_closure, omega_t_sharp_closure, and the operational
        eq. omega_sgs_operational): k_sgs = |tau_kk| / (2 rho_ref) with rho_ref = rho_bar
        or 1; nu_t = C_nu Delta sqrt(k_sgs); omega_t = (max(nu, nu_t)/theta + dt/2)^-1.
    """
    p = dict(DEFAULT_PARAMS)
    if params:
        p.update(params)
    coef = m2 if p["m2_mode"] == 0 else delta * delta / 12.0
    tau_gm = np.empty_like(G)
    for i in range(3):
        for j in range(3):
            if p["gm_form"] == 0:
                s = G[i, 0] * G[j, 0] + G[i, 1] * G[j, 1] + G[i, 2] * G[j, 2]
            else:
                s = G[0, i] * G[0, j] + G[1, i] * G[1, j] + G[2, i] * G[2, j]
            tau_gm[i, j] = rho_bar * coef * s
    S, _ = strain_rotation(G)
    SS = np.einsum("ij...,ij...->...", S, S)
    smag = np.sqrt(2.0 * SS)
    trS = S[0, 0] + S[1, 1] + S[2, 2]
    tau_sm = np.empty_like(G)
    for i in range(3):
        for j in range(3):
            sd = S[i, j] - (trS / 3.0 if i == j else 0.0)
            tau_sm[i, j] = -2.0 * rho_bar * (p["c_s"] * delta) ** 2 * smag * sd
    rho_ref = rho_bar if p["ksgs_rho_ref"] == 0 else 1.0
    k_sgs = np.abs(tau[0, 0] + tau[1, 1] + tau[2, 2]) / (2.0 * rho_ref)
    nu_t = p["c_nu"] * delta * np.sqrt(k_sgs)
    with np.errstate(divide="ignore"):
        omega_t = 1.0 / (np.maximum(p["nu_mol"], nu_t) / p["theta"] + 0.5 * p["dt"])
    return dict(tau_gm=tau_gm, tau_smag=tau_sm, k_sgs=k_sgs, nu_t=nu_t, omega_t=omega_t)


# --------------------------------------------------------------------------------------
# Statistics (two-pass, FP64)
# --------------------------------------------------------------------------------------
def pearson(a, b) -> float:
    """Pearson correlation over all points, two-pass: cov / sqrt(var var)."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    da = a - a.mean()
    db = b - b.mean()
    den = math.sqrt(np.sum(da * da) * np.sum(db * db))
    return float(np.sum(da * db) / den) if den > 0 else float("nan")


def width_stats(rho_bar, ut, tau, G, tau_gm):
    """Global statistics of one filter width.

    mean_rho_bar, ke_resolved = <rho_bar |ut|^2 / 2>,
    pi = -<tau_ij S_ij> (SGS dissipation, all 9 pairs), pi_gm likewise with tau_gm,
    corr_tau_gm[c] = r(tau_c, tau_gm_c) for the 6 stored components,
    corr_pi = r(-tau:S, -tau_gm:S) pointwise.
    """
    S, _ = strain_rotation(G)
    pi_loc = -np.einsum("ij...,ij...->...", tau, S)
    pi_gm_loc = -np.einsum("ij...,ij...->...", tau_gm, S)
    out = dict(
        mean_rho_bar=float(np.mean(rho_bar)),
        ke_resolved=float(np.mean(0.5 * rho_bar * np.sum(ut * ut, axis=0))),
        pi=float(np.mean(pi_loc)),
        pi_gm=float(np.mean(pi_gm_loc)),
        corr_tau_gm=[pearson(tau[i, j], tau_gm[i, j]) for (i, j) in PAIRS],
        corr_pi=pearson(pi_loc, pi_gm_loc),
    )
    return out


def input_stats(rho, u, h: float):
    """Volume averages of eq. tgv_energy_enstrophy: E_k = <rho |u|^2 / 2>,
    Z = <|omega|^2 / 2> with sixth-order vorticity; plus <rho>."""
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    om = curl6(u, h)
    return dict(mean_rho=float(rho.mean()),
                ek=float(np.mean(0.5 * rho * np.sum(u * u, axis=0))),
                enstrophy=float(np.mean(0.5 * np.sum(om * om, axis=0))))


# --------------------------------------------------------------------------------------
# Whole path on a full field, and on sampled points
# --------------------------------------------------------------------------------------
def full_path(rho, u, kind: int, n_delta: int, h: float, params=None, separable=True):
    """Every output of one filter width on the full grid (FP64)."""
    w, R = filter_weights(kind, n_delta)
    delta = n_delta * h
    m2 = second_moment(w, h)
    rho_bar, ut, tau = filter_favre(rho, u, w, separable=separable)
    G = grad2(ut, h)
    cl = closures(rho_bar, G, tau, delta, m2, params)
    st = width_stats(rho_bar, ut, tau, G, cl["tau_gm"])
    return dict(rho_bar=rho_bar, ut=ut, tau=tau, G=G, m2=m2, delta=delta, R=R, stats=st, **cl)


def sampled_points(rho, u, kind: int, n_delta: int, h: float, pts, params=None):
    """Outputs at selected points (k, j, i) by direct 3-D sums, for grids too large for
    the full-field oracle. The Favre velocity at the six face neighbours is computed
    the same way, so the centred gradient is exact with respect to the definition."""
    w, R = filter_weights(kind, n_delta)
    delta = n_delta * h
    m2 = second_moment(w, h)
    rho = np.asarray(rho)
    u = np.asarray(u)
    nz, ny, nx = rho.shape
    w3 = np.einsum("a,b,c->abc", w, w, w)
    offs = np.arange(-R, R + 1)
    nb = [(0, 0, 0), (0, 0, 1), (0, 0, -1), (0, 1, 0), (0, -1, 0), (1, 0, 0), (-1, 0, 0)]
    res = {k: [] for k in ("rho_bar", "ut", "tau", "G", "tau_gm", "tau_smag", "k_sgs", "nu_t", "omega_t")}
    for (k, j, i) in np.asarray(pts).reshape(-1, 3):
        vals = []
        for (dz, dy, dx) in nb:
            iz = (k + dz + offs) % nz
            iy = (j + dy + offs) % ny
            ix = (i + dx + offs) % nx
            r = rho[np.ix_(iz, iy, ix)].astype(np.float64)
            uu = np.stack([u[a][np.ix_(iz, iy, ix)] for a in range(3)]).astype(np.float64)
            rb = float(np.sum(w3 * r))
            mb = np.array([np.sum(w3 * r * uu[a]) for a in range(3)])
            pb = np.array([[np.sum(w3 * r * uu[a] * uu[b]) for b in range(3)] for a in range(3)])
            vals.append((rb, mb, pb))
        rb, mb, pb = vals[0]
        ut = mb / rb
        tau = pb - rb * np.outer(ut, ut)
        utn = [v[1] / v[0] for v in vals]
        G = np.empty((3, 3))
        for jd, (ip, im) in enumerate(((1, 2), (3, 4), (5, 6))):
            G[:, jd] = (utn[ip] - utn[im]) / (2.0 * h)
        cl = closures(np.array(rb), G[..., None], tau[..., None], delta, m2, params)
        res["rho_bar"].append(rb)
        res["ut"].append(ut)
        res["tau"].append(tau)
        res["G"].append(G)
        for key in ("tau_gm", "tau_smag"):
            res[key].append(cl[key][..., 0])
        for key in ("k_sgs", "nu_t", "omega_t"):
            res[key].append(float(np.asarray(cl[key]).ravel()[0]))
    return {k: np.array(v) for k, v in res.items()} | dict(m2=m2, delta=delta, R=R)

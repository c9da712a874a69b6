"""FP64 oracle: a priori KC-MP estimate of the SGS second moment and the KC relaxation-rate
field.

TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this module; the product path never calls it. It shares no code with
the HIP library.

Reading (the paper computes these quantities inside its lattice-Boltzmann solver; here they
are evaluated a priori on given fields):

* The fine-grained state is f = f0(rho, u) + f1 with the Chapman-Enskog first-order part,
  whose second moment is m1 = -2 rho theta tau_hat S(u) (the form of the CE reference stress,
  eq. m_ce_reference and its operational counterpart in App. "Operational implementation of
  KC-MP"), with tau_hat = nu / theta + dt / 2 and S(u) from second-order central differences
  (eqs. fd, strain_rate_discrete) on the fine grid.
* Filtering gives the coarse non-equilibrium moment m_cneq = sum_i (f_bar_i - f0_i(rho_bar,
  ut)) xi xi = tau + bar(m1) = tau - 2 theta tau_hat bar(rho S).
* KC-MP (eqs. m_sgs_KCMP, kcmp_operational_msgstrace): m_sgs = m_cneq - m_CE with
  m_CE = -2 rho_bar theta tau_hat S_t, S_t = S(ut) by the same differences, so
      m_sgs_kcmp = tau - 2 theta tau_hat (bar(rho S) - rho_bar S_t).
* Rates (eq. omega_sgs_operational): k_sgs = |m_sgs_aa| / (2 rho_ref) (rho_ref = 1, the
  operational reference density, or rho_bar), nu_t_eff = max(nu, C_nu Delta sqrt(k_sgs)),
  omega_sgs = (nu_t_eff / theta + dt / 2)^-1; the same from the exact tau for comparison.

Parity status: pinned by the closed form of a shear wave with a density wave along z
(transfer functions evaluated pointwise), m_sgs_kcmp = tau exactly at constant density
(the discrete filter commutes with the differences) and for tau_hat = 0, invariance under a
constant velocity shift, and the exact-tau rates against the closure oracle.
"""
from __future__ import annotations

import numpy as np

from . import fields as F


def rates(m_sgs, rho_bar, delta, nu, dt, theta, c_nu, rho_ref_one=True):
    """k_sgs, nu_t_eff, omega_sgs from a second-moment tensor (3, 3, ...)."""
    rho_ref = 1.0 if rho_ref_one else rho_bar
    k = np.abs(m_sgs[0, 0] + m_sgs[1, 1] + m_sgs[2, 2]) / (2.0 * rho_ref)
    nu_eff = np.maximum(nu, c_nu * delta * np.sqrt(k))
    om = 1.0 / (nu_eff / theta + 0.5 * dt)
    return k, nu_eff, om


def kc_mp(rho, u, kind: int, n_delta: int, h: float, nu: float, dt: float = 0.0,
          theta: float = 1.0, c_nu: float = 0.035, rho_ref_one=True, separable=True):
    """Every field of the a priori KC-MP evaluation of one filter width."""
    w, _ = F.filter_weights(kind, n_delta)
    filt = F.filter_separable if separable else F.filter_direct
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    rb, ut, tau = F.filter_favre(rho, u, w, separable=separable)
    S, _ = F.strain_rotation(F.grad2(u, h))
    rs_bar = np.stack([np.stack([filt(rho * S[i, j], w) for j in range(3)]) for i in range(3)])
    St, _ = F.strain_rotation(F.grad2(ut, h))
    tau_hat = nu / theta + 0.5 * dt
    m_ce = -2.0 * rb * theta * tau_hat * St
    m_sgs = tau - 2.0 * theta * tau_hat * (rs_bar - rb * St)
    delta = n_delta * h
    k, nu_eff, om = rates(m_sgs, rb, delta, nu, dt, theta, c_nu, rho_ref_one)
    ke, nue, ome = rates(tau, rb, delta, nu, dt, theta, c_nu, rho_ref_one)
    return dict(rho_bar=rb, ut=ut, tau=tau, rs_bar=rs_bar, S_t=St, m_ce=m_ce, m_sgs=m_sgs,
                k_sgs=k, nu_t_eff=nu_eff, omega_sgs=om, k_exact=ke, nu_t_exact=nue,
                omega_exact=ome, tau_hat=tau_hat)


def kc_mp_at(rho, u, kind: int, n_delta: int, h: float, nu: float, dt: float, theta: float,
             c_nu: float, rho_ref_one, pts):
    """m_sgs (npts, 3, 3), k_sgs, nu_t_eff, omega_sgs at points (k, j, i) by direct sums:
    rho_bar, tau and G from fields.sampled_points, bar(rho S) from the strain of the
    (2R+1)^3 neighbourhood (itself from the neighbours one cell further out)."""
    w, R = F.filter_weights(kind, n_delta)
    rho = np.asarray(rho)
    u = np.asarray(u)
    nz, ny, nx = rho.shape
    sp = F.sampled_points(rho, u, kind, n_delta, h, pts)
    w3 = np.einsum("a,b,c->abc", w, w, w)
    offs = np.arange(-R - 1, R + 2)
    tau_hat = nu / theta + 0.5 * dt
    m_all, k_all, nue_all, om_all = [], [], [], []
    for n, (k, j, i) in enumerate(np.asarray(pts).reshape(-1, 3)):
        ix = np.ix_((k + offs) % nz, (j + offs) % ny, (i + offs) % nx)
        r = rho[ix].astype(np.float64)
        uu = np.stack([u[a][ix] for a in range(3)]).astype(np.float64)
        G = np.empty((3, 3) + r.shape)
        for a in range(3):
            for b in range(3):
                ax = F.AXIS[b]
                G[a, b] = (np.roll(uu[a], -1, axis=ax) - np.roll(uu[a], 1, axis=ax)) / (2.0 * h)
        S = 0.5 * (G + np.swapaxes(G, 0, 1))
        inner = (slice(1, -1),) * 3
        rs = np.array([[np.sum(w3 * (r * S[a, b])[inner]) for b in range(3)] for a in range(3)])
        Gt = sp["G"][n]
        St = 0.5 * (Gt + Gt.T)
        rb = sp["rho_bar"][n]
        m = sp["tau"][n] - 2.0 * theta * tau_hat * (rs - rb * St)
        kk, nue, om = rates(m[..., None, None], np.array([rb]), n_delta * h, nu, dt, theta, c_nu,
                            rho_ref_one)
        m_all.append(m)
        k_all.append(float(kk[0, 0]))
        nue_all.append(float(nue[0, 0]))
        om_all.append(float(om[0, 0]))
    return np.array(m_all), np.array(k_all), np.array(nue_all), np.array(om_all)


def kc_mp_stats(r, nu):
    """Comparison of the KC-MP estimate with the exact tau: Pearson r per stored component,
    relative Frobenius error, means of the rates and the fractions clipped to nu."""
    m, t = r["m_sgs"], r["tau"]
    corr = [F.pearson(m[i, j], t[i, j]) for (i, j) in F.PAIRS]
    err = float(np.sum((m - t) ** 2))
    nrm = float(np.sum(t ** 2))
    return dict(corr=corr, rel_err=float(np.sqrt(err / nrm)), mean_k=float(np.mean(r["k_sgs"])),
                mean_k_exact=float(np.mean(r["k_exact"])),
                mean_omega=float(np.mean(r["omega_sgs"])),
                mean_omega_exact=float(np.mean(r["omega_exact"])),
                clip=float(np.mean(r["nu_t_eff"] <= nu)),
                clip_exact=float(np.mean(r["nu_t_exact"] <= nu)))

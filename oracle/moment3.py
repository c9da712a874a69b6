"""FP64 oracle: the third-order SGS moment and the Favre temperature.

TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this module; the product path never calls it. It shares no code with
the HIP library.

Definitions (paper: Sec. "Filtered nondimensional recorrelated BGK-BE"):

* m3_ijk = bar(rho u_i u_j u_k) - rho_bar ut_i ut_j ut_k, the Favre third-order correlation
  minus the product of the Favre velocities times rho_bar: the coefficient of the
  third-order Hermite term of the carrier's series (eq. f_sgs_hermite). Symmetric; the ten
  components are stored in the order of TRIPLES (xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz).
* theta_t = bar(rho theta) / rho_bar, the Favre temperature (definition after eq.
  f0resolved).

Parity status: pinned by the closed form of a single cosine mode through the kernel's
transfer function, the Galilean shift rule m3(u + U) = m3(u) + U_i tau_jk + U_j tau_ik +
U_k tau_ij with tau of the field oracle, vanishing for a uniform velocity, the mixed
components against the order-3 Hermite coefficients of the carrier oracle's f_sgs (filtered
equilibria, an independent route), and, for theta_t, constant and density-weighted cases;
direct sums at points against the separable field.
"""
from __future__ import annotations

import numpy as np

from . import fields as F

TRIPLES = ((0, 0, 0), (0, 0, 1), (0, 0, 2), (0, 1, 1), (0, 1, 2), (0, 2, 2), (1, 1, 1),
           (1, 1, 2), (1, 2, 2), (2, 2, 2))


def moment3(rho, u, kind: int, n_delta: int, separable=True):
    """rho_bar, ut (3, ...) and m3 (10, ...) of one filter width."""
    w, _ = F.filter_weights(kind, n_delta)
    filt = F.filter_separable if separable else F.filter_direct
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    rb = filt(rho, w)
    ut = np.stack([filt(rho * u[a], w) / rb for a in range(3)])
    m3 = np.stack([filt(rho * u[i] * u[j] * u[k], w) - rb * ut[i] * ut[j] * ut[k]
                   for (i, j, k) in TRIPLES])
    return dict(rho_bar=rb, ut=ut, m3=m3)


def favre_temperature(rho, theta, kind: int, n_delta: int, separable=True):
    """theta_t = bar(rho theta) / rho_bar."""
    w, _ = F.filter_weights(kind, n_delta)
    filt = F.filter_separable if separable else F.filter_direct
    rho = np.asarray(rho, dtype=np.float64)
    return filt(rho * np.asarray(theta, dtype=np.float64), w) / filt(rho, w)


def moment3_at(rho, u, theta, kind: int, n_delta: int, pts):
    """m3 (npts, 10) and theta_t (npts,) (None without theta) at points (k, j, i) by direct
    3-D sums over each point's (2R+1)^3 neighbourhood."""
    w, R = F.filter_weights(kind, n_delta)
    rho = np.asarray(rho)
    u = np.asarray(u)
    nz, ny, nx = rho.shape
    w3 = np.einsum("a,b,c->abc", w, w, w)
    offs = np.arange(-R, R + 1)
    m3, tt = [], []
    for (k, j, i) in np.asarray(pts).reshape(-1, 3):
        ix = np.ix_((k + offs) % nz, (j + offs) % ny, (i + offs) % nx)
        r = rho[ix].astype(np.float64)
        uu = np.stack([u[a][ix] for a in range(3)]).astype(np.float64)
        rb = float(np.sum(w3 * r))
        ut = np.array([np.sum(w3 * r * uu[a]) for a in range(3)]) / rb
        m3.append([np.sum(w3 * r * uu[a] * uu[b] * uu[c]) - rb * ut[a] * ut[b] * ut[c]
                   for (a, b, c) in TRIPLES])
        if theta is not None:
            tt.append(float(np.sum(w3 * r * np.asarray(theta)[ix])) / rb)
    return np.array(m3), (np.array(tt) if theta is not None else None)

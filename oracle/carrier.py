"""FP64 oracle: the a priori D3Q27 SGS carrier f_sgs,i = bar(f0_i(rho, u)) - f0_i(rho_bar, ut)
and its second-order Hermite reconstruction from tau.

TEST INFRASTRUCTURE. Only the tests and the smoke check may import this module; the product
path never calls it. It shares no code with the HIP library.

Definitions (paper: Sec. "Filtered nondimensional recorrelated BGK-BE", eqs. f0bar, fsgs_def;
App. "Lattice-Boltzmann discretization", eq. discrete_equilibrium; App. "Hermite
representation" and the KC-MP closure, eq. f_sgs_KCMP):

* D3Q27 velocities xi_i in {-1, 0, 1}^3 (lattice units), weights w_i = prod of the D1Q3
  weights (2/3 for 0, 1/6 for +-1), reference temperature theta_R = 1/3.
* Velocities of the fields are given in units of sqrt(theta_R) (Mach numbers, the units of
  the synthetic inputs); with xh = xi / sqrt(theta_R) in {0, +-sqrt(3)} the product
  equilibrium reads f0_i(rho, u) = w_i rho prod_a (1 + xh_ia u_a + (xh_ia^2 - 1) u_a^2 / 2).
* Exact carrier: f_sgs,i = bar(f0_i(rho, u)) - f0_i(rho_bar, ut), the filter applied to each
  of the 27 equilibria.
* Second-order Hermite reconstruction: f_h2,i = w_i / 2 * sum_ab H_iab tau_ab,
  H_iab = xh_ia xh_ib - delta_ab, with tau in the same units.

* Hermite-order energies: f projected on the tensor-product D1Q3 Hermite basis by lattice
  quadrature; E_n is the weighted energy of the terms of total degree n.

Parity status: pinned by the moment identities (sum f_sgs = 0, sum xh f_sgs = 0,
sum xh xh f_sgs = tau of the field oracle), vanishing on constant and uniform-velocity fields,
exactness of the reconstruction for a one-component velocity at unit density, and the
brute-force lattice equilibrium against its moment form; the Hermite energies by Parseval,
by E_2 against tau of the field oracle, by vanishing E_0, E_1 of the carrier and by single
basis functions of known norm.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import fields as F

W1 = {0: 2.0 / 3.0, 1: 1.0 / 6.0, -1: 1.0 / 6.0}
SQ3 = math.sqrt(3.0)


def lattice():
    """(xi (27, 3) integers, xh (27, 3) = xi sqrt(3), w (27,)) in the order of itertools.product
    over (x, y, z) in (-1, 0, 1)."""
    xi = np.array(list(itertools.product((-1, 0, 1), repeat=3)), dtype=np.int64)
    w = np.array([W1[a] * W1[b] * W1[c] for a, b, c in xi])
    return xi, xi * SQ3, w


def equilibrium(rho, u):
    """f0_i(rho, u) of every population, shape (27,) + rho.shape (eq. discrete_equilibrium)."""
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    _, xh, w = lattice()
    out = np.empty((27,) + rho.shape)
    for i in range(27):
        f = w[i] * rho
        for a in range(3):
            f = f * (1.0 + xh[i, a] * u[a] + 0.5 * (xh[i, a] ** 2 - 1.0) * u[a] ** 2)
        out[i] = f
    return out


def moments(f):
    """Zeroth, first and second moments of populations f (27, ...) in xh units."""
    _, xh, _ = lattice()
    m0 = f.sum(0)
    m1 = np.einsum("ia,i...->a...", xh, f)
    m2 = np.einsum("ia,ib,i...->ab...", xh, xh, f)
    return m0, m1, m2


def hermite2(tau):
    """f_h2,i = w_i / 2 sum_ab (xh_ia xh_ib - delta_ab) tau_ab; tau (3, 3, ...)."""
    _, xh, w = lattice()
    H = np.einsum("ia,ib->iab", xh, xh) - np.eye(3)[None]
    return 0.5 * w.reshape((27,) + (1,) * (tau.ndim - 2)) * np.einsum("iab,ab...->i...", H, tau)


def carrier(rho, u, kind: int, n_delta: int, separable=True):
    """Exact carrier, its Hermite reconstruction and the Favre fields of one filter width."""
    w, _ = F.filter_weights(kind, n_delta)
    f0 = equilibrium(rho, u)
    filt = F.filter_separable if separable else F.filter_direct
    f0bar = np.stack([filt(f0[i], w) for i in range(27)])
    rho_bar, ut, tau = F.filter_favre(rho, u, w, separable=separable)
    f_sgs = f0bar - equilibrium(rho_bar, ut)
    f_h2 = hermite2(tau)
    return dict(f_sgs=f_sgs, f_h2=f_h2, rho_bar=rho_bar, ut=ut, tau=tau)


def carrier_at(rho, u, kind: int, n_delta: int, pts):
    """f_sgs and f_h2 (each (npts, 27)) at points (k, j, i) by direct 3-D sums of the 27
    equilibria over each point's (2R+1)^3 neighbourhood, for grids too large for carrier()."""
    w, R = F.filter_weights(kind, n_delta)
    rho = np.asarray(rho)
    u = np.asarray(u)
    nz, ny, nx = rho.shape
    w3 = np.einsum("a,b,c->abc", w, w, w)
    offs = np.arange(-R, R + 1)
    fs, fh = [], []
    for (k, j, i) in np.asarray(pts).reshape(-1, 3):
        ix = np.ix_((k + offs) % nz, (j + offs) % ny, (i + offs) % nx)
        r = rho[ix].astype(np.float64)
        uu = np.stack([u[a][ix] for a in range(3)]).astype(np.float64)
        f0bar = np.array([np.sum(w3 * f) for f in equilibrium(r, uu)])
        rb = float(np.sum(w3 * r))
        ut = np.array([np.sum(w3 * r * uu[a]) for a in range(3)]) / rb
        tau = np.array([[np.sum(w3 * r * uu[a] * uu[b]) for b in range(3)] for a in range(3)])
        tau = tau - rb * np.outer(ut, ut)
        fs.append(f0bar - equilibrium(np.array(rb), ut))
        fh.append(hermite2(tau))
    return np.array(fs), np.array(fh)


def hermite_coefficients(f):
    """Coefficients d_abc (a, b, c in 0..2; shape (3, 3, 3) + point shape) of populations f in
    the tensor-product D1Q3 Hermite basis P_0 = 1, P_1 = xh, P_2 = (xh^2 - 1)/2, by quadrature:
    d_abc = sum_i f_i P_a(xh_ix) P_b(xh_iy) P_c(xh_iz) / (n_a n_b n_c) with the norms
    n_a = sum_k w_k P_a(xh_k)^2 = (1, 1, 1/2). Their total degree a + b + c is the Hermite
    order of the term (the expansion of eq. f_sgs_hermite, truncated to the lattice)."""
    _, xh, _ = lattice()
    P = np.stack([np.ones_like(xh), xh, 0.5 * (xh ** 2 - 1.0)])  # (3 degrees, 27, 3 dims)
    nrm = np.array([1.0, 1.0, 0.5])
    d = np.einsum("ai,bi,ci,i...->abc...", P[:, :, 0], P[:, :, 1], P[:, :, 2], f)
    return d / np.einsum("a,b,c->abc", nrm, nrm, nrm).reshape((3, 3, 3) + (1,) * (f.ndim - 1))


def hermite_energies(f):
    """E_n = <sum_{a+b+c=n} n_a n_b n_c d_abc^2>, n = 0..6: the split of the weighted energy
    <sum_i f_i^2 / w_i> over the Hermite orders of f (Parseval under the lattice weights)."""
    d = hermite_coefficients(f)
    nrm = np.array([1.0, 1.0, 0.5])
    out = np.zeros(7)
    for a, b, c in itertools.product(range(3), repeat=3):
        out[a + b + c] += nrm[a] * nrm[b] * nrm[c] * float(np.mean(d[a, b, c] ** 2))
    return out


def carrier_stats(f_sgs, f_h2):
    """<sum_i f_sgs,i^2>, <sum_i (f_sgs,i - f_h2,i)^2>, their ratio's square root (the
    relative L2 error of the second-order reconstruction) and the Hermite-order energies of
    f_sgs."""
    e2 = float(np.mean(np.sum((f_sgs - f_h2) ** 2, 0)))
    s2 = float(np.mean(np.sum(f_sgs ** 2, 0)))
    return dict(sgs_l2=s2, err_l2=e2, rel_err=math.sqrt(e2 / s2) if s2 > 0 else 0.0,
                hermite=hermite_energies(f_sgs))

"""Seeded synthetic inputs: spectral turbulence, the Taylor-Green field, single Fourier modes.

This module produces input fields only. It holds none of the filtering, Favre or
closure arithmetic, and it is the one module that both the HIP path's callers and
the FP64 checker's callers share.

Conventions (shared by every consumer):
  * periodic box [0, 2*pi)^3 with n points per side, spacing h = 2*pi/n;
  * fields are C-ordered (z, y, x) float32 arrays or tensors, so x is fastest and a
    point (i, j, k) lives at i + n*(j + n*k);
  * velocity is a (3, n, n, n) block, components x|y|z.

Spectral recipe (random-phase solenoidal field):
  integer wavenumbers; every Fourier coefficient of the half spectrum gets a complex
  normal variate from a seeded torch.Generator, scaled so that the shell energy
  follows E(k) ~ k^4 exp(-2 (k/k0)^2); the velocity coefficients are projected onto
  the plane normal to k (divergence free); k = 0 and the Nyquist planes are zeroed;
  an inverse real FFT gives the field, which is rescaled to an exact rms magnitude
  sqrt(<u_i u_i>) = urms.  The density is 1 + amp * s, where s has the same spectrum,
  zero mean and unit peak amplitude (max |s| = 1), so rho stays in [1 - amp, 1 + amp]
  at every grid size (a unit-rms Gaussian scalar would reach 5-6 sigma on 10^7 points).
"""
from __future__ import annotations

import math

import numpy as np
import torch


def _wavenumbers(n: int, device):
    k_full = torch.fft.fftfreq(n, d=1.0 / n, device=device, dtype=torch.float64)
    k_half = torch.fft.rfftfreq(n, d=1.0 / n, device=device, dtype=torch.float64)
    kz = k_full.view(n, 1, 1)
    ky = k_full.view(1, n, 1)
    kx = k_half.view(1, 1, n // 2 + 1)
    return kx, ky, kz


def _spectral_amplitude(n: int, k0: float, device):
    kx, ky, kz = _wavenumbers(n, device)
    k2 = kx * kx + ky * ky + kz * kz
    k = torch.sqrt(k2)
    # |c(k)|^2 ~ E(k) / (4 pi k^2) with E ~ k^4 exp(-2 (k/k0)^2)
    amp = k * torch.exp(-(k / k0) ** 2) / math.sqrt(4.0 * math.pi)
    nyq = float(n // 2)
    mask = (k2 == 0) | (kx.abs() == nyq) | (ky.abs() == nyq) | (kz.abs() == nyq)
    amp = torch.where(mask, torch.zeros_like(amp), amp)
    return kx, ky, kz, k2, amp


def _complex_normal(shape, gen, device):
    re = torch.randn(shape, generator=gen, device=device, dtype=torch.float64)
    im = torch.randn(shape, generator=gen, device=device, dtype=torch.float64)
    return torch.complex(re, im) * math.sqrt(0.5)


def spectral_velocity(n: int, k0: float, urms: float, seed: int, device="cpu") -> torch.Tensor:
    """Divergence-free random-phase velocity, shape (3, n, n, n) float32, rms magnitude urms."""
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    kx, ky, kz, k2, amp = _spectral_amplitude(n, k0, device)
    shape = (n, n, n // 2 + 1)
    c = [_complex_normal(shape, gen, device) * amp for _ in range(3)]
    k2s = torch.where(k2 == 0, torch.ones_like(k2), k2)
    kdotc = (kx * c[0] + ky * c[1] + kz * c[2]) / k2s
    c = [c[0] - kx * kdotc, c[1] - ky * kdotc, c[2] - kz * kdotc]
    del kdotc
    u = torch.empty((3, n, n, n), dtype=torch.float64, device=device)
    for a in range(3):
        u[a] = torch.fft.irfftn(c[a], s=(n, n, n), dim=(0, 1, 2))
    del c
    scale = urms / torch.sqrt((u * u).sum(dim=0).mean())
    u *= scale
    return u.to(torch.float32)


def spectral_scalar(n: int, k0: float, seed: int, device="cpu") -> torch.Tensor:
    """Zero-mean random-phase scalar with the velocity's spectrum and max |s| = 1, float64."""
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    _, _, _, _, amp = _spectral_amplitude(n, k0, device)
    c = _complex_normal((n, n, n // 2 + 1), gen, device) * amp
    s = torch.fft.irfftn(c, s=(n, n, n), dim=(0, 1, 2))
    s = s - s.mean()
    s = s / s.abs().max()
    return s


def turbulence(n: int, k0: float, urms: float, rho_amp: float, vel_seed: int, scal_seed: int,
               device="cpu"):
    """(rho, u) float32 tensors: rho (n,n,n), u (3,n,n,n). Raises if min(rho) <= 0.05."""
    u = spectral_velocity(n, k0, urms, vel_seed, device)
    s = spectral_scalar(n, k0, scal_seed, device)
    rho = (1.0 + rho_amp * s).to(torch.float32)
    del s
    rmin = float(rho.min())
    if rmin <= 0.05:
        raise ValueError(f"synthetic density has min {rmin:.3g} <= 0.05; lower rho_amp")
    return rho, u


# Named workloads: grid, spectral peak, density amplitude, seeds.
WORKLOADS = {
    "c32_box4": dict(n=32, k0=4.0, urms=0.3, rho_amp=0.1, vel_seed=1001, scal_seed=2001),
    "c256_gauss8": dict(n=256, k0=8.0, urms=0.3, rho_amp=0.2, vel_seed=1002, scal_seed=2002),
    "c256_heldout": dict(n=256, k0=8.0, urms=0.3, rho_amp=0.2, vel_seed=1003, scal_seed=2003),
    "c512_box_multi": dict(n=512, k0=16.0, urms=0.3, rho_amp=0.2, vel_seed=1004, scal_seed=2004),
    "c1024_learned": dict(n=1024, k0=32.0, urms=0.3, rho_amp=0.2, vel_seed=1005, scal_seed=2005),
}


def workload_fields(name: str, device="cpu", n=None):
    p = dict(WORKLOADS[name])
    if n is not None:
        p["k0"] = p["k0"] * n / p["n"]
        p["n"] = n
    return turbulence(device=device, **p)


def workload_temperature(name: str, amp: float = 0.05, device="cpu", n=None):
    """Temperature theta = 1 + amp s (float32, (n, n, n)) for a named workload: s is a
    spectral scalar with the workload's spectrum and its own seed (scalar seed + 1000)."""
    p = dict(WORKLOADS[name])
    if n is not None:
        p["k0"] = p["k0"] * n / p["n"]
        p["n"] = n
    s = spectral_scalar(p["n"], p["k0"], p["scal_seed"] + 1000, device)
    return (1.0 + amp * s).to(torch.float32)


def grid_coords(n: int, dtype=np.float64):
    """Coordinates X, Y, Z in [0, 2 pi) broadcast as (z, y, x)."""
    x = 2.0 * np.pi * np.arange(n, dtype=dtype) / n
    return x.reshape(1, 1, n), x.reshape(1, n, 1), x.reshape(n, 1, 1)


def taylor_green(n: int, u0: float = 0.1, rho_fluct: float = 0.0, dtype=np.float32):
    """Taylor-Green initial velocity and density (numpy float32).

    u_x = u0 sin X cos Y cos Z, u_y = -u0 cos X sin Y cos Z, u_z = 0;
    rho = 1 + rho_fluct * (cos 2X + cos 2Y)(cos 2Z + 2).
    """
    X, Y, Z = grid_coords(n)
    ux = u0 * np.sin(X) * np.cos(Y) * np.cos(Z)
    uy = -u0 * np.cos(X) * np.sin(Y) * np.cos(Z)
    uz = np.zeros((n, n, n))
    u = np.stack([np.broadcast_to(ux, (n, n, n)), np.broadcast_to(uy, (n, n, n)), uz])
    rho = 1.0 + rho_fluct * (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0)
    rho = np.broadcast_to(rho, (n, n, n))
    return np.ascontiguousarray(rho, dtype=dtype), np.ascontiguousarray(u, dtype=dtype)


def single_mode(n: int, kvec, avec, phase: float = 0.0, rho_b: float = 0.0, qvec=(0, 0, 0),
                rho_phase: float = 0.0, dtype=np.float64):
    """u_i = a_i cos(k.x + phase); rho = 1 + b cos(q.x + rho_phase). Returns (rho, u) arrays."""
    X, Y, Z = grid_coords(n)
    phi = kvec[0] * X + kvec[1] * Y + kvec[2] * Z + phase
    u = np.stack([np.broadcast_to(a * np.cos(phi), (n, n, n)) for a in avec])
    psi = qvec[0] * X + qvec[1] * Y + qvec[2] * Z + rho_phase
    rho = np.broadcast_to(1.0 + rho_b * np.cos(psi), (n, n, n))
    return np.ascontiguousarray(rho, dtype=dtype), np.ascontiguousarray(u, dtype=dtype)


def random_fields(shape, seed: int, urms: float = 0.3, rho_amp: float = 0.1, dtype=np.float32):
    """White-noise fields for small ragged grids (nz, ny, nx): rho in [1-amp, 1+amp]."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    u = rng.standard_normal((3, nz, ny, nx)) * (urms / math.sqrt(3.0))
    rho = 1.0 + rho_amp * (2.0 * rng.random((nz, ny, nx)) - 1.0)
    return rho.astype(dtype), u.astype(dtype)

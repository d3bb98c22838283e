"""Spectral judge of the coarse runs (host, numpy FFT).

E(k) = 1/2 sum over the shell k - 1/2 <= |kappa| < k + 1/2 of
(|u_hat(kappa)|^2 + |b_hat(kappa)|^2), with u_hat = FFT2(u) / (Nx Ny) and
integer mode vectors kappa.  Fine fields are box-filtered onto the coarse
grid before the transform.  eps_spec = sqrt(mean_{k=1..K} (E_c(k)/E_ref(k)
- 1)^2).  "Within 5 %" means eps_spec <= 0.05 and the kinetic and magnetic
energies within 5 % at every compared time.
"""
from __future__ import annotations

import numpy as np


def box_filter(field: np.ndarray, factor: int) -> np.ndarray:
    """Average a [..., ny, nx] array over factor x factor blocks."""
    *lead, ny, nx = field.shape
    f = field.reshape(*lead, ny // factor, factor, nx // factor, factor)
    return f.mean(axis=(-1, -3))


def shell_spectrum(u: np.ndarray, b: np.ndarray) -> np.ndarray:
    """E(k) for k = 0..N/2 of vector fields u, b [2][N][N]."""
    n = u.shape[-1]
    e = np.zeros((n, n))
    for f in (u[0], u[1], b[0], b[1]):
        h = np.fft.fft2(f) / (n * n)
        e += 0.5 * np.abs(h) ** 2
    k = np.fft.fftfreq(n, 1.0 / n)
    kk = np.sqrt(k[:, None] ** 2 + k[None, :] ** 2)
    shell = np.floor(kk + 0.5).astype(int)
    return np.bincount(shell.ravel(), weights=e.ravel(), minlength=n)[: n // 2 + 1]


def kinetic_magnetic_spectra(u: np.ndarray, b: np.ndarray):
    """The two parts of E(k): (E_u(k), E_b(k)), E = E_u + E_b."""
    z = np.zeros_like(u)
    return shell_spectrum(u, z), shell_spectrum(z, b)


def eps_spec(e_c: np.ndarray, e_ref: np.ndarray, kmax: int) -> float:
    r = e_c[1:kmax + 1] / e_ref[1:kmax + 1]
    return float(np.sqrt(np.mean((r - 1.0) ** 2)))


def energies(u: np.ndarray, b: np.ndarray):
    n = u.shape[-1] * u.shape[-2]
    return float(np.sum(u ** 2) / (2 * n)), float(np.sum(b ** 2) / (2 * n))

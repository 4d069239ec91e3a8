"""Fourier coefficients of an incident plane wave (paper Prop. 4).

Oracle module (test infrastructure only).

For u_inc(x) = exp(i k beta_hat . x), beta_hat = (cos beta, sin beta):
  U^p_m = d^p_m J_m(k a_p),  d^p_m = sqrt(2 pi a_p) exp(i k beta_hat . b_p) exp(i m (pi/2 - beta))
with b_p the vector from the origin to O_p.  The EFIE system is L rho = -U (sec. 5).
"""
from __future__ import annotations

import numpy as np

from .bessel import besselj
from .geometry import mode_index


def planewave(centers, radii, n_modes, k, betas):
    """U for each incidence angle: shape [R, N_tot] (complex128)."""
    c = np.asarray(centers, dtype=np.float64)
    a = np.asarray(radii, dtype=np.float64)
    betas = np.atleast_1d(np.asarray(betas, dtype=np.float64))
    disk, m = mode_index(n_modes)
    kbp = k * (np.cos(betas)[:, None] * c[disk, 0][None, :]
               + np.sin(betas)[:, None] * c[disk, 1][None, :])
    d = (np.sqrt(2.0 * np.pi * a[disk])[None, :] * np.exp(1j * kbp)
         * np.exp(1j * m[None, :] * (0.5 * np.pi - betas[:, None])))
    return d * besselj(m, k * a[disk])[None, :]

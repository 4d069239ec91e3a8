"""Far field of the single-layer potential (paper sec. 4.4).

Oracle module (test infrastructure only).

u(r, theta) ~ exp(i k r) r^{-1/2} a_L(theta), with a_L(theta) = (a_L)^T rho and
  (a_L)^p_m = (i e^{-i pi/4} sqrt(a_p) / (2 sqrt(k))) exp(-i b_p k cos(theta - alpha_p))
              J_m(k a_p) exp(i m (theta - pi/2)),
(b_p, alpha_p) the polar coordinates of O_p.  The transpose is plain (the far
field uses the bilinear product).
"""
from __future__ import annotations

import numpy as np

from .bessel import besselj
from .geometry import mode_index


def farfield_rows(centers, radii, n_modes, k, thetas):
    """The row vectors (a_L)(theta_j), shape [n_theta, N_tot]."""
    c = np.asarray(centers, dtype=np.float64)
    a = np.asarray(radii, dtype=np.float64)
    th = np.atleast_1d(np.asarray(thetas, dtype=np.float64))
    disk, m = mode_index(n_modes)
    bp = np.hypot(c[:, 0], c[:, 1])[disk]
    alp = np.arctan2(c[:, 1], c[:, 0])[disk]
    pref = 1j * np.exp(-0.25j * np.pi) * np.sqrt(a[disk]) / (2.0 * np.sqrt(k))
    return (pref[None, :] * np.exp(-1j * k * bp[None, :] * np.cos(th[:, None] - alp[None, :]))
            * besselj(m, k * a[disk])[None, :]
            * np.exp(1j * m[None, :] * (th[:, None] - 0.5 * np.pi)))


def farfield(centers, radii, n_modes, k, thetas, rho):
    """a(theta_j) = (a_L)(theta_j)^T rho.  rho: [N_tot] or [R, N_tot];
    returns [n_theta] or [R, n_theta]."""
    G = farfield_rows(centers, radii, n_modes, k, thetas)
    rho = np.asarray(rho)
    return rho @ G.T if rho.ndim == 2 else G @ rho

"""Near field: single- and double-layer potentials at points of the propagation
domain, and the total field (paper sec. 4.4, Graf's addition theorem).

Oracle module (test infrastructure only).

For x outside every disk, with (r_p, theta_p) the polar coordinates of x - O_p,
  L rho(x)   =  sum_p sum_m rho^p_m (i pi a_p / 2) J_m(k a_p) H_m(k r_p) e^{i m theta_p} / sqrt(2 pi a_p)
  M lam(x)   = -sum_p sum_m lam^p_m (i pi k a_p / 2) J'_m(k a_p) H_m(k r_p) e^{i m theta_p} / sqrt(2 pi a_p)
(e^{i m theta_p} / sqrt(2 pi a_p) is the basis function Phi^p_m continued off the
circle).  The scattered field of a formulation with far-field weights (f_L, f_M)
is u = f_L L rho + f_M M rho; the total field adds u_inc = e^{i k beta_hat . x}.
Points inside a disk get 0.
"""
from __future__ import annotations

import numpy as np

from .bessel import besselj, besselj_d, hankel1
from .geometry import mode_offsets


def potential(centers, radii, n_modes, k, dens, points, f_L=1.0, f_M=0.0):
    """f_L L dens + f_M M dens at points [P, 2]; dens [N_tot] or [R, N_tot];
    returns [P] or [R, P] (0 at points inside a disk)."""
    c = np.asarray(centers, dtype=np.float64)
    a = np.asarray(radii, dtype=np.float64)
    n_modes = np.asarray(n_modes)
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 2)
    d = np.atleast_2d(np.asarray(dens, dtype=np.complex128))
    off, _ = mode_offsets(n_modes)
    out = np.zeros((d.shape[0], len(pts)), dtype=np.complex128)
    inside = np.zeros(len(pts), dtype=bool)
    for p in range(len(a)):
        dx, dy = pts[:, 0] - c[p, 0], pts[:, 1] - c[p, 1]
        r = np.hypot(dx, dy)
        inside |= r < a[p]
        th = np.arctan2(dy, dx)
        m = np.arange(-n_modes[p], n_modes[p] + 1)
        coef = (0.5j * np.pi * a[p] / np.sqrt(2 * np.pi * a[p])) * (
            f_L * besselj(m, k * a[p]) - f_M * k * besselj_d(m, k * a[p]))
        rr = np.where(r < a[p], a[p], r)
        basis = hankel1(m[None, :], k * rr[:, None]) * np.exp(1j * m[None, :] * th[:, None])  # [P, n]
        out += (d[:, off[p]:off[p + 1]] * coef[None, :]) @ basis.T
    out[:, inside] = 0.0
    return out if np.asarray(dens).ndim == 2 else out[0]


def total_field(centers, radii, n_modes, k, dens, points, betas, f_L=1.0, f_M=0.0):
    """u_inc + u for each incidence (dens [R, N_tot], betas [R]); 0 inside disks."""
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 2)
    betas = np.atleast_1d(np.asarray(betas, dtype=np.float64))
    u = np.atleast_2d(potential(centers, radii, n_modes, k, dens, pts, f_L, f_M))
    uinc = np.exp(1j * k * (np.cos(betas)[:, None] * pts[None, :, 0] + np.sin(betas)[:, None] * pts[None, :, 1]))
    c = np.asarray(centers, dtype=np.float64)
    a = np.asarray(radii, dtype=np.float64)
    inside = np.zeros(len(pts), dtype=bool)
    for p in range(len(a)):
        inside |= np.hypot(pts[:, 0] - c[p, 0], pts[:, 1] - c[p, 1]) < a[p]
    t = uinc + u
    t[:, inside] = 0.0
    return t

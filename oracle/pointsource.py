"""Incident wave of a point source: Fourier coefficients of its trace and
normal-derivative trace (paper Prop. 5) and the incident field itself.

Oracle module (test infrastructure only).

For u_inc(x) = G(x, s) = (i/4) H_0(k |x - s|) with s outside every disk, and
(r_p, theta_p) the polar coordinates of s - O_p (r_p > a_p):
  U^p_m  = (i pi a_p / 2) J_m(k a_p)  H_m(k r_p) conj(Phi~^p_m(s)),
  dU^p_m = k (i pi a_p / 2) J'_m(k a_p) H_m(k r_p) conj(Phi~^p_m(s)),
with Phi~^p_m(s) = e^{i m theta_p} / sqrt(2 pi a_p), the basis function of disk
p continued off its circle.  Every formulation takes these in place of the
plane-wave U, dU (the system does not change).
"""
from __future__ import annotations

import numpy as np

from .bessel import besselj, besselj_d, hankel1
from .geometry import mode_index


def _polar(centers, disk, sources):
    c = np.asarray(centers, dtype=np.float64)
    s = np.atleast_2d(np.asarray(sources, dtype=np.float64))
    dx = s[:, None, 0] - c[disk, 0][None, :]
    dy = s[:, None, 1] - c[disk, 1][None, :]
    return np.hypot(dx, dy), np.arctan2(dy, dx)


def _coef(centers, radii, n_modes, k, sources):
    disk, m = mode_index(n_modes)
    a = np.asarray(radii, dtype=np.float64)[disk]
    r, th = _polar(centers, disk, sources)
    if np.any(r <= a[None, :]):
        raise ValueError("a point source lies inside or on a disk")
    w = (0.5j * np.pi * a / np.sqrt(2 * np.pi * a))[None, :] * hankel1(m[None, :], k * r) * np.exp(-1j * m[None, :] * th)
    return w, m, a


def point_source(centers, radii, n_modes, k, sources):
    """U for sources [R, 2]: shape [R, N_tot]."""
    w, m, a = _coef(centers, radii, n_modes, k, sources)
    return w * besselj(m, k * a)[None, :]


def point_source_dn(centers, radii, n_modes, k, sources):
    """dU for sources [R, 2]: shape [R, N_tot]."""
    w, m, a = _coef(centers, radii, n_modes, k, sources)
    return w * (k * besselj_d(m, k * a))[None, :]


def incident(k, sources, points):
    """(i/4) H_0(k |x - s|): shape [R, P]."""
    s = np.atleast_2d(np.asarray(sources, dtype=np.float64))
    x = np.asarray(points, dtype=np.float64).reshape(-1, 2)
    d = np.hypot(x[None, :, 0] - s[:, None, 0], x[None, :, 1] - s[:, None, 1])
    return 0.25j * hankel1(0, k * d)

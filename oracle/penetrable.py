"""Transmission problem for penetrable disks (paper sec. 7, Example II).

Oracle module (test infrastructure only).

Wavenumber k+ outside, k-_p inside disk p, and the transmission conditions
u+ - u- = -u_inc, d_n u+ - mu_p d_n u- = -d_n u_inc on Gamma.  Single-layer
representations u+ = L+ rho+ (exterior wavenumber) and u- = L- rho- give, with
the jump relations of sec. 3 (exterior trace d_n L -> -I/2 + N, interior trace
d_n L -> I/2 + N, one outward normal), the block system

  [ L+            -L-             ] [rho+]   [ -U  ]
  [ -I/2 + N+     -mu (I/2 + N-)  ] [rho-] = [ -dU ]

(the (2,2) block is printed with a + sign, which contradicts the -L- of the
first row and the jump relations: with k- = k+ and mu = 1 it does not give a
vanishing scattered field, while the - sign does);

where L+, N+ are the exterior operators of the EFIE/operators oracles at k+.
Each interior field lives in its own disk with its own k-_p, so L- and N- are
the self blocks only: (i pi a/2) J_m H_m and -1/2 + (i pi k a/2) J'_m H_m at
k-_p a_p, diagonal in m (I/2 + N- = (i pi k- a/2) J'_m H_m).  The far field is
a_L(k+) rho+; the interior field of disk p is
u-(x) = sum_m rho-_m (i pi a/2) H_m(k- a) J_m(k- r) e^{i m theta} / sqrt(2 pi a).
"""
from __future__ import annotations

import numpy as np

from .bessel import besselj, besselj_d, hankel1
from .farfield import farfield_rows
from .geometry import mode_index, mode_offsets
from .operators import operator_matrix, planewave_dn
from .rhs import planewave


def interior_diagonals(radii, n_modes, k_int):
    """Per unknown: L-_{mm} = (i pi a/2) J H and (I/2 + N-)_{mm} = (i pi k a/2) J' H at k-_p a_p."""
    disk, m = mode_index(n_modes)
    a = np.asarray(radii, dtype=np.float64)[disk]
    ki = np.asarray(k_int, dtype=np.float64)[disk]
    x = ki * a
    H = hankel1(m, x)
    return 0.5j * np.pi * a * besselj(m, x) * H, 0.5j * np.pi * ki * a * besselj_d(m, x) * H


def system(centers, radii, n_modes, k, k_int, mu=None):
    """The 2 N_tot x 2 N_tot block matrix."""
    n_modes = np.asarray(n_modes)
    mu = np.ones(len(n_modes)) if mu is None else np.asarray(mu, dtype=np.float64)
    disk, _ = mode_index(n_modes)
    Lp = operator_matrix("L", centers, radii, n_modes, k)
    Np = operator_matrix("N", centers, radii, n_modes, k)
    Lm, Nm = interior_diagonals(radii, n_modes, k_int)
    n = Lp.shape[0]
    A = np.zeros((2 * n, 2 * n), dtype=np.complex128)
    A[:n, :n] = Lp
    A[:n, n:] = -np.diag(Lm)
    A[n:, :n] = Np - 0.5 * np.eye(n)
    A[n:, n:] = -np.diag(mu[disk] * Nm)
    return A


def solve(centers, radii, n_modes, k, k_int, betas, mu=None):
    """(rho+ [R, N_tot], rho- [R, N_tot]) for plane waves of incidence betas."""
    U = planewave(centers, radii, n_modes, k, betas)
    dU = planewave_dn(centers, radii, n_modes, k, betas)
    return solve_coefficients(centers, radii, n_modes, k, k_int, U, dU, mu)


def solve_coefficients(centers, radii, n_modes, k, k_int, U, dU, mu=None):
    """(rho+, rho-) for given trace coefficients U, dU [R, N_tot] of the
    incident wave (plane wave, Prop. 4; point source, Prop. 5)."""
    A = system(centers, radii, n_modes, k, k_int, mu)
    U, dU = np.atleast_2d(U), np.atleast_2d(dU)
    x = np.linalg.solve(A, np.concatenate([-U, -dU], axis=1).T).T
    n = U.shape[1]
    return x[:, :n], x[:, n:]


def farfield(centers, radii, n_modes, k, rho_plus, thetas):
    return np.atleast_2d(rho_plus) @ farfield_rows(centers, radii, n_modes, k, thetas).T


def interior_field(centers, radii, n_modes, k_int, rho_minus, p, points):
    """u- of disk p at points [P, 2] (inside disk p); rho_minus [N_tot]."""
    c = np.asarray(centers, dtype=np.float64)[p]
    a = float(np.asarray(radii)[p])
    ki = float(np.asarray(k_int)[p])
    off, _ = mode_offsets(n_modes)
    m = np.arange(-n_modes[p], n_modes[p] + 1)
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 2)
    r = np.hypot(pts[:, 0] - c[0], pts[:, 1] - c[1])
    th = np.arctan2(pts[:, 1] - c[1], pts[:, 0] - c[0])
    coef = rho_minus[off[p]:off[p + 1]] * (0.5j * np.pi * a) * hankel1(m, ki * a) / np.sqrt(2 * np.pi * a)
    return (besselj(m[None, :], ki * r[:, None]) * np.exp(1j * m[None, :] * th[:, None])) @ coef

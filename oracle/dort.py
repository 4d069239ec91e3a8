"""Time-reversal operator of a far-field mirror and its Herglotz waves (the
DORT experiment of the paper's Example III, sec. 7, in its far-field form).

Oracle module (test infrastructure only).

A mirror at infinity with N_alpha cells at the angles alpha_j = 2 pi j / N_alpha
sends plane waves exp(i k alpha_hat_j . x) and records the far field in the
opposite direction, alpha_i + pi:
  F[i, j] = a(alpha_i + pi; alpha_j)                 (far field of incidence j)
  T = conj(F)^T F                                      (time-reversal matrix)
An eigenvector g of T parameterises the discrete Herglotz wave
  u_I(x) = sum_j h g_j exp(i k (x_1 cos alpha_j + x_2 sin alpha_j)),  h = 2 pi / N_alpha,
which focuses on one obstacle when its eigenvalue is significant.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .farfield import farfield_rows
from .operator import efie_matrix
from .rhs import planewave


def mirror_angles(n_alpha: int) -> np.ndarray:
    """alpha_j = 2 pi j / N_alpha, j = 0..N_alpha-1."""
    return 2.0 * np.pi * np.arange(n_alpha) / n_alpha


def farfield_matrix(centers, radii, n_modes, k, n_alpha):
    """F[i, j] = a(alpha_i + pi; alpha_j) of the EFIE solution (dense LU),
    shape [N_alpha, N_alpha]."""
    al = mirror_angles(n_alpha)
    L = efie_matrix(centers, radii, n_modes, k)
    U = planewave(centers, radii, n_modes, k, al)            # [N_alpha (incidence), N_tot]
    rho = sla.lu_solve(sla.lu_factor(L), -U.T)                # [N_tot, N_alpha]
    G = farfield_rows(centers, radii, n_modes, k, al + np.pi)  # [N_alpha (receiver), N_tot]
    return G @ rho


def time_reversal(F):
    """T = conj(F)^T F (Hermitian, positive semi-definite)."""
    F = np.asarray(F)
    return F.conj().T @ F


def eig_desc(T):
    """Eigenvalues in decreasing order and the matching unit eigenvectors
    (columns) of the Hermitian matrix T."""
    w, V = np.linalg.eigh(T)
    order = np.argsort(w)[::-1]
    return w[order], V[:, order]


def herglotz(n_alpha, f, k, points):
    """u_I at points [P, 2] for the parameter f [N_alpha] (plain double sum)."""
    al = mirror_angles(n_alpha)
    h = 2.0 * np.pi / n_alpha
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 2)
    ph = k * (pts[:, 0:1] * np.cos(al)[None, :] + pts[:, 1:2] * np.sin(al)[None, :])
    return np.exp(1j * ph) @ (h * np.asarray(f, dtype=np.complex128))

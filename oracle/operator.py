"""Dense truncated EFIE matrix and its single-scattering preconditioning.

Oracle module (test infrastructure only).

Paper sec. 4.2 (block formulas) and sec. 5 (truncation, system, preconditioner):

  L^{pp}_{mm} = (i pi a_p / 2) J_m(k a_p) H_m(k a_p)                 (diagonal blocks)
  L^{pq}_{mn} = (i pi sqrt(a_p a_q) / 2) J_m(k a_p) [(S^{pq})^T]_{mn} J_n(k a_q)
  S^{pq}_{mn} = H_{m-n}(k b_pq) exp(i (m-n) alpha_pq)   (so (S^T)_{mn} = H_{n-m} e^{i(n-m)alpha})

for m = -N_p..N_p, n = -N_q..N_q.  The separation matrix prints alpha_{bq};
it is read as alpha_pq (the only angle defined for the pair).  The transpose is
the plain transpose.  The preconditioner is the block diagonal of L (single
scattering, sec. 5): D = diag(L^{pp}), applied on the left, A = D^{-1} L.
"""
from __future__ import annotations

import numpy as np

from .bessel import besselj, hankel1
from .geometry import mode_index, mode_offsets, pair_geometry


def pair_hankel_table(centers, k, nu_max):
    """H_nu(k b_pq) for nu = 0..nu_max and every ordered pair (p, q), p != q
    (entries with p == q are left as 0).  Shape [M, M, nu_max + 1]."""
    b, _ = pair_geometry(centers)
    M = b.shape[0]
    bb = b.copy()
    np.fill_diagonal(bb, 1.0)
    nu = np.arange(nu_max + 1)
    H = hankel1(nu[None, None, :], k * bb[:, :, None])
    H[np.arange(M), np.arange(M), :] = 0.0
    return H


def efie_diagonal(radii, n_modes, k):
    """D_i = L^{pp}_{mm} = (i pi a_p / 2) J_m(k a_p) H_m(k a_p) for every unknown i."""
    disk, m = mode_index(n_modes)
    a = np.asarray(radii, dtype=np.float64)[disk]
    return 0.5j * np.pi * a * besselj(m, k * a) * hankel1(m, k * a)


def efie_row_block(centers, radii, n_modes, k, p):
    """Rows of disk p of L: the (2N_p+1) x N_tot block [L^{p1} ... L^{pM}]."""
    n_modes = np.asarray(n_modes)
    a = np.asarray(radii, dtype=np.float64)
    off, N = mode_offsets(n_modes)
    disk, m = mode_index(n_modes)
    b, alpha = pair_geometry(centers)
    nu_max = int(n_modes[p]) + int(np.max(n_modes))
    bp = b[p].copy()
    bp[p] = 1.0
    Hrow = hankel1(np.arange(nu_max + 1)[None, :], k * bp[:, None])   # H_nu(k b_pq)
    rows = slice(off[p], off[p + 1])
    mi = m[rows]
    nu = m[None, :] - mi[:, None]                         # n - m
    anu = np.abs(nu)
    sign = np.where((nu < 0) & (anu % 2 == 1), -1.0, 1.0)
    Hv = Hrow[disk[None, :], anu] * sign                  # H_{n-m}(k b_pq)
    ph = np.exp(1j * nu * alpha[p][disk][None, :])        # e^{i(n-m) alpha_pq}
    cpq = 0.5j * np.pi * np.sqrt(a[p] * a[disk])[None, :]
    Jcol = besselj(m, k * a[disk])                        # J_n(k a_q) per column unknown
    blk = cpq * besselj(mi, k * a[p])[:, None] * Hv * ph * Jcol[None, :]
    blk[:, off[p]:off[p + 1]] = 0.0
    d = efie_diagonal(a, n_modes, k)[rows]
    blk[np.arange(len(mi)), off[p] + np.arange(len(mi))] = d
    return blk


def efie_matrix(centers, radii, n_modes, k):
    """Dense N_tot x N_tot complex128 matrix L of the truncated EFIE (sec. 5)."""
    n_modes = np.asarray(n_modes)
    off, N = mode_offsets(n_modes)
    L = np.zeros((N, N), dtype=np.complex128)
    for p in range(len(n_modes)):
        L[off[p]:off[p + 1], :] = efie_row_block(centers, radii, n_modes, k, p)
    return L


def preconditioned(L, D):
    """A = D^{-1} L (left single-scattering preconditioning, sec. 5)."""
    return L / D[:, None]


def mode_flip(n_modes):
    """Permutation P mapping unknown (p, m) to (p, -m), as an index array:
    (P x)_i = x_{flip[i]}."""
    off, _ = mode_offsets(n_modes)
    disk, m = mode_index(n_modes)
    return (off[disk] + (np.asarray(n_modes)[disk] - m)).astype(np.int64)

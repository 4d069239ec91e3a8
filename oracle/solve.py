"""Solvers for the truncated EFIE L rho = -U (paper sec. 5).

Oracle module (test infrastructure only).

  * ``solve_lu``: the direct (Gauss) solve, the parity reference.
  * ``gmres``: textbook restarted GMRES(m) (Saad, Iterative Methods for Sparse
    Linear Systems, Arnoldi with modified Gram-Schmidt and Givens rotations),
    used by the paper with the single-scattering preconditioner.  It is run on
    the left-preconditioned system A x = f, A = D^{-1} L, f = -D^{-1} U, from
    x0 = 0 unless given.  Outputs follow the paper's solver call: x, FLAG,
    RELRES, ITER, RESVEC.  Conventions where the paper is silent: ``maxit``
    counts inner iterations (operator applications inside the Arnoldi
    process), RELRES is the true relative residual ||f - A x|| / ||f||
    recomputed at exit, RESVEC holds the Arnoldi estimates |g_{j+1}| / ||f||
    (index 0 is the initial relative residual), FLAG is 0 when RELRES <= tol,
    1 when maxit was reached, 2 on a non-finite value.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def solve_lu(L, rhs):
    """x = L^{-1} rhs by LU with partial pivoting; rhs [N] or [N, R]."""
    return sla.lu_solve(sla.lu_factor(L), rhs)


def efie_solve_lu(L, U):
    """rho = L^{-1} (-U) for U of shape [R, N_tot]; returns [R, N_tot]."""
    return solve_lu(L, -np.asarray(U).T).T


def _givens(a, b):
    """Complex Givens rotation (c real, s complex) with
    [c, s; -conj(s), c] [a; b] = [r; 0]."""
    if b == 0:
        return 1.0, 0.0j
    if a == 0:
        return 0.0, 1.0 + 0.0j
    rho = np.hypot(abs(a), abs(b))
    c = abs(a) / rho
    s = (a / abs(a)) * np.conj(b) / rho
    return c, s


def gmres(apply, f, restart, tol, maxit, x0=None):
    """Restarted GMRES(restart) for apply(x) = A x = f.

    Returns (x, flag, relres, iters, resvec)."""
    f = np.asarray(f, dtype=np.complex128)
    n = f.shape[0]
    normf = np.linalg.norm(f)
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    if normf == 0.0:
        return np.zeros(n, dtype=np.complex128), 0, 0.0, 0, np.zeros(1)
    r = f - apply(x) if x0 is not None else f.copy()
    beta = np.linalg.norm(r)
    resvec = [beta / normf]
    iters = 0
    flag = 1
    if beta / normf <= tol:
        return x, 0, beta / normf, 0, np.array(resvec)
    while iters < maxit:
        V = np.zeros((restart + 1, n), dtype=np.complex128)
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart)
        sn = np.zeros(restart, dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        V[0] = r / beta
        g[0] = beta
        j_end = 0
        breakdown = False
        for j in range(restart):
            w = apply(V[j])
            iters += 1
            for i in range(j + 1):               # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if not np.isfinite(H[j + 1, j]):
                return x, 2, np.nan, iters, np.array(resvec)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            else:
                breakdown = True
            for i in range(j):                   # previous rotations on column j
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            resvec.append(abs(g[j + 1]) / normf)
            j_end = j + 1
            if abs(g[j + 1]) / normf <= tol or breakdown or iters >= maxit:
                break
        y = sla.solve_triangular(H[:j_end, :j_end], g[:j_end])
        x = x + V[:j_end].T @ y
        r = f - apply(x)
        beta = np.linalg.norm(r)
        if not np.isfinite(beta):
            return x, 2, np.nan, iters, np.array(resvec)
        if beta / normf <= tol:
            flag = 0
            break
        if breakdown:
            break
    return x, flag, beta / normf, iters, np.array(resvec)

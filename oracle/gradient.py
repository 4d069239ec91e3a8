"""Far-field misfit and its gradient w.r.t. disk centers, radii and k.

Oracle module (test infrastructure only).  The paper has no gradients; this
is the adjoint of its forward map, derived from the sec. 4.2 block formulas,
Prop. 4 and the sec. 4.4 far-field vector, with the truncation orders N_p
held fixed.

  rho_beta = L^{-1}(-U_beta),  a_{beta,r} = g_r^T rho_beta,  e = a - a_target,
  loss = sum_{beta, r} |e_{beta,r}|^2,
  c_beta = sum_r conj(e_{beta,r}) g_r,   L^T lambda_beta = c_beta,
  d loss / ds = 2 Re sum_beta [ sum_r conj(e_{beta,r}) (d g_r / ds)^T rho_beta
                                - lambda_beta^T (dL/ds rho_beta + dU_beta/ds) ].

Derivatives are written by the chain rule on each factor of the block formulas:
the separation symbol t_nu = H_nu(k b) e^{i nu alpha} is differentiated through
b and alpha of the vector O_p - O_q, and H'_nu = (H_{nu-1} - H_{nu+1})/2.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .bessel import besselj, besselj_d, hankel1, hankel1_d
from .farfield import farfield_rows
from .geometry import mode_index, mode_offsets, pair_geometry
from .operator import efie_matrix, pair_hankel_table
from .rhs import planewave


def forward(centers, radii, n_modes, k, betas, thetas):
    """Far field a [R, n_theta] of the EFIE solution (dense LU)."""
    L = efie_matrix(centers, radii, n_modes, k)
    U = planewave(centers, radii, n_modes, k, betas)
    rho = sla.lu_solve(sla.lu_factor(L), -U.T).T
    return rho @ farfield_rows(centers, radii, n_modes, k, thetas).T


def misfit(centers, radii, n_modes, k, betas, thetas, target):
    """loss = sum |a - target|^2 (no 1/2, no normalisation)."""
    a = forward(centers, radii, n_modes, k, betas, thetas)
    return float(np.sum(np.abs(a - target) ** 2))


def misfit_grad(centers, radii, n_modes, k, betas, thetas, target):
    """Returns (loss, d_centers [M,2], d_radii [M], d_k) by the adjoint method."""
    c = np.asarray(centers, dtype=np.float64)
    a = np.asarray(radii, dtype=np.float64)
    n_modes = np.asarray(n_modes)
    M = len(a)
    betas = np.atleast_1d(np.asarray(betas, dtype=np.float64))
    thetas = np.atleast_1d(np.asarray(thetas, dtype=np.float64))
    off, N = mode_offsets(n_modes)
    disk, m = mode_index(n_modes)

    L = efie_matrix(c, a, n_modes, k)
    lu = sla.lu_factor(L)
    U = planewave(c, a, n_modes, k, betas)                       # [R, N]
    rho = sla.lu_solve(lu, -U.T).T                               # [R, N]
    G = farfield_rows(c, a, n_modes, k, thetas)                  # [T, N]
    amp = rho @ G.T                                              # [R, T]
    e = amp - target
    loss = float(np.sum(np.abs(e) ** 2))
    C = np.conj(e) @ G                                           # c_beta, [R, N]
    lam = sla.lu_solve(lu, C.T, trans=1).T                       # L^T lambda = c

    dc = np.zeros((M, 2))
    da = np.zeros(M)
    dk = 0.0

    # --- per-unknown factors: s = sqrt(a_p) J_m(k a_p) and its derivatives
    ap = a[disk]
    J = besselj(m, k * ap)
    Jd = besselj_d(m, k * ap)
    s = np.sqrt(ap) * J
    s_a = J / (2.0 * np.sqrt(ap)) + k * np.sqrt(ap) * Jd            # d s / d a_p
    s_k = np.sqrt(ap) * ap * Jd                                     # d s / d k

    # --- off-diagonal blocks: L_ij = (i pi / 2) s_i t_{n-m}(O_p - O_q) s_j
    b, alpha = pair_geometry(c)
    nu_max = 2 * int(np.max(n_modes)) + 1
    Htab = pair_hankel_table(c, k, nu_max)
    Hd_tab = np.zeros_like(Htab)
    Hd_tab[:, :, 1:nu_max] = 0.5 * (Htab[:, :, 0:nu_max - 1] - Htab[:, :, 2:nu_max + 1])
    Hd_tab[:, :, 0] = -Htab[:, :, 1]                              # H'_0 = -H_1
    ih = 0.5j * np.pi
    for p in range(M):
        rows = slice(off[p], off[p + 1])
        mi = m[rows]
        nu = m[None, :] - mi[:, None]
        anu = np.abs(nu)
        sign = np.where((nu < 0) & (anu % 2 == 1), -1.0, 1.0)
        q = disk[None, :]
        H = Htab[p][q, anu] * sign
        Hd = Hd_tab[p][q, anu] * sign
        al = alpha[p][q]
        bb = b[p][q].copy()
        bb[:, off[p]:off[p + 1]] = 1.0
        ph = np.exp(1j * nu * al)
        ca, sa = np.cos(al), np.sin(al)
        T = H * ph
        Tx = (k * Hd * ca - 1j * nu * H * sa / bb) * ph            # d t / d(x_p - x_q)
        Ty = (k * Hd * sa + 1j * nu * H * ca / bb) * ph            # d t / d(y_p - y_q)
        Tk = bb * Hd * ph                                          # d t / d k
        for X in (T, Tx, Ty, Tk):
            X[:, off[p]:off[p + 1]] = 0.0
        Gam = lam[:, rows].T @ rho                                 # sum_beta lambda_i rho_j
        si = s[rows][:, None]
        sj = s[None, :]
        # contraction sum_ij dL_ij Gam_ij, reduced per column disk
        def per_disk(W):
            return np.bincount(disk, weights=np.real(W.sum(axis=0)), minlength=M) + \
                1j * np.bincount(disk, weights=np.imag(W.sum(axis=0)), minlength=M)
        gx = per_disk(ih * si * Tx * sj * Gam)
        gy = per_disk(ih * si * Ty * sj * Gam)
        dc[p, 0] -= 2.0 * np.real(np.sum(gx))
        dc[p, 1] -= 2.0 * np.real(np.sum(gy))
        dc[:, 0] += 2.0 * np.real(gx)
        dc[:, 1] += 2.0 * np.real(gy)
        ga_row = np.sum(ih * s_a[rows][:, None] * T * sj * Gam)
        ga_col = per_disk(ih * si * T * s_a[None, :] * Gam)
        da[p] -= 2.0 * np.real(ga_row)
        da -= 2.0 * np.real(ga_col)
        gk = np.sum(ih * (s_k[rows][:, None] * T * sj + si * Tk * sj + si * T * s_k[None, :]) * Gam)
        dk -= 2.0 * np.real(gk)

    # --- diagonal blocks D_m = (i pi a_p / 2) J_m H_m
    H0 = hankel1(m, k * ap)
    H0d = hankel1_d(m, k * ap)
    gdiag = np.sum(lam * rho, axis=0)                             # sum_beta lambda_i rho_i
    dD_da = ih * (J * H0 + k * ap * (Jd * H0 + J * H0d))
    dD_dk = ih * ap * ap * (Jd * H0 + J * H0d)
    da -= 2.0 * np.real(np.bincount(disk, weights=np.real(dD_da * gdiag), minlength=M)
                        + 1j * np.bincount(disk, weights=np.imag(dD_da * gdiag), minlength=M))
    dk -= 2.0 * np.real(np.sum(dD_dk * gdiag))

    # --- right-hand side U (Prop. 4)
    cb, sb = np.cos(betas)[:, None], np.sin(betas)[:, None]
    phase = (np.exp(1j * k * (cb * c[disk, 0][None, :] + sb * c[disk, 1][None, :]))
             * np.exp(1j * m[None, :] * (0.5 * np.pi - betas[:, None])) * np.sqrt(2.0 * np.pi))
    dUx = 1j * k * cb * U
    dUy = 1j * k * sb * U
    dUa = phase * s_a[None, :]
    dUk = 1j * (cb * c[disk, 0][None, :] + sb * c[disk, 1][None, :]) * U + phase * s_k[None, :]

    def lamdot(dU):
        v = np.sum(lam * dU, axis=0)
        return (np.bincount(disk, weights=np.real(v), minlength=M)
                + 1j * np.bincount(disk, weights=np.imag(v), minlength=M))
    dc[:, 0] -= 2.0 * np.real(lamdot(dUx))
    dc[:, 1] -= 2.0 * np.real(lamdot(dUy))
    da -= 2.0 * np.real(lamdot(dUa))
    dk -= 2.0 * np.real(np.sum(lamdot(dUk)))

    # --- far-field rows g_r (sec. 4.4)
    E = np.conj(e).T @ rho                                        # [T, N]
    ct, st = np.cos(thetas)[:, None], np.sin(thetas)[:, None]
    gphase = (1j * np.exp(-0.25j * np.pi) / (2.0 * np.sqrt(k))
              * np.exp(-1j * k * (ct * c[disk, 0][None, :] + st * c[disk, 1][None, :]))
              * np.exp(1j * m[None, :] * (thetas[:, None] - 0.5 * np.pi)))
    dGx = -1j * k * ct * G
    dGy = -1j * k * st * G
    dGa = gphase * s_a[None, :]
    dGk = (-0.5 / k - 1j * (ct * c[disk, 0][None, :] + st * c[disk, 1][None, :])) * G \
        + gphase * s_k[None, :]

    def edot(dG):
        v = np.sum(dG * E, axis=0)
        return (np.bincount(disk, weights=np.real(v), minlength=M)
                + 1j * np.bincount(disk, weights=np.imag(v), minlength=M))
    dc[:, 0] += 2.0 * np.real(edot(dGx))
    dc[:, 1] += 2.0 * np.real(edot(dGy))
    da += 2.0 * np.real(edot(dGa))
    dk += 2.0 * np.real(np.sum(edot(dGk)))
    return loss, dc, da, float(dk)


def misfit_fd(centers, radii, n_modes, k, betas, thetas, target, h=1e-5):
    """Central differences of ``misfit`` (N_p frozen): (d_centers, d_radii, d_k)."""
    c = np.asarray(centers, dtype=np.float64)
    a = np.asarray(radii, dtype=np.float64)
    f = lambda cc, aa, kk: misfit(cc, aa, n_modes, kk, betas, thetas, target)
    dc = np.zeros_like(c)
    da = np.zeros_like(a)
    for p in range(len(a)):
        for d in range(2):
            cp, cm = c.copy(), c.copy()
            cp[p, d] += h
            cm[p, d] -= h
            dc[p, d] = (f(cp, a, k) - f(cm, a, k)) / (2 * h)
        ap_, am_ = a.copy(), a.copy()
        ap_[p] += h
        am_[p] -= h
        da[p] = (f(c, ap_, k) - f(c, am_, k)) / (2 * h)
    dk = (f(c, a, k + h) - f(c, a, k - h)) / (2 * h)
    return dc, da, float(dk)

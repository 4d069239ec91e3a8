"""The four boundary integral operators L, M, N, D in the Fourier basis and the
integral equations built from them: EFIE, MFIE, CFIE and Brakhage-Werner for a
sound-soft boundary, and the single- and double-layer equations for a
sound-hard one.

Oracle module (test infrastructure only).

Paper sec. 4.2 block formulas, for p != q (S^{pq} the separation matrix of
the EFIE oracle, (S^T)_{mn} = H_{n-m}(k b_pq) e^{i(n-m) alpha_pq}):
  L^{pq} =  (i pi / 2)     sqrt(a_p a_q) J^p  S^T J^q
  M^{pq} = -(i k pi / 2)   sqrt(a_p a_q) J^p  S^T J'^q
  N^{pq} =  (i k pi / 2)   sqrt(a_p a_q) J'^p S^T J^q
  D^{pq} = -(i k^2 pi / 2) sqrt(a_p a_q) J'^p S^T J'^q
and for p = q, per mode m (J, H at k a_p):
  L: (i pi a / 2) J H      M:  1/2 - (i pi k a / 2) J' H
  N: -1/2 + (i pi k a / 2) J' H       D: -(i pi k^2 a / 2) J' H'.
The D diagonal is printed with a + sign; the normal derivative at r = a of the
double-layer potential of a mode, -(i pi k a / 2) J'_m k H'_m, the off-diagonal D
blocks and the sound-hard single-disk solution all give the - sign used here.
Incident plane wave (Prop. 4): U = d J, dU = k d J' (normal-derivative trace).
Far fields (sec. 4.4): a = a_L^T rho + a_M^T lambda with
  (a_L)^p_m = (i e^{-i pi/4} sqrt(a_p) / (2 sqrt k)) e^{-i k b_p cos(theta - alpha_p)} J_m e^{i m (theta - pi/2)}
  (a_M)^p_m = -k (J'_m / J_m) (a_L)^p_m.
The sign of a_M is the one of the double-layer potential's Fourier expansion
(M Phi^p_m(x) = -(i pi k a_p / 2) J'_m H_m(k r_p) e^{i m theta_p} / sqrt(2 pi a_p)),
whose large-r form gives exactly this vector; the printed far-field vector has
the opposite sign, at odds with that expansion and with the M blocks above.

Formulations (the jump relations of sec. 3 for the exterior trace: M -> -1/2 + M,
d_n L -> -1/2 + N):
  efie        L rho = -U                                     a = a_L rho
  mfie        (1/2 + N) rho = -dU                             a = a_L rho
  cfie        (alpha eta L + (1 - alpha)(1/2 + N)) rho = -alpha eta U - (1 - alpha) dU
  bwie        (1/2 - eta L - M) psi = -U                      a = -(eta a_L + a_M) psi
              (from u = -(eta L + M) psi; the printed script passes +U, which
              with that representation gives -u on the boundary)
  neumann_sl  (-1/2 + N) rho = -dU        (u = L rho, d_n u_tot = 0)     a = a_L rho
  neumann_dl  D lam = -dU                 (u = M lam, d_n u_tot = 0)     a = a_M lam
"""
from __future__ import annotations

import numpy as np

from .bessel import besselj, besselj_d, hankel1, hankel1_d
from .farfield import farfield_rows
from .geometry import mode_index, mode_offsets, pair_geometry
from .rhs import planewave

# (scalar, row factor, column factor) of the off-diagonal blocks
_OFFDIAG = {
    "L": (lambda k: 0.5j * np.pi, "J", "J"),
    "M": (lambda k: -0.5j * k * np.pi, "J", "Jd"),
    "N": (lambda k: 0.5j * k * np.pi, "Jd", "J"),
    "D": (lambda k: -0.5j * k * k * np.pi, "Jd", "Jd"),
}


def _bess(kind, m, x):
    return besselj(m, x) if kind == "J" else besselj_d(m, x)


def diagonal(name, radii, n_modes, k):
    """Diagonal-block values X^{pp}_{mm} of operator `name` for every unknown."""
    disk, m = mode_index(n_modes)
    a = np.asarray(radii, dtype=np.float64)[disk]
    x = k * a
    if name == "I":
        return np.ones(len(m), dtype=np.complex128)
    if name == "L":
        return 0.5j * np.pi * a * besselj(m, x) * hankel1(m, x)
    if name == "M":
        return 0.5 - 0.5j * np.pi * k * a * besselj_d(m, x) * hankel1(m, x)
    if name == "N":
        return -0.5 + 0.5j * np.pi * k * a * besselj_d(m, x) * hankel1(m, x)
    if name == "D":
        return -0.5j * np.pi * k * k * a * besselj_d(m, x) * hankel1_d(m, x)
    raise ValueError(name)


def operator_matrix(name, centers, radii, n_modes, k):
    """Dense N_tot x N_tot matrix of I, L, M, N or D (truncated, sec. 5)."""
    n_modes = np.asarray(n_modes)
    a = np.asarray(radii, dtype=np.float64)
    off, N = mode_offsets(n_modes)
    X = np.zeros((N, N), dtype=np.complex128)
    if name != "I":
        disk, m = mode_index(n_modes)
        b, alpha = pair_geometry(centers)
        scal, rk, ck = _OFFDIAG[name]
        c = scal(k)
        for p in range(len(n_modes)):
            rows = slice(off[p], off[p + 1])
            mi = m[rows]
            nu_max = int(n_modes[p]) + int(np.max(n_modes))
            bp = b[p].copy()
            bp[p] = 1.0
            Hrow = hankel1(np.arange(nu_max + 1)[None, :], k * bp[:, None])
            nu = m[None, :] - mi[:, None]                       # n - m
            anu = np.abs(nu)
            sign = np.where((nu < 0) & (anu % 2 == 1), -1.0, 1.0)
            St = Hrow[disk[None, :], anu] * sign * np.exp(1j * nu * alpha[p][disk][None, :])
            blk = (c * np.sqrt(a[p] * a[disk])[None, :] * _bess(rk, mi, k * a[p])[:, None] * St
                   * _bess(ck, m, k * a[disk])[None, :])
            blk[:, rows] = 0.0
            X[rows, :] = blk
    X[np.arange(N), np.arange(N)] += diagonal(name, a, n_modes, k)
    return X


def combination(weights, centers, radii, n_modes, k):
    """sum_X w_X X over a dict {name: weight} of I, L, M, N, D."""
    n = int(np.sum(2 * np.asarray(n_modes) + 1))
    A = np.zeros((n, n), dtype=np.complex128)
    for name, w in weights.items():
        if w != 0:
            A += w * operator_matrix(name, centers, radii, n_modes, k)
    return A


def planewave_dn(centers, radii, n_modes, k, betas):
    """Coefficients of the normal-derivative trace of a plane wave (Prop. 4):
    dU^p_m = k d^p_m J'_m(k a_p), d^p_m = sqrt(2 pi a_p) e^{i k beta_hat . b_p}
    e^{i m (pi/2 - beta)}; shape [R, N_tot]."""
    c = np.asarray(centers, dtype=np.float64)
    a = np.asarray(radii, dtype=np.float64)
    betas = np.atleast_1d(np.asarray(betas, dtype=np.float64))
    disk, m = mode_index(n_modes)
    kbp = k * (np.cos(betas)[:, None] * c[disk, 0][None, :] + np.sin(betas)[:, None] * c[disk, 1][None, :])
    d = (np.sqrt(2.0 * np.pi * a[disk])[None, :] * np.exp(1j * kbp)
         * np.exp(1j * m[None, :] * (0.5 * np.pi - betas[:, None])))
    return d * (k * besselj_d(m, k * a[disk]))[None, :]


def farfield_rows_dl(centers, radii, n_modes, k, thetas):
    """Rows (a_M)(theta_j) of the double-layer far field, shape [n_theta, N_tot]."""
    disk, m = mode_index(n_modes)
    a = np.asarray(radii, dtype=np.float64)[disk]
    th = np.atleast_1d(np.asarray(thetas, dtype=np.float64))
    c = np.asarray(centers, dtype=np.float64)
    bp = np.hypot(c[:, 0], c[:, 1])[disk]
    alp = np.arctan2(c[:, 1], c[:, 0])[disk]
    pref = -1j * np.exp(-0.25j * np.pi) * np.sqrt(k * a) / 2.0
    return (pref[None, :] * np.exp(-1j * k * bp[None, :] * np.cos(th[:, None] - alp[None, :]))
            * besselj_d(m, k * a)[None, :] * np.exp(1j * m[None, :] * (th[:, None] - 0.5 * np.pi)))


def formulation(name, alpha=0.5, eta=None, k=None):
    """(operator weights, right-hand-side weights {U, dU}, far-field weights {L, M})."""
    if name == "efie":
        return {"L": 1.0}, {"U": -1.0}, {"L": 1.0}
    if name == "mfie":
        return {"I": 0.5, "N": 1.0}, {"dU": -1.0}, {"L": 1.0}
    if name == "cfie":
        return ({"L": alpha * eta, "I": 0.5 * (1 - alpha), "N": 1 - alpha},
                {"U": -alpha * eta, "dU": -(1 - alpha)}, {"L": 1.0})
    if name == "bwie":
        return {"I": 0.5, "L": -eta, "M": -1.0}, {"U": -1.0}, {"L": -eta, "M": -1.0}
    if name == "neumann_sl":
        return {"I": -0.5, "N": 1.0}, {"dU": -1.0}, {"L": 1.0}
    if name == "neumann_dl":
        return {"D": 1.0}, {"dU": -1.0}, {"M": 1.0}
    raise ValueError(name)


def solve_farfield(name, centers, radii, n_modes, k, betas, thetas, **kw):
    """Density [R, N_tot] (dense solve) and far field [R, n_theta] of a formulation."""
    ops, rw, fw = formulation(name, k=k, **kw)
    A = combination(ops, centers, radii, n_modes, k)
    b = np.zeros((len(np.atleast_1d(betas)), A.shape[0]), dtype=np.complex128)
    if rw.get("U", 0):
        b += rw["U"] * planewave(centers, radii, n_modes, k, betas)
    if rw.get("dU", 0):
        b += rw["dU"] * planewave_dn(centers, radii, n_modes, k, betas)
    dens = np.linalg.solve(A, b.T).T
    G = np.zeros((len(np.atleast_1d(thetas)), A.shape[0]), dtype=np.complex128)
    if fw.get("L", 0):
        G += fw["L"] * farfield_rows(centers, radii, n_modes, k, thetas)
    if fw.get("M", 0):
        G += fw["M"] * farfield_rows_dl(centers, radii, n_modes, k, thetas)
    return dens, dens @ G.T

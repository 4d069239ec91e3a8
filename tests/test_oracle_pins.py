"""Pins of the CPU oracle against things other than itself.

Each test ties one oracle function to a closed form, a quadrature of the
defining integral, an exact identity of the truncated system or brute force,
so that a dropped term, a wrong sign, a wrong index or a transposed operand
in the oracle fails at least one of them.
"""
import math

import mpmath
import numpy as np
import pytest
import scipy.special as sp

import synth
from oracle import bessel, farfield, geometry, gradient, operator, rhs, solve


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


# ---------------------------------------------------------------- Bessel values
def test_bessel_vs_mpmath():
    """J_m and H_m^(1) against 40-digit mpmath on a grid spanning the orders
    and arguments of the workloads (orders up to 60, arguments 0.3..2500)."""
    mpmath.mp.dps = 40
    xs = [0.3, 0.5, 1.7, 3.14159, 7.9, 12.5, 19.0, 31.0, 64.2, 250.0, 1000.3, 2499.0]
    for m in (0, 1, 2, 5, 13, 24, 40, 57, 60):
        for x in xs:
            jr = float(mpmath.besselj(m, x))
            yr = float(mpmath.bessely(m, x))
            h = bessel.hankel1(m, x)
            # AMOS reaches ~1e-13 relative to |H| (at x ~ 1e3 the argument's own
            # rounding already moves the phase by ~1e-13)
            assert abs(h - (jr + 1j * yr)) <= 1e-12 * abs(jr + 1j * yr)
            # J is compared absolutely, scaled by |H| (J alone has zeros)
            assert abs(bessel.besselj(m, x) - jr) <= 1e-12 * abs(jr + 1j * yr)
            # reflection to negative orders is exact
            assert bessel.hankel1(-m, x) == (-1) ** m * h


def test_wronskian():
    """J_{n+1} Y_n - J_n Y_{n+1} = 2 / (pi x)."""
    x = np.array([0.4, 1.0, 3.3, 10.0, 55.5, 700.0])
    for n in range(0, 30):
        # J from besselj (H's real part carries an error ~eps |Y| where J << Y)
        Y0 = bessel.hankel1(n, x).imag
        Y1 = bessel.hankel1(n + 1, x).imag
        w = bessel.besselj(n + 1, x) * Y0 - bessel.besselj(n, x) * Y1
        np.testing.assert_allclose(w, 2.0 / (np.pi * x), rtol=1e-12)


def test_bessel_derivative_vs_scipy():
    x = np.array([0.7, 4.2, 33.0])
    for n in (-3, 0, 2, 11):
        np.testing.assert_allclose(bessel.besselj_d(n, x), sp.jvp(n, x), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(bessel.hankel1_d(n, x), sp.h1vp(n, x), rtol=1e-12)


# ------------------------------------------------ quadrature of defining integrals
def _circle(center, a, Q):
    t = 2.0 * np.pi * np.arange(Q) / Q
    return center[0] + a * np.cos(t), center[1] + a * np.sin(t), t


def test_offdiag_block_vs_quadrature():
    """L^{pq}_{mn} = <L Phi^q_n, Phi^p_m> (Hermitian product on Gamma_p), with
    L Phi(x) = int_{Gamma_q} (i/4) H_0(k|x - y|) Phi(y) dGamma(y), computed by
    the trapezoid rule on both circles (smooth periodic integrand: the disks
    are disjoint)."""
    centers = np.array([[0.3, -0.2], [1.9, 1.1], [-1.4, 1.6]])
    radii = np.array([0.5, 0.7, 0.4])
    n_modes = np.array([4, 6, 3])
    k = 3.1
    L = operator.efie_matrix(centers, radii, n_modes, k)
    off, _ = geometry.mode_offsets(n_modes)
    Q = 96
    for p, q in [(0, 1), (1, 0), (2, 1), (0, 2)]:
        xp, yp, tp = _circle(centers[p], radii[p], Q)
        xq, yq, tq = _circle(centers[q], radii[q], Q)
        G = 0.25j * sp.hankel1(0, k * np.hypot(xp[:, None] - xq[None, :], yp[:, None] - yq[None, :]))
        wq = 2.0 * np.pi * radii[q] / Q
        wp = 2.0 * np.pi * radii[p] / Q
        for mi, m in enumerate(range(-n_modes[p], n_modes[p] + 1)):
            phim = np.exp(1j * m * tp) / np.sqrt(2 * np.pi * radii[p])
            for ni, n in enumerate(range(-n_modes[q], n_modes[q] + 1)):
                phin = np.exp(1j * n * tq) / np.sqrt(2 * np.pi * radii[q])
                val = np.sum(np.conj(phim)[:, None] * G * phin[None, :]) * wq * wp
                got = L[off[p] + mi, off[q] + ni]
                assert abs(got - val) <= 1e-11 * max(1.0, abs(val)), (p, q, m, n, got, val)


def test_planewave_vs_quadrature():
    """U^p_m = <u_inc, Phi^p_m> on Gamma_p (Prop. 4 from its definition)."""
    centers = np.array([[0.3, -0.2], [2.5, 1.0]])
    radii = np.array([0.5, 1.2])
    n_modes = np.array([5, 9])
    k, beta = 4.2, 0.77
    U = rhs.planewave(centers, radii, n_modes, k, [beta])[0]
    off, _ = geometry.mode_offsets(n_modes)
    Q = 128
    for p in range(2):
        x, y, t = _circle(centers[p], radii[p], Q)
        uinc = np.exp(1j * k * (np.cos(beta) * x + np.sin(beta) * y))
        for mi, m in enumerate(range(-n_modes[p], n_modes[p] + 1)):
            phim = np.exp(1j * m * t) / np.sqrt(2 * np.pi * radii[p])
            val = np.sum(uinc * np.conj(phim)) * 2 * np.pi * radii[p] / Q
            assert abs(U[off[p] + mi] - val) < 1e-13


def test_farfield_vs_quadrature():
    """a_L(theta) = (e^{i pi/4} / sqrt(8 k pi)) int_Gamma e^{-i k theta_hat.y} rho(y) dGamma
    for rho = Phi^p_m (sec. 4.4 definition)."""
    centers = np.array([[0.3, -0.2], [2.5, 1.0]])
    radii = np.array([0.5, 1.2])
    n_modes = np.array([5, 9])
    k = 4.2
    thetas = np.array([0.0, 0.4, 2.0, 4.4])
    G = farfield.farfield_rows(centers, radii, n_modes, k, thetas)
    off, _ = geometry.mode_offsets(n_modes)
    Q = 128
    for p in range(2):
        x, y, t = _circle(centers[p], radii[p], Q)
        for j, th in enumerate(thetas):
            ker = np.exp(-1j * k * (np.cos(th) * x + np.sin(th) * y))
            for mi, m in enumerate(range(-n_modes[p], n_modes[p] + 1)):
                phim = np.exp(1j * m * t) / np.sqrt(2 * np.pi * radii[p])
                val = (np.exp(0.25j * np.pi) / np.sqrt(8 * k * np.pi)
                       * np.sum(ker * phim) * 2 * np.pi * radii[p] / Q)
                assert abs(G[j, off[p] + mi] - val) < 1e-13


# ------------------------------------------------------------- closed forms
def _mie_farfield(center, a, k, beta, thetas, N):
    """Textbook sound-soft cylinder: u_s = -sum_m i^m (J_m(ka)/H_m(ka)) H_m(kr) e^{im(phi-beta)}
    about the cylinder center, times the incident phase e^{ik beta_hat.O};
    H_m(kr) ~ sqrt(2/(pi k r)) e^{i(kr - m pi/2 - pi/4)} and the shift of origin
    gives e^{-ik theta_hat.O}."""
    m = np.arange(-N, N + 1)
    ratio = sp.jv(m, k * a) / sp.hankel1(m, k * a)
    O = np.asarray(center)
    ph = np.exp(1j * k * ((np.cos(beta) - np.cos(thetas)) * O[0] + (np.sin(beta) - np.sin(thetas)) * O[1]))
    s = np.sum(ratio[None, :] * np.exp(1j * m[None, :] * (thetas[:, None] - beta)), axis=1)
    return -np.exp(-0.25j * np.pi) * np.sqrt(2.0 / (np.pi * k)) * ph * s


@pytest.mark.parametrize("center,a,k,N", [((0.0, 0.0), 1.0, 2 * math.pi, 15),
                                          ((1.3, -0.7), 0.45, 9.0, 12),
                                          ((-2.0, 3.0), 2.0, 1.5, 10)])
def test_single_disk_mie(center, a, k, N):
    centers = np.array([center])
    radii = np.array([a])
    n_modes = np.array([N])
    beta = 0.6
    thetas = synth.uniform_angles(90)
    L = operator.efie_matrix(centers, radii, n_modes, k)
    U = rhs.planewave(centers, radii, n_modes, k, [beta])
    rho = solve.efie_solve_lu(L, U)[0]
    af = farfield.farfield(centers, radii, n_modes, k, thetas, rho)
    ref = _mie_farfield(center, a, k, beta, thetas, N)
    assert rel(af, ref) < 1e-13


# ------------------------------------------------- boundary condition residual
def test_boundary_condition_residual(tiny):
    """u_inc + sum_q (single-layer potential of rho_q) vanishes on every Gamma_p.
    The potentials of the other disks are integrated directly (trapezoid rule
    on Gamma_q of (i/4) H_0(k|x-y|) rho_q(y)); the self term is the exact
    on-boundary value of the potential of a Fourier mode.  This pins the
    off-diagonal blocks (separation direction, transpose) independently of
    the addition theorem: the residual is truncation-limited and shrinks with N."""
    res = []
    for N in (10, 15):
        cl = tiny
        n_modes = np.full(4, N)
        L = operator.efie_matrix(cl.centers, cl.radii, n_modes, cl.k)
        U = rhs.planewave(cl.centers, cl.radii, n_modes, cl.k, [0.0])
        rho = solve.efie_solve_lu(L, U)[0]
        off, _ = geometry.mode_offsets(n_modes)
        Q = 128
        worst = 0.0
        m = np.arange(-N, N + 1)
        for p in range(4):
            x, y, t = _circle(cl.centers[p], cl.radii[p], 64)
            tot = np.exp(1j * cl.k * x)
            # self term: (i pi a/2) J_m H_m e^{im t} / sqrt(2 pi a)
            rp = rho[off[p]:off[p + 1]]
            coef = 0.5j * np.pi * cl.radii[p] * sp.jv(m, cl.k * cl.radii[p]) * sp.hankel1(m, cl.k * cl.radii[p])
            tot = tot + np.exp(1j * np.outer(t, m)) @ (coef * rp) / np.sqrt(2 * np.pi * cl.radii[p])
            for q in range(4):
                if q == p:
                    continue
                xq, yq, tq = _circle(cl.centers[q], cl.radii[q], Q)
                rq = np.exp(1j * np.outer(tq, m)) @ rho[off[q]:off[q + 1]] / np.sqrt(2 * np.pi * cl.radii[q])
                G = 0.25j * sp.hankel1(0, cl.k * np.hypot(x[:, None] - xq[None, :], y[:, None] - yq[None, :]))
                tot = tot + G @ rq * (2 * np.pi * cl.radii[q] / Q)
            worst = max(worst, float(np.max(np.abs(tot))))
        res.append(worst)
    assert res[1] < 1e-4 and res[1] < res[0] / 10, res


# --------------------------------------------------- exact identities of the system
def test_transpose_identity():
    """L^T = P L P with P the mode flip m -> -m in every block."""
    cl = synth.small_random(11, 7, 0.3, 0.9, 8.0, 0.2, 4.0, 3)
    L = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    P = operator.mode_flip(cl.n_modes)
    assert rel(L[np.ix_(P, P)], L.T) < 1e-14


def _solve_far(cl, betas, thetas):
    L = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    U = rhs.planewave(cl.centers, cl.radii, cl.n_modes, cl.k, betas)
    rho = solve.efie_solve_lu(L, U)
    return farfield.farfield(cl.centers, cl.radii, cl.n_modes, cl.k, thetas, rho)


def test_reciprocity():
    """a(theta; beta) = a(beta + pi; theta + pi) for the truncated system."""
    cl = synth.small_random(12, 6, 0.3, 0.8, 6.0, 0.2, 5.0, 4)
    phi = np.array([0.1, 1.3, 2.9, 4.0, 5.5])
    Fa = _solve_far(cl, phi, phi)                   # Fa[j, i] = a(phi_i; phi_j)
    Fb = _solve_far(cl, phi + np.pi, phi + np.pi)   # Fb[j, i] = a(phi_i + pi; phi_j + pi)
    assert rel(Fa, Fb.T) < 1e-12


def test_optical_theorem():
    """int_0^{2pi} |a(theta; beta)|^2 dtheta = -sqrt(8 pi / k) Re(e^{i pi/4} a(beta; beta))."""
    cl = synth.small_random(13, 8, 0.2, 0.9, 7.0, 0.2, 3.7, 5)
    beta = 0.9
    rmax = np.max(np.hypot(cl.centers[:, 0], cl.centers[:, 1]))
    nt = int(2 * (cl.k * rmax + np.max(cl.n_modes)) + 64)
    th = synth.uniform_angles(nt)
    a = _solve_far(cl, [beta], th)[0]
    lhs = np.sum(np.abs(a) ** 2) * 2 * np.pi / nt
    a0 = _solve_far(cl, [beta], [beta])[0, 0]
    rhs_ = -np.sqrt(8 * np.pi / cl.k) * np.real(np.exp(0.25j * np.pi) * a0)
    assert abs(lhs - rhs_) < 1e-12 * abs(rhs_)


def test_tiny_reflection_symmetry(tiny):
    """The 4-disk square is symmetric under y -> 3 - y; with beta = 0 this gives
    a(theta) = e^{-3ik sin(theta)} a(-theta)."""
    th = synth.uniform_angles(360)
    a = _solve_far(tiny, [0.0], th)[0]
    am = _solve_far(tiny, [0.0], -th)[0]
    assert rel(a, np.exp(-3j * tiny.k * np.sin(th)) * am) < 1e-13


def test_spectral_convergence(tiny):
    th = synth.uniform_angles(90)
    ref = None
    errs = []
    for N in (30, 8, 10, 12, 15, 18):
        tiny_N = synth.Cluster(tiny.centers, tiny.radii, np.full(4, N), tiny.k)
        a = _solve_far(tiny_N, [0.0], th)[0]
        if ref is None:
            ref = a
            continue
        errs.append(rel(a, ref))
    assert all(errs[i + 1] < errs[i] / 5 for i in range(len(errs) - 1)), errs
    assert errs[3] < 1e-8 and errs[-1] < 1e-11, errs


def test_preconditioner_and_gmres_vs_lu(tiny):
    """The single-scattering preconditioned system has the LU solution; GMRES at
    tol 1e-12 reaches it (brute force)."""
    cl = tiny
    L = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    D = operator.efie_diagonal(cl.radii, cl.n_modes, cl.k)
    A = operator.preconditioned(L, D)
    U = rhs.planewave(cl.centers, cl.radii, cl.n_modes, cl.k, [0.0])[0]
    f = -U / D
    x_lu = solve.efie_solve_lu(L, U[None])[0]
    assert rel(np.linalg.solve(A, f), x_lu) < 1e-13
    x, flag, relres, it, resvec = solve.gmres(lambda v: A @ v, f, 30, 1e-12, 2000)
    assert flag == 0 and relres <= 1e-12 and it > 5
    assert rel(x, x_lu) < 1e-10
    assert resvec[0] == 1.0 and len(resvec) == it + 1
    # maxit forces FLAG 1
    _, flag1, _, it1, _ = solve.gmres(lambda v: A @ v, f, 30, 1e-12, 3)
    assert flag1 == 1 and it1 == 3


def test_preconditioned_k_form():
    """A = D^{-1} L has identity diagonal blocks and off-diagonal entries
    sqrt(a_q/a_p) t_{n-m} J_n(k a_q) / H_m(k a_p) (J_m(k a_p) cancels)."""
    cl = synth.small_random(14, 4, 0.3, 0.8, 5.0, 0.3, 3.0, 3)
    L = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    A = operator.preconditioned(L, operator.efie_diagonal(cl.radii, cl.n_modes, cl.k))
    off, _ = geometry.mode_offsets(cl.n_modes)
    b, al = geometry.pair_geometry(cl.centers)
    p, q = 2, 0
    for mi, m in enumerate(range(-cl.n_modes[p], cl.n_modes[p] + 1)):
        for ni, n in enumerate(range(-cl.n_modes[q], cl.n_modes[q] + 1)):
            ref = (np.sqrt(cl.radii[q] / cl.radii[p]) * sp.hankel1(n - m, cl.k * b[p, q])
                   * np.exp(1j * (n - m) * al[p, q]) * sp.jv(n, cl.k * cl.radii[q])
                   / sp.hankel1(m, cl.k * cl.radii[p]))
            assert abs(A[off[p] + mi, off[q] + ni] - ref) < 1e-13 * max(1, abs(ref))
    blk = A[off[p]:off[p + 1], off[p]:off[p + 1]]
    assert np.allclose(blk, np.eye(blk.shape[0]), atol=1e-15)


def test_adjoint_via_forward_solve():
    """lambda = P solve(L, P c) equals solve(L^T, c)."""
    cl = synth.small_random(15, 6, 0.3, 0.8, 6.0, 0.2, 4.5, 3)
    L = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    P = operator.mode_flip(cl.n_modes)
    rng = np.random.default_rng(0)
    c = rng.normal(size=L.shape[0]) + 1j * rng.normal(size=L.shape[0])
    lam = np.linalg.solve(L.T, c)
    lam2 = np.linalg.solve(L, c[P])[P]
    assert rel(lam2, lam) < 1e-13


# ---------------------------------------------------------------- gradient
def _grad_case(seed=16):
    base = synth.small_random(seed, 4, 0.4, 0.7, 5.0, 0.3, 3.0, 4, R=3, n_theta=5)
    rng = np.random.default_rng(seed + 100)
    tgt = synth.perturb(rng, base)
    target = gradient.forward(tgt.centers, tgt.radii, tgt.n_modes, tgt.k, base.betas, base.thetas)
    return base, target


def test_gradient_vs_central_differences():
    base, target = _grad_case()
    args = (base.centers, base.radii, base.n_modes, base.k, base.betas, base.thetas, target)
    loss, dc, da, dk = gradient.misfit_grad(*args)
    assert abs(loss - gradient.misfit(*args)) < 1e-12 * loss
    fc, fa, fk = gradient.misfit_fd(*args, h=1e-5)
    g = np.concatenate([dc.ravel(), da, [dk]])
    f = np.concatenate([fc.ravel(), fa, [fk]])
    assert rel(g, f) < 1e-6
    assert np.all(np.abs(g - f) <= 1e-6 * np.max(np.abs(f)) + 1e-6 * np.abs(f))


def test_gradient_translation_and_scaling():
    """Exact invariances of the truncated far field: translating every center by d
    multiplies a(theta; beta) by e^{ik(beta_hat - theta_hat).d}; scaling lengths by s
    and k by 1/s multiplies it by sqrt(s).  For the misfit this gives
      sum_p dl/dx_p = 2 Re sum conj(e) ik(cos beta - cos theta) a   (same for y, sin),
      sum_p (O_p . grad_p l + a_p dl/da_p) - k dl/dk = Re sum conj(e) a."""
    base, target = _grad_case(17)
    args = (base.centers, base.radii, base.n_modes, base.k, base.betas, base.thetas, target)
    loss, dc, da, dk = gradient.misfit_grad(*args)
    a = gradient.forward(*args[:-1])
    e = a - target
    cb, ct = np.cos(base.betas)[:, None], np.cos(base.thetas)[None, :]
    sb, st = np.sin(base.betas)[:, None], np.sin(base.thetas)[None, :]
    tx = 2 * np.real(np.sum(np.conj(e) * 1j * base.k * (cb - ct) * a))
    ty = 2 * np.real(np.sum(np.conj(e) * 1j * base.k * (sb - st) * a))
    scale = np.real(np.sum(np.conj(e) * a))
    assert abs(np.sum(dc[:, 0]) - tx) < 1e-10 * (abs(tx) + np.max(np.abs(dc)))
    assert abs(np.sum(dc[:, 1]) - ty) < 1e-10 * (abs(ty) + np.max(np.abs(dc)))
    lhs = np.sum(base.centers * dc) + np.sum(base.radii * da) - base.k * dk
    assert abs(lhs - scale) < 1e-10 * (abs(scale) + np.max(np.abs(dc)))


# ------------------------------------------- time reversal (sec. 7, Example III)
def test_dort_single_disk_spectrum():
    """One disk: F = D C D with D a unitary diagonal (the translation phases)
    and C circulant in alpha_i - alpha_j, whose eigenvalues are N_alpha times
    the Mie far-field coefficients -e^{-i pi/4} sqrt(2/(pi k)) J_m(ka)/H_m(ka)
    (times (-1)^m from the receiver shift by pi).  So T = conj(F)^T F has the
    2N+1 eigenvalues N_alpha^2 |c_m|^2 and is zero otherwise."""
    from oracle import dort
    center, a, k, N, n_alpha = (0.8, -0.3), 0.7, 5.0, 6, 32
    F = dort.farfield_matrix(np.array([center]), np.array([a]), np.array([N]), k, n_alpha)
    w, V = dort.eig_desc(dort.time_reversal(F))
    m = np.arange(-N, N + 1)
    c = -np.exp(-0.25j * np.pi) * np.sqrt(2.0 / (np.pi * k)) * sp.jv(m, k * a) / sp.hankel1(m, k * a)
    ref = np.sort(n_alpha ** 2 * np.abs(c) ** 2)[::-1]
    np.testing.assert_allclose(w[:2 * N + 1], ref, rtol=1e-11)
    assert np.max(np.abs(w[2 * N + 1:])) < 1e-12 * w[0]
    # unit eigenvectors
    np.testing.assert_allclose(np.linalg.norm(V, axis=0), 1.0, rtol=1e-12)


def test_dort_farfield_matrix_is_symmetric():
    """With receivers at alpha_i + pi, reciprocity a(theta; beta) =
    a(beta + pi; theta + pi) makes F complex symmetric (F = F^T) for any
    configuration; receivers at alpha_i would not."""
    from oracle import dort
    cl = synth.small_random(21, 5, 0.3, 0.8, 6.0, 0.3, 4.0, 4)
    F = dort.farfield_matrix(cl.centers, cl.radii, cl.n_modes, cl.k, 24)
    assert rel(F, F.T) < 1e-12
    al = dort.mirror_angles(24)
    from oracle import gradient
    F_same = gradient.forward(cl.centers, cl.radii, cl.n_modes, cl.k, al, al).T
    assert rel(F_same, F_same.T) > 1e-3


def test_dort_time_reversal_is_hermitian_psd():
    from oracle import dort
    cl = synth.small_random(22, 4, 0.3, 0.8, 6.0, 0.3, 4.0, 3)
    F = dort.farfield_matrix(cl.centers, cl.radii, cl.n_modes, cl.k, 20)
    T = dort.time_reversal(F)
    assert rel(T, T.conj().T) < 1e-15
    w, V = dort.eig_desc(T)
    assert w[-1] > -1e-12 * w[0]
    assert np.all(np.diff(w) <= 0)
    assert rel(V @ np.diag(w) @ V.conj().T, T) < 1e-12
    # the nonzero spectrum of T is that of F F^H (brute force: singular values of F)
    s = np.linalg.svd(F, compute_uv=False)
    np.testing.assert_allclose(w[:len(s)], s ** 2, rtol=1e-10, atol=1e-12 * w[0])


@pytest.mark.parametrize("m", [0, 1, -3, 7])
def test_herglotz_jacobi_anger(m):
    """f_j = e^{-i m alpha_j}: u_I(x) -> int_0^{2pi} e^{i k r cos(alpha - phi)} e^{-i m alpha}
    d alpha = 2 pi i^m J_m(k r) e^{-i m phi}; the trapezoid rule is exact to
    rounding once N_alpha exceeds k r + |m| by a margin."""
    from oracle import dort
    k, n_alpha = 2 * math.pi, 128
    rng = np.random.default_rng(5)
    pts = rng.uniform(-4, 4, size=(20, 2))
    f = np.exp(-1j * m * dort.mirror_angles(n_alpha))
    u = dort.herglotz(n_alpha, f, k, pts)
    r, phi = np.hypot(pts[:, 0], pts[:, 1]), np.arctan2(pts[:, 1], pts[:, 0])
    ref = 2 * np.pi * (1j ** m) * sp.jv(m, k * r) * np.exp(-1j * m * phi)
    assert np.max(np.abs(u - ref)) < 1e-12


def test_dort_example_three_significant_eigenvalues_and_focusing():
    """The paper's example: three small scatterers give three significant
    eigenvalues of T, and the Herglotz wave of each of the three eigenvectors
    focuses on one obstacle, from the most to the least reflecting (largest
    to smallest radius).  512 mirror cells resolve the Herglotz waves out to
    |x| ~ N_alpha / (2k) ~ 40, beyond the obstacles at distance 20-22."""
    from oracle import dort
    cl = synth.dort_example(512)
    F = dort.farfield_matrix(cl.centers, cl.radii, cl.n_modes, cl.k, 512)
    w, V = dort.eig_desc(dort.time_reversal(F))
    assert w[2] > 100 * w[3]
    for j in range(3):
        u = np.abs(dort.herglotz(512, V[:, j], cl.k, cl.centers))
        assert np.argmax(u) == j
        assert u[j] > 2 * np.max(np.delete(u, j))


# ------------------------------- operators M, N, D and the other formulations
def _green_derivs(k, x, y, nx, ny):
    """G = (i/4) H_0(k r) and its normal derivatives for x on one circle, y on
    another: d_{n_y} G, d_{n_x} G, d_{n_x} d_{n_y} G (d = x - y, r = |d|)."""
    dx = x[0][:, None] - y[0][None, :]
    dy = x[1][:, None] - y[1][None, :]
    r = np.hypot(dx, dy)
    H0, H1 = sp.hankel1(0, k * r), sp.hankel1(1, k * r)
    dny = dx * ny[0][None, :] + dy * ny[1][None, :]          # d . n_y
    dnx = dx * nx[0][:, None] + dy * nx[1][:, None]          # d . n_x
    nn = nx[0][:, None] * ny[0][None, :] + nx[1][:, None] * ny[1][None, :]
    dG_ny = 0.25j * k * H1 / r * dny
    dG_nx = -0.25j * k * H1 / r * dnx
    ddG = 0.25j * k * (dny * dnx / r * (k * H0 / r - 2.0 * H1 / r ** 2) + H1 / r * nn)
    return dG_ny, dG_nx, ddG


def test_mnd_offdiag_blocks_vs_quadrature():
    """X^{pq}_{mn} = <X Phi^q_n, Phi^p_m> with the kernels of sec. 3:
    M: -d_{n_y} G, N: d_{n_x} G, D: -d_{n_x} d_{n_y} G, by the trapezoid rule on
    both circles (smooth periodic integrand for disjoint disks)."""
    from oracle import operators as ops
    centers = np.array([[0.3, -0.2], [1.9, 1.1], [-1.4, 1.6]])
    radii = np.array([0.5, 0.7, 0.4])
    n_modes = np.array([4, 6, 3])
    k = 3.1
    mats = {n: ops.operator_matrix(n, centers, radii, n_modes, k) for n in "MND"}
    off, _ = geometry.mode_offsets(n_modes)
    Q = 96
    for p, q in [(0, 1), (1, 0), (2, 1), (0, 2)]:
        xp, yp, tp = _circle(centers[p], radii[p], Q)
        xq, yq, tq = _circle(centers[q], radii[q], Q)
        dG_ny, dG_nx, ddG = _green_derivs(k, (xp, yp), (xq, yq), (np.cos(tp), np.sin(tp)),
                                          (np.cos(tq), np.sin(tq)))
        kern = {"M": -dG_ny, "N": dG_nx, "D": -ddG}
        w = (2.0 * np.pi * radii[q] / Q) * (2.0 * np.pi * radii[p] / Q)
        for mi, m in enumerate(range(-n_modes[p], n_modes[p] + 1)):
            phim = np.exp(1j * m * tp) / np.sqrt(2 * np.pi * radii[p])
            for ni, n in enumerate(range(-n_modes[q], n_modes[q] + 1)):
                phin = np.exp(1j * n * tq) / np.sqrt(2 * np.pi * radii[q])
                for name, K in kern.items():
                    val = np.sum(np.conj(phim)[:, None] * K * phin[None, :]) * w
                    got = mats[name][off[p] + mi, off[q] + ni]
                    assert abs(got - val) <= 1e-10 * max(1.0, abs(val)), (name, p, q, m, n, got, val)


def test_planewave_dn_vs_quadrature():
    """dU^p_m = <d_n u_inc, Phi^p_m> on Gamma_p (Prop. 4 from its definition)."""
    from oracle import operators as ops
    centers = np.array([[0.3, -0.2], [2.5, 1.0]])
    radii = np.array([0.5, 1.2])
    n_modes = np.array([5, 9])
    k, beta = 4.2, 0.77
    dU = ops.planewave_dn(centers, radii, n_modes, k, [beta])[0]
    off, _ = geometry.mode_offsets(n_modes)
    Q = 128
    for p in range(2):
        x, y, t = _circle(centers[p], radii[p], Q)
        dn = 1j * k * (np.cos(beta) * np.cos(t) + np.sin(beta) * np.sin(t)) * np.exp(
            1j * k * (np.cos(beta) * x + np.sin(beta) * y))
        for mi, m in enumerate(range(-n_modes[p], n_modes[p] + 1)):
            phim = np.exp(1j * m * t) / np.sqrt(2 * np.pi * radii[p])
            val = np.sum(dn * np.conj(phim)) * 2 * np.pi * radii[p] / Q
            assert abs(dU[off[p] + mi] - val) < 1e-12


def test_double_layer_farfield_is_the_potentials_limit():
    """a_M(theta) = lim r^{1/2} e^{-ikr} (M Phi)(r theta_hat) for the volume
    double-layer potential M lambda(x) = -int d_{n_y} G(x, y) lambda(y) dGamma,
    integrated by the trapezoid rule at r = 1e6 (error O(1/r))."""
    from oracle import operators as ops
    centers = np.array([[0.6, -0.3], [-1.0, 0.8]])
    radii = np.array([0.45, 0.7])
    n_modes = np.array([4, 5])
    k = 3.3
    th = np.array([0.2, 1.7, 3.9])
    A = ops.farfield_rows_dl(centers, radii, n_modes, k, th)
    off, _ = geometry.mode_offsets(n_modes)
    R, Q = 1e6, 256
    for j, t in enumerate(th):
        x = (np.array([R * np.cos(t)]), np.array([R * np.sin(t)]))
        for p in range(2):
            xq, yq, tq = _circle(centers[p], radii[p], Q)
            dG_ny, _, _ = _green_derivs(k, x, (xq, yq), (np.array([0.0]), np.array([0.0])),
                                        (np.cos(tq), np.sin(tq)))
            for mi, m in enumerate(range(-n_modes[p], n_modes[p] + 1)):
                phin = np.exp(1j * m * tq) / np.sqrt(2 * np.pi * radii[p])
                pot = -np.sum(dG_ny[0] * phin) * 2 * np.pi * radii[p] / Q
                lim = pot * np.sqrt(R) * np.exp(-1j * k * R)
                assert abs(lim - A[j, off[p] + mi]) < 1e-4 * max(abs(A[j, off[p] + mi]), 1e-3)


def _mie_general(center, a, k, beta, thetas, N, hard):
    m = np.arange(-N, N + 1)
    ratio = (sp.jvp(m, k * a) / sp.h1vp(m, k * a)) if hard else (sp.jv(m, k * a) / sp.hankel1(m, k * a))
    O = np.asarray(center)
    ph = np.exp(1j * k * ((np.cos(beta) - np.cos(thetas)) * O[0] + (np.sin(beta) - np.sin(thetas)) * O[1]))
    s = np.sum(ratio[None, :] * np.exp(1j * m[None, :] * (thetas[:, None] - beta)), axis=1)
    return -np.exp(-0.25j * np.pi) * np.sqrt(2.0 / (np.pi * k)) * ph * s


FORMS = [("efie", {}, False), ("mfie", {}, False), ("cfie", {"alpha": 0.5, "eta": 3j}, False),
         ("bwie", {"eta": 3j}, False), ("neumann_sl", {}, True), ("neumann_dl", {}, True)]


@pytest.mark.parametrize("name,kw,hard", FORMS)
def test_formulations_single_disk_mie(name, kw, hard):
    """Every formulation reproduces the textbook single-disk far field:
    -sqrt(2/(pi k)) e^{-i pi/4} sum_m c_m e^{i m (theta - beta)}, c_m = J_m/H_m
    (sound-soft) or J'_m/H'_m (sound-hard)."""
    from oracle import operators as ops
    c, a, k, N, beta = (0.7, -0.4), 0.9, 4.0, 14, 0.6
    th = synth.uniform_angles(40)
    _, af = ops.solve_farfield(name, np.array([c]), np.array([a]), np.array([N]), k, [beta], th, **kw)
    ref = _mie_general(c, a, k, beta, th, N, hard)
    assert rel(af[0], ref) < 1e-13


def test_formulations_agree_on_a_cluster():
    """Four disks: EFIE, MFIE, CFIE and BWIE give one sound-soft far field, the
    single- and double-layer equations one sound-hard far field, and the two
    differ."""
    from oracle import operators as ops
    cl = synth.small_random(31, 4, 0.4, 0.8, 6.0, 0.4, 3.0, 12)
    th = synth.uniform_angles(48)
    far = {}
    for name, kw, _ in FORMS:
        kw = {k: (v * cl.k / 3.0 if k == "eta" else v) for k, v in kw.items()}
        far[name] = ops.solve_farfield(name, cl.centers, cl.radii, cl.n_modes, cl.k, [0.3], th, **kw)[1][0]
    for name in ("mfie", "cfie", "bwie"):
        assert rel(far[name], far["efie"]) < 1e-12, name
    assert rel(far["neumann_dl"], far["neumann_sl"]) < 1e-12
    assert rel(far["neumann_sl"], far["efie"]) > 1e-2


# -------------------------------------------------------------------- near field
def test_layer_potentials_vs_quadrature():
    """L rho(x) = int_Gamma G(x, y) rho(y) dGamma and M lam(x) = -int d_{n_y} G lam
    by the trapezoid rule, at points at least half a radius from every circle."""
    from oracle import nearfield
    centers = np.array([[0.3, -0.2], [2.4, 1.1], [-1.5, 1.7]])
    radii = np.array([0.5, 0.7, 0.4])
    n_modes = np.array([6, 8, 5])
    k = 2.7
    rng = np.random.default_rng(3)
    n = int(np.sum(2 * n_modes + 1))
    dens = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    pts = np.array([[1.4, -1.3], [0.9, 0.9], [-1.9, 0.2], [3.6, 2.6], [0.2, 2.9]])
    uL = nearfield.potential(centers, radii, n_modes, k, dens, pts, 1.0, 0.0)
    uM = nearfield.potential(centers, radii, n_modes, k, dens, pts, 0.0, 1.0)
    off, _ = geometry.mode_offsets(n_modes)
    Q = 256
    refL = np.zeros(len(pts), complex)
    refM = np.zeros(len(pts), complex)
    for p in range(3):
        xq, yq, tq = _circle(centers[p], radii[p], Q)
        m = np.arange(-n_modes[p], n_modes[p] + 1)
        rho = np.exp(1j * np.outer(tq, m)) @ dens[off[p]:off[p + 1]] / np.sqrt(2 * np.pi * radii[p])
        w = 2 * np.pi * radii[p] / Q
        G = 0.25j * sp.hankel1(0, k * np.hypot(pts[:, 0:1] - xq[None, :], pts[:, 1:2] - yq[None, :]))
        refL += G @ rho * w
        dG_ny, _, _ = _green_derivs(k, (pts[:, 0], pts[:, 1]), (xq, yq),
                                    (np.zeros(len(pts)), np.zeros(len(pts))), (np.cos(tq), np.sin(tq)))
        refM += -(dG_ny @ rho) * w
    assert rel(uL, refL) < 1e-12
    assert rel(uM, refM) < 1e-12


def test_total_field_single_disk_mie():
    """Sound-soft disk at O: u_t = sum_m i^m [J_m(k r) - J_m(k a) H_m(k r) / H_m(k a)]
    e^{i m (theta - beta)} e^{i k beta_hat . O} (polar coordinates about O)."""
    from oracle import nearfield
    O, a, k, N, beta = np.array([0.4, -0.3]), 0.8, 3.5, 16, 0.9
    L = operator.efie_matrix(O[None, :], [a], [N], k)
    U = rhs.planewave(O[None, :], [a], [N], k, [beta])
    rho = solve.efie_solve_lu(L, U)[0]
    rng = np.random.default_rng(4)
    rr = rng.uniform(1.05 * a, 4.0, 30)
    tt = rng.uniform(0, 2 * np.pi, 30)
    pts = np.stack([O[0] + rr * np.cos(tt), O[1] + rr * np.sin(tt)], 1)
    ut = nearfield.total_field(O[None, :], [a], [N], k, rho[None, :], pts, [beta])[0]
    m = np.arange(-40, 41)
    ref = np.exp(1j * k * (np.cos(beta) * O[0] + np.sin(beta) * O[1])) * np.sum(
        (1j ** m)[None, :] * (sp.jv(m[None, :], k * rr[:, None])
                              - sp.jv(m, k * a)[None, :] * sp.hankel1(m[None, :], k * rr[:, None])
                              / sp.hankel1(m, k * a)[None, :])
        * np.exp(1j * m[None, :] * (tt[:, None] - beta)), axis=1)
    # the truncation at N = 16 leaves ~1e-12 at these radii (k a = 2.8)
    assert np.max(np.abs(ut - ref)) < 1e-10


def test_total_field_vanishes_on_the_boundaries(tiny):
    """Four disks: u_t on every circle shrinks with N (truncation-limited)."""
    from oracle import nearfield
    worst = []
    for N in (10, 16):
        cl = tiny
        n_modes = np.full(4, N)
        L = operator.efie_matrix(cl.centers, cl.radii, n_modes, cl.k)
        U = rhs.planewave(cl.centers, cl.radii, n_modes, cl.k, [0.0])
        rho = solve.efie_solve_lu(L, U)[0]
        pts = np.concatenate([np.stack(_circle(cl.centers[p], cl.radii[p] * (1 + 1e-12), 48)[:2], 1)
                              for p in range(4)])
        ut = nearfield.total_field(cl.centers, cl.radii, n_modes, cl.k, rho[None, :], pts, [0.0])[0]
        worst.append(np.max(np.abs(ut)))
    assert worst[1] < 1e-5 and worst[1] < worst[0] / 10, worst


def test_near_field_tends_to_the_far_field():
    """sqrt(r) e^{-i k r} u(r theta_hat) -> a(theta) (sec. 4.4), single and double layer."""
    from oracle import nearfield, operators as ops
    cl = synth.small_random(61, 3, 0.3, 0.7, 4.0, 0.3, 3.0, 5)
    rng = np.random.default_rng(6)
    dens = rng.standard_normal(cl.n_tot) + 1j * rng.standard_normal(cl.n_tot)
    th = np.array([0.3, 2.0, 4.4])
    R = 1e7
    pts = np.stack([R * np.cos(th), R * np.sin(th)], 1)
    for fL, fM in ((1.0, 0.0), (0.0, 1.0)):
        u = nearfield.potential(cl.centers, cl.radii, cl.n_modes, cl.k, dens, pts, fL, fM)
        lim = u * np.sqrt(R) * np.exp(-1j * cl.k * R)
        G = fL * farfield.farfield_rows(cl.centers, cl.radii, cl.n_modes, cl.k, th) + \
            fM * ops.farfield_rows_dl(cl.centers, cl.radii, cl.n_modes, cl.k, th)
        assert rel(lim, G @ dens) < 1e-5


# -------------------------------------------------------------- penetrable disks
def _transmission_mie(center, a, k, ki, mu, beta, thetas, N):
    """Penetrable disk: matching J_m(k a) + c_m H_m(k a) = b_m J_m(ki a) and
    k (J'_m(k a) + c_m H'_m(k a)) = mu ki b_m J'_m(ki a) per mode gives
    c_m = (mu ki J'_m(ki a) J_m(k a) - k J_m(ki a) J'_m(k a))
          / (k J_m(ki a) H'_m(k a) - mu ki J'_m(ki a) H_m(k a)),
    far field sqrt(2/(pi k)) e^{-i pi/4} sum_m c_m e^{i m (theta - beta)}."""
    m = np.arange(-N, N + 1)
    Ji, Jid = sp.jv(m, ki * a), sp.jvp(m, ki * a)
    J, Jd, H, Hd = sp.jv(m, k * a), sp.jvp(m, k * a), sp.hankel1(m, k * a), sp.h1vp(m, k * a)
    c = (mu * ki * Jid * J - k * Ji * Jd) / (k * Ji * Hd - mu * ki * Jid * H)
    O = np.asarray(center)
    ph = np.exp(1j * k * ((np.cos(beta) - np.cos(thetas)) * O[0] + (np.sin(beta) - np.sin(thetas)) * O[1]))
    return np.exp(-0.25j * np.pi) * np.sqrt(2.0 / (np.pi * k)) * ph * np.sum(
        c[None, :] * np.exp(1j * m[None, :] * (thetas[:, None] - beta)), axis=1)


@pytest.mark.parametrize("ki,mu", [(2.0 * 4.0, 1.0), (0.6 * 4.0, 1.0), (1.5 * 4.0, 2.5)])
def test_penetrable_single_disk_mie(ki, mu):
    from oracle import penetrable as pen
    c, a, k, N, beta = (0.4, -0.6), 0.8, 4.0, 18, 0.7
    th = synth.uniform_angles(36)
    rp, _ = pen.solve(np.array([c]), np.array([a]), np.array([N]), k, [ki], [beta], mu=[mu])
    af = pen.farfield(np.array([c]), np.array([a]), np.array([N]), k, rp, th)[0]
    assert rel(af, _transmission_mie(c, a, k, ki, mu, beta, th, N)) < 1e-12


def test_penetrable_matched_medium_does_not_scatter():
    """k- = k+ and mu = 1: no scattered field (the truncated system reproduces it exactly)."""
    from oracle import penetrable as pen
    cl = synth.small_random(81, 4, 0.3, 0.8, 6.0, 0.3, 3.0, 6)
    rp, rm = pen.solve(cl.centers, cl.radii, cl.n_modes, cl.k, np.full(4, cl.k), [0.5])
    a = pen.farfield(cl.centers, cl.radii, cl.n_modes, cl.k, rp, synth.uniform_angles(24))
    assert np.max(np.abs(a)) < 1e-12
    assert np.max(np.abs(rp)) < 1e-12 * np.max(np.abs(rm))


def test_penetrable_transmission_conditions_on_the_boundaries():
    """Three disks with different interior wavenumbers and mu: on every circle
    the exterior total field equals the interior field, and its radial
    derivative equals mu times the interior one (second-order one-sided
    differences on each side), to a truncation-limited level that shrinks
    with N."""
    from oracle import nearfield, penetrable as pen
    centers = np.array([[0.0, 0.0], [2.2, 0.4], [0.6, 2.1]])
    radii = np.array([0.6, 0.5, 0.45])
    k, beta = 3.0, 0.3
    ki, mu = np.array([5.0, 2.0, 4.0]), np.array([1.0, 1.5, 0.8])
    t = np.linspace(0, 2 * np.pi, 40, endpoint=False)
    dirs = np.stack([np.cos(t), np.sin(t)], 1)
    h = 2e-4
    worst = []
    for N in (8, 14):
        n_modes = np.full(3, N)
        rp, rm = pen.solve(centers, radii, n_modes, k, ki, [beta], mu=mu)
        err = 0.0
        for p in range(3):
            a = radii[p]
            out = [nearfield.total_field(centers, radii, n_modes, k, rp, centers[p] + (a * (1 + 1e-13) + j * h) * dirs,
                                         [beta])[0] for j in range(3)]
            inn = [pen.interior_field(centers, radii, n_modes, ki, rm[0], p, centers[p] + (a * (1 - 1e-13) - j * h) * dirs)
                   for j in range(3)]
            du_o = (-3 * out[0] + 4 * out[1] - out[2]) / (2 * h)
            du_i = (3 * inn[0] - 4 * inn[1] + inn[2]) / (2 * h)
            err = max(err, np.max(np.abs(out[0] - inn[0])), np.max(np.abs(du_o - mu[p] * du_i)) / k)
        worst.append(err)
    assert worst[1] < 1e-5 and worst[1] < worst[0] / 10, worst


def test_penetrable_optical_theorem():
    """Real k- and mu: no energy is absorbed inside, and the truncated system
    keeps int |a|^2 = -sqrt(8 pi / k) Re(e^{i pi/4} a(beta; beta)) exactly.  A
    phase error in an interior block (a lost i, a conjugated Hankel function)
    breaks it; a real rescaling of mu does not (the matched-medium and Mie pins
    cover those)."""
    from oracle import penetrable as pen
    cl = synth.small_random(13, 8, 0.2, 0.9, 7.0, 0.2, 3.7, 5)
    ki = np.linspace(0.6, 2.2, 8) * cl.k
    mu = np.linspace(0.7, 2.0, 8)
    beta, nt = 0.9, 512
    th = synth.uniform_angles(nt)
    rp, _ = pen.solve(cl.centers, cl.radii, cl.n_modes, cl.k, ki, [beta], mu=mu)
    a = pen.farfield(cl.centers, cl.radii, cl.n_modes, cl.k, rp, th)[0]
    a0 = pen.farfield(cl.centers, cl.radii, cl.n_modes, cl.k, rp, [beta])[0, 0]
    lhs = np.sum(np.abs(a) ** 2) * 2 * np.pi / nt
    rhs_ = -np.sqrt(8 * np.pi / cl.k) * np.real(np.exp(0.25j * np.pi) * a0)
    assert abs(lhs - rhs_) < 1e-12 * abs(rhs_)


# -------------------------------------------------------------- point source
def _circle_coefficients(fun, O, a, N, nq=512):
    """<f, Phi_m> = int_0^{2 pi} f(O + a e^{it}) e^{-imt} a dt / sqrt(2 pi a) by the
    trapezoid rule (spectrally accurate for a smooth periodic integrand)."""
    t = 2 * np.pi * np.arange(nq) / nq
    x = np.asarray(O)[None, :] + a * np.stack([np.cos(t), np.sin(t)], 1)
    f = fun(x, t)
    m = np.arange(-N, N + 1)
    return (f[None, :] * np.exp(-1j * m[:, None] * t[None, :])).sum(1) * (2 * np.pi / nq) * a / np.sqrt(2 * np.pi * a)


def test_point_source_coefficients_by_quadrature():
    """Prop. 5 against quadrature of G(x, s) = (i/4) H_0(k|x - s|) and of its
    normal derivative -(i/4) k H_1(k|x - s|) (x - s).n / |x - s| over each circle."""
    from oracle import pointsource as ps
    from oracle.geometry import mode_offsets
    cl = synth.small_random(101, 4, 0.3, 0.9, 6.0, 0.3, 3.3, 7)
    src = np.array([[-1.5, 2.0], [7.5, -0.5]])
    U = ps.point_source(cl.centers, cl.radii, cl.n_modes, cl.k, src)
    dU = ps.point_source_dn(cl.centers, cl.radii, cl.n_modes, cl.k, src)
    off, _ = mode_offsets(cl.n_modes)
    for r, s in enumerate(src):
        for p in range(len(cl.radii)):
            O, a, N = cl.centers[p], cl.radii[p], int(cl.n_modes[p])

            def g(x, t):
                return 0.25j * sp.hankel1(0, cl.k * np.hypot(*(x - s).T))

            def dg(x, t):
                d = x - s
                rr = np.hypot(*d.T)
                nrm = np.stack([np.cos(t), np.sin(t)], 1)
                return -0.25j * cl.k * sp.hankel1(1, cl.k * rr) * np.sum(d * nrm, 1) / rr
            assert rel(U[r, off[p]:off[p + 1]], _circle_coefficients(g, O, a, N)) < 1e-12
            assert rel(dU[r, off[p]:off[p + 1]], _circle_coefficients(dg, O, a, N)) < 1e-12


def test_point_source_single_disk_closed_form():
    """Sound-soft disk, source s: u = -(i/4) sum_m J_m(ka)/H_m(ka) H_m(k r_s)
    H_m(k r) e^{i m (theta - theta_s)} outside (Graf's theorem plus u + G = 0 on
    the circle), against the EFIE solve and its near field."""
    from oracle import nearfield, pointsource as ps
    O, a, k, N = np.array([0.3, -0.2]), 0.7, 2.7, 22
    s = np.array([1.9, 1.1])
    U = ps.point_source(O[None, :], [a], [N], k, s[None, :])
    L = operator.efie_matrix(O[None, :], np.array([a]), np.array([N]), k)
    rho = np.linalg.solve(L, -U[0])
    rng = np.random.default_rng(7)
    rr = rng.uniform(1.05 * a, 3.0, 40)
    tt = rng.uniform(0, 2 * np.pi, 40)
    pts = O[None, :] + rr[:, None] * np.stack([np.cos(tt), np.sin(tt)], 1)
    u = nearfield.potential(O[None, :], [a], [N], k, rho, pts)
    rs, ts = np.hypot(*(s - O)), np.arctan2(*(s - O)[::-1])
    m = np.arange(-40, 41)
    ref = -0.25j * np.sum((sp.jv(m, k * a) / sp.hankel1(m, k * a) * sp.hankel1(m, k * rs))[None, :]
                          * sp.hankel1(m[None, :], k * rr[:, None]) * np.exp(1j * m[None, :] * (tt[:, None] - ts)), 1)
    assert rel(u, ref) < 1e-12


def test_point_source_reciprocity():
    """The scattered field is symmetric in source and receiver:
    u^s(x; s) = u^s(s; x), for sound-soft (EFIE) and penetrable disks."""
    from oracle import nearfield, penetrable as pen, pointsource as ps
    cl = synth.small_random(102, 5, 0.3, 0.8, 6.0, 0.3, 3.1, 8)
    s1, s2 = np.array([-1.0, 1.5]), np.array([7.0, 4.0])
    src = np.stack([s1, s2])
    U = ps.point_source(cl.centers, cl.radii, cl.n_modes, cl.k, src)
    L = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    rho = np.linalg.solve(L, -U.T).T
    u12 = nearfield.potential(cl.centers, cl.radii, cl.n_modes, cl.k, rho[0], s2[None, :])[0]
    u21 = nearfield.potential(cl.centers, cl.radii, cl.n_modes, cl.k, rho[1], s1[None, :])[0]
    assert abs(u12 - u21) < 1e-12 * abs(u12)
    ki, mu = np.linspace(0.6, 2.0, 5) * cl.k, np.linspace(0.8, 1.6, 5)
    dU = ps.point_source_dn(cl.centers, cl.radii, cl.n_modes, cl.k, src)
    rp, _ = pen.solve_coefficients(cl.centers, cl.radii, cl.n_modes, cl.k, ki, U, dU, mu)
    v12 = nearfield.potential(cl.centers, cl.radii, cl.n_modes, cl.k, rp[0], s2[None, :])[0]
    v21 = nearfield.potential(cl.centers, cl.radii, cl.n_modes, cl.k, rp[1], s1[None, :])[0]
    assert abs(v12 - v21) < 1e-11 * abs(v12)


def test_mixed_reciprocity_point_source_and_plane_wave():
    """The far field in direction theta of the wave scattered from a point
    source at s equals e^{i pi/4} / sqrt(8 pi k) (the far-field factor of
    G(., s) = (i/4) H_0) times the scattered field at s of the plane wave
    travelling in direction -theta: ties Prop. 5 to Prop. 4, the near field and
    the far field of sec. 4.4 (sound-soft and penetrable)."""
    from oracle import farfield, nearfield, penetrable as pen, pointsource as ps
    cl = synth.small_random(131, 5, 0.3, 0.8, 6.0, 0.3, 3.3, 8)
    src = np.array([[-1.5, 2.0], [8.0, 1.0]])
    th = np.array([0.3, 1.7, 4.0])
    gam = np.exp(0.25j * np.pi) / np.sqrt(8 * np.pi * cl.k)
    L = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    G = farfield.farfield_rows(cl.centers, cl.radii, cl.n_modes, cl.k, th)
    U = ps.point_source(cl.centers, cl.radii, cl.n_modes, cl.k, src)
    a_ps = np.linalg.solve(L, -U.T).T @ G.T                                  # [source, theta]
    Up = rhs.planewave(cl.centers, cl.radii, cl.n_modes, cl.k, th + np.pi)
    rp = np.linalg.solve(L, -Up.T).T
    u_pw = np.stack([nearfield.potential(cl.centers, cl.radii, cl.n_modes, cl.k, rp[j], src)
                     for j in range(len(th))], 1)
    assert rel(a_ps, gam * u_pw) < 1e-12
    ki, mu = np.linspace(0.6, 2.0, 5) * cl.k, np.linspace(0.8, 1.6, 5)
    dU = ps.point_source_dn(cl.centers, cl.radii, cl.n_modes, cl.k, src)
    rps, _ = pen.solve_coefficients(cl.centers, cl.radii, cl.n_modes, cl.k, ki, U, dU, mu)
    rpw, _ = pen.solve(cl.centers, cl.radii, cl.n_modes, cl.k, ki, th + np.pi, mu=mu)
    v_pw = np.stack([nearfield.potential(cl.centers, cl.radii, cl.n_modes, cl.k, rpw[j], src)
                     for j in range(len(th))], 1)
    assert rel(rps @ G.T, gam * v_pw) < 1e-11


def test_point_source_incident_field_by_graf():
    """The incident field (i/4) H_0(k |x - s|) of a point source (Prop. 5)
    against Graf's addition theorem about a center O with |x - O| < |s - O|:
    (i/4) sum_m J_m(k rho) H_m(k r_s) e^{i m (phi - theta_s)}, evaluated at
    scattered points and through its Fourier coefficients on a circle; and the
    Prop. 5 coefficients as the <u_inc, Phi^p_m> quadrature of this field."""
    from oracle import pointsource as ps
    k = 3.7
    O = np.array([0.4, -0.3])
    s = np.array([2.9, 1.6])
    rs, ts = np.hypot(*(s - O)), math.atan2(*(s - O)[::-1])
    rng = np.random.default_rng(11)
    rho = rng.uniform(0.05, 0.6 * rs, 30)
    phi = rng.uniform(0.0, 2 * np.pi, 30)
    pts = O[None, :] + rho[:, None] * np.stack([np.cos(phi), np.sin(phi)], 1)
    m = np.arange(-90, 91)
    ref = 0.25j * np.sum(sp.jv(m[None, :], k * rho[:, None]) * sp.hankel1(m, k * rs)[None, :]
                         * np.exp(1j * m[None, :] * (phi[:, None] - ts)), 1)
    u = ps.incident(k, s[None, :], pts)[0]
    assert rel(u, ref) < 1e-12
    # Fourier coefficients on the circle |x - O| = a
    a, N = 0.9, 14
    c = _circle_coefficients(lambda x, t: ps.incident(k, s[None, :], x)[0], O, a, N)
    mm = np.arange(-N, N + 1)
    want = 0.25j * sp.jv(mm, k * a) * sp.hankel1(mm, k * rs) * np.exp(-1j * mm * ts) * np.sqrt(2 * np.pi * a)
    assert rel(c, want) < 1e-12
    # Prop. 5 coefficients of a cluster are the projections of this field
    cl = synth.small_random(103, 3, 0.3, 0.8, 5.0, 0.3, 2.6, 6)
    src = np.array([[-1.2, 1.4]])
    U = ps.point_source(cl.centers, cl.radii, cl.n_modes, cl.k, src)
    off, _ = geometry.mode_offsets(cl.n_modes)
    for p in range(cl.M):
        cp = _circle_coefficients(lambda x, t: ps.incident(cl.k, src, x)[0], cl.centers[p],
                                  cl.radii[p], int(cl.n_modes[p]))
        assert rel(U[0, off[p]:off[p + 1]], cp) < 1e-12


def test_point_source_incident_field_is_the_outgoing_green_function():
    """(i/4) H_0(k |x - s|) is the outgoing fundamental solution of
    -(Laplace + k^2): the Helmholtz residual vanishes away from s (fourth-order
    finite differences), the flux of its gradient through a small circle about
    s is -1 (a unit source), its imaginary part tends to 1/4 at s, and it
    satisfies the radiation condition r^{1/2} (d_r u - i k u) -> 0."""
    from oracle import pointsource as ps
    k = 2.3
    s = np.array([[0.7, -0.4]])
    u = lambda x: ps.incident(k, s, np.atleast_2d(x))[0]
    h = 1e-2
    for x0 in ([1.9, 0.3], [-2.0, 1.1], [0.9, 2.5]):
        x0 = np.array(x0)
        lap = 0.0
        for e in (np.array([1.0, 0.0]), np.array([0.0, 1.0])):
            f = u(np.stack([x0 - 2 * h * e, x0 - h * e, x0, x0 + h * e, x0 + 2 * h * e]))
            lap = lap + (-f[0] + 16 * f[1] - 30 * f[2] + 16 * f[3] - f[4]) / (12 * h * h)
        res = lap + k * k * u(x0)[0]
        assert abs(res) < 1e-6 * abs(k * k * u(x0)[0])
    # flux through |x - s| = eps by the trapezoid rule on d_r u (central differences)
    eps, d = 1e-3, 1e-6
    t = 2 * np.pi * np.arange(64) / 64
    e = np.stack([np.cos(t), np.sin(t)], 1)
    dr = (u(s + (eps + d) * e) - u(s + (eps - d) * e)) / (2 * d)
    flux = np.sum(dr) * (2 * np.pi / 64) * eps
    assert abs(flux - (-1.0)) < 1e-4
    assert abs(u(s + 1e-7 * e[:1])[0].imag - 0.25) < 1e-6
    # radiation condition: r^{1/2} |d_r u - i k u| decays like r^{-1}
    vals = []
    for r in (50.0, 200.0, 800.0):
        x = s + r * e[3:4]
        drr = (u(x + 1e-4 * e[3:4]) - u(x - 1e-4 * e[3:4]))[0] / 2e-4
        vals.append(np.sqrt(r) * abs(drr - 1j * k * u(x)[0]))
    assert vals[1] < 0.3 * vals[0] and vals[2] < 0.3 * vals[1]

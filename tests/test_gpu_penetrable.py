"""GPU parity of the penetrable-disk transmission problem (sec. 7, Example II)
against the CPU oracle, through the C ABI via the binding.

The GPU solves the reduced one-unknown equation (rho- eliminated mode by mode);
the oracle solves the 2 x 2 block system, so the comparison of rho+ and of the
far field also checks the reduction.  Tolerances: applies 1e-12 (norm-wise);
solves at tol 1e-13: densities and far fields 1e-10; closed forms 1e-10;
properties at full size (optical theorem) 1e-9.
"""
import numpy as np
import pytest
import torch
from scipy import special as sp

import synth
from oracle import nearfield, operators as ops, penetrable as pen, rhs as orhs

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def P():
    from paper_1409_8186_amd import Problem
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return Problem


CLUSTERS = {
    # uniform N <= 12: one-lane kernel for R = 1, MFMA for R >= 8
    "uniform": lambda: synth.Cluster(*synth.random_disks(np.random.default_rng(91), 9, 0.3, 0.7, 0.0, 7.0, 0.3),
                                     np.full(9, 8, np.int32), 3.5),
    # uneven N: generic kernel for R = 1
    "uneven": lambda: synth.small_random(92, 7, 0.3, 0.9, 7.0, 0.3, 4.0, 4),
}


def _media(M, k, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.5, 2.5, M) * k, rng.uniform(0.6, 2.0, M)


def _reduced(cl, ki, mu):
    """(N+ - I/2) - diag(mu (I/2 + N-) / L-) L+: the second block row after
    eliminating rho- with the first (any per-row scaling gives the same D^-1 op)."""
    Lp = ops.operator_matrix("L", cl.centers, cl.radii, cl.n_modes, cl.k)
    Np = ops.operator_matrix("N", cl.centers, cl.radii, cl.n_modes, cl.k)
    Lm, Nm = pen.interior_diagonals(cl.radii, cl.n_modes, ki)
    disk = np.repeat(np.arange(len(cl.radii)), 2 * np.asarray(cl.n_modes) + 1)
    return Np - 0.5 * np.eye(len(Lm)) - (mu[disk] * Nm / Lm)[:, None] * Lp


@pytest.mark.parametrize("cname", ["uniform", "uneven"])
@pytest.mark.parametrize("R", [1, 9])
def test_penetrable_apply_matches_oracle(P, cname, R):
    from paper_1409_8186_amd import _lib as L
    cl = CLUSTERS[cname]()
    ki, mu = _media(len(cl.radii), cl.k, 1)
    red = _reduced(cl, ki, mu)
    A = red / np.diag(red)[:, None]
    rng = np.random.default_rng(R)
    x = rng.standard_normal((R, red.shape[0])) + 1j * rng.standard_normal((R, red.shape[0]))
    pr = P.from_cluster(cl)
    pr.set_penetrable(ki, mu)
    y = pr.matvec(torch.tensor(x.reshape(-1), device="cuda"), R=R, op=L.OP_A).cpu().numpy().reshape(R, -1)
    say(cname, R, "D^-1 op x rel", rel(y, x @ A.T))
    assert rel(y, x @ A.T) < 1e-12


def test_penetrable_solve_and_farfield_match_oracle(P):
    """Two instances (different k), per-disk k- and mu, three incidences."""
    c1 = synth.small_random(93, 6, 0.3, 0.8, 6.0, 0.3, 3.0, 5)
    c2 = synth.small_random(94, 5, 0.3, 0.9, 6.0, 0.3, 4.5, 5)
    k1, m1 = _media(6, c1.k, 2)
    k2, m2 = _media(5, c2.k, 3)
    betas = np.array([[0.3, 1.9, 4.4], [2.0, 0.1, 5.5]])
    th = synth.uniform_angles(48)
    pr = P.from_clusters([c1, c2])
    pr.set_penetrable(np.concatenate([k1, k2]), np.concatenate([m1, m2]))
    rho, flag, relres, iters, _ = pr.gmres(betas=betas, restart=30, tol=1e-13, maxit=2000)
    assert np.all(flag.cpu().numpy() == 0), relres
    parts = pr.split(rho, R=3)
    af = pr.farfield(rho, th, R=3).cpu().numpy().reshape(2, 3, -1)
    for b, (cl, ki, mu) in enumerate([(c1, k1, m1), (c2, k2, m2)]):
        rp, _ = pen.solve(cl.centers, cl.radii, cl.n_modes, cl.k, ki, betas[b], mu=mu)
        say("instance", b, "rho+ rel", rel(parts[b].cpu().numpy(), rp))
        assert rel(parts[b].cpu().numpy(), rp) < 1e-10
        ref = pen.farfield(cl.centers, cl.radii, cl.n_modes, cl.k, rp, th)
        assert rel(af[b], ref) < 1e-10
    # near field of the first instance against the oracle total field of rho+
    pr1 = P.from_cluster(c1)
    pr1.set_penetrable(k1, m1)
    rho1, flag1, _, _, _ = pr1.gmres(betas=betas[:1], restart=30, tol=1e-13, maxit=2000)
    rp, _ = pen.solve(c1.centers, c1.radii, c1.n_modes, c1.k, k1, betas[0], mu=m1)
    g = np.linspace(-2.0, 8.0, 30)
    pts = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    ut = pr1.nearfield(rho1, pts, R=3, betas=betas[:1]).cpu().numpy()
    ref = nearfield.total_field(c1.centers, c1.radii, c1.n_modes, c1.k, rp, pts, betas[0])
    assert rel(ut, ref) < 1e-10


@pytest.mark.parametrize("ki,mu", [(8.0, 1.0), (2.4, 1.0), (6.0, 2.5)])
def test_penetrable_single_disk_transmission_mie(P, ki, mu):
    """One disk: matching the field and mu times its normal derivative across
    the circle mode by mode gives c_m = (mu k- J'(k- a) J(k a) - k J(k- a) J'(k a))
    / (k J(k- a) H'(k a) - mu k- J'(k- a) H(k a)) for the scattered field."""
    O, a, k, N, beta = np.array([0.4, -0.6]), 0.8, 4.0, 18, 0.7
    cl = synth.Cluster(O[None, :], np.array([a]), np.array([N], np.int32), k)
    pr = P.from_cluster(cl)
    pr.set_penetrable([ki], [mu])
    rho, flag, _, _, _ = pr.gmres(betas=[[beta]], restart=40, tol=1e-14, maxit=400)
    th = synth.uniform_angles(36)
    af = pr.farfield(rho, th).cpu().numpy()[0]
    m = np.arange(-N, N + 1)
    Ji, Jid = sp.jv(m, ki * a), sp.jvp(m, ki * a)
    J, Jd, H, Hd = sp.jv(m, k * a), sp.jvp(m, k * a), sp.hankel1(m, k * a), sp.h1vp(m, k * a)
    c = (mu * ki * Jid * J - k * Ji * Jd) / (k * Ji * Hd - mu * ki * Jid * H)
    ph = np.exp(1j * k * ((np.cos(beta) - np.cos(th)) * O[0] + (np.sin(beta) - np.sin(th)) * O[1]))
    ref = np.exp(-0.25j * np.pi) * np.sqrt(2.0 / (np.pi * k)) * ph * np.sum(
        c[None, :] * np.exp(1j * m[None, :] * (th[:, None] - beta)), axis=1)
    assert rel(af, ref) < 1e-10


def test_penetrable_matched_medium_has_no_right_hand_side(P):
    """k- = k and mu = 1: the reduced right-hand side -J dU + k J' U vanishes mode
    by mode (no scattered field), to rounding of the two Bessel tables."""
    cl = synth.small_random(95, 6, 0.3, 0.8, 6.0, 0.3, 3.0, 6)
    betas = [0.5, 2.0]
    pr = P.from_cluster(cl)
    pr.set_penetrable(cl.k)
    b = pr.rhs([betas]).cpu().numpy().reshape(2, -1)
    U = orhs.planewave(cl.centers, cl.radii, cl.n_modes, cl.k, betas)
    dU = ops.planewave_dn(cl.centers, cl.radii, cl.n_modes, cl.k, betas)
    assert np.all(np.abs(b) <= 1e-13 * np.maximum(np.abs(U), np.abs(dU)) + 1e-300)


def test_penetrable_reset_and_gradient_guard(P):
    from paper_1409_8186_amd import _lib as L
    cl = CLUSTERS["uneven"]()
    pr = P.from_cluster(cl)
    r0, _, _, _, _ = pr.gmres(betas=[[0.8]], tol=1e-12)
    pr.set_penetrable(1.7 * cl.k, 1.3)
    with pytest.raises(L.MudiffError):
        pr.grad([[0.8]], [0.1, 0.2], torch.zeros(2, dtype=torch.complex128, device="cuda"))
    pr.set_operator(None)
    r1, _, _, _, _ = pr.gmres(betas=[[0.8]], tol=1e-12)
    assert torch.allclose(r0, r1, rtol=0, atol=1e-13 * float(r0.abs().max()))


def test_penetrable_full_size_optical_theorem(P):
    """The one-RHS geometry (M = 400, N_p = 12, k = 2 pi) with k- = 1.5 k and mu
    in [0.6, 2]: solve to 1e-12, then energy conservation
    int |a|^2 = -sqrt(8 pi / k) Re(e^{i pi/4} a(beta; beta)), which the truncated
    system keeps exactly for real k- and mu (4096 far-field angles integrate |a|^2
    exactly here)."""
    cl = synth.one_rhs()
    beta = np.pi / 4
    mu = np.random.default_rng(6).uniform(0.6, 2.0, len(cl.radii))
    pr = P.from_cluster(cl)
    pr.set_penetrable(1.5 * cl.k, mu)
    rho, flag, relres, iters, _ = pr.gmres(betas=[[beta]], restart=50, tol=1e-12, maxit=20000, graph=True)
    say("iterations", int(iters[0]), "relres", float(relres[0]))
    assert int(flag[0]) == 0
    nt = 4096
    a = pr.farfield(rho, synth.uniform_angles(nt)).cpu().numpy()[0]
    a0 = pr.farfield(rho, [beta]).cpu().numpy()[0, 0]
    lhs = np.sum(np.abs(a) ** 2) * 2 * np.pi / nt
    rhs_ = -np.sqrt(8 * np.pi / cl.k) * np.real(np.exp(0.25j * np.pi) * a0)
    say("optical theorem", lhs, rhs_)
    assert abs(lhs - rhs_) < 1e-9 * abs(rhs_)


def _inside_points(cl, n, rng):
    p = rng.integers(0, len(cl.radii), n)
    rr = cl.radii[p] * np.sqrt(rng.uniform(0, 1, n))
    t = rng.uniform(0, 2 * np.pi, n)
    return cl.centers[p] + rr[:, None] * np.stack([np.cos(t), np.sin(t)], 1), p


@pytest.mark.parametrize("kind", ["plane", "point"])
def test_penetrable_interior_field_matches_oracle(P, kind):
    """Interior field (from the Dirichlet trace U + L+ rho+) against the oracle's
    L- rho- with rho- from its block solve; points outside the disks keep the
    near field's total field.  (Continuity across the circles is truncation-
    limited, 1e-6..5e-4 here; the oracle pins it with its convergence in N.)"""
    from oracle import pointsource as ps
    cl = synth.small_random(96, 5, 0.3, 0.8, 6.0, 0.3, 3.2, 6)
    ki, mu = _media(5, cl.k, 4)
    rng = np.random.default_rng(11)
    pin, which = _inside_points(cl, 300, rng)
    g = np.linspace(-1.0, 7.0, 20)
    pout = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    pts = np.concatenate([pin, pout])
    pr = P.from_cluster(cl)
    pr.set_penetrable(ki, mu)
    if kind == "plane":
        inc = dict(betas=[[0.6, 2.5]])
        rp, rm = pen.solve(cl.centers, cl.radii, cl.n_modes, cl.k, ki, [0.6, 2.5], mu=mu)
    else:
        src = np.array([[-1.5, 2.0], [8.0, 1.0]])
        inc = dict(sources=[src])
        U = ps.point_source(cl.centers, cl.radii, cl.n_modes, cl.k, src)
        dU = ps.point_source_dn(cl.centers, cl.radii, cl.n_modes, cl.k, src)
        rp, rm = pen.solve_coefficients(cl.centers, cl.radii, cl.n_modes, cl.k, ki, U, dU, mu)
    rho, flag, _, _, _ = pr.gmres(restart=30, tol=1e-13, maxit=2000, **inc)
    assert np.all(flag.cpu().numpy() == 0)
    tot = pr.nearfield(rho, pts, R=2, **inc)
    ext = tot.clone()
    u = pr.interior_field(rho, pts, R=2, out=tot, **inc).cpu().numpy()
    n_in = len(pin)
    ref = np.stack([np.concatenate([pen.interior_field(cl.centers, cl.radii, cl.n_modes, ki, rm[r], p, x[None, :])
                                    for x, p in zip(pin, which)]) for r in range(2)])
    say(kind, "interior rel", rel(u[:, :n_in], ref))
    assert rel(u[:, :n_in], ref) < 1e-10
    outside = np.ones(len(pts), bool)
    for c, a in zip(cl.centers, cl.radii):
        outside &= np.hypot(*(pts - c).T) >= a
    assert outside[n_in:].sum() > 300
    keep = torch.tensor(outside, device="cuda")
    assert torch.equal(tot[:, keep], ext[:, keep])


def test_penetrable_interior_field_many_incidences(P):
    """Nine incidences (the trace L+ rho+ on the FP64-MFMA apply), twice in a row
    with fresh workspaces, against the oracle."""
    cl = synth.Cluster(*synth.random_disks(np.random.default_rng(97), 6, 0.3, 0.7, 0.0, 6.0, 0.3),
                       np.full(6, 8, np.int32), 3.0)
    ki, mu = _media(6, cl.k, 5)
    betas = 2 * np.pi * np.arange(9) / 9
    rp, rm = pen.solve(cl.centers, cl.radii, cl.n_modes, cl.k, ki, betas, mu=mu)
    pin, which = _inside_points(cl, 60, np.random.default_rng(12))
    ref = np.stack([np.concatenate([pen.interior_field(cl.centers, cl.radii, cl.n_modes, ki, rm[r], p, x[None, :])
                                    for x, p in zip(pin, which)]) for r in range(9)])
    pr = P.from_cluster(cl)
    pr.set_penetrable(ki, mu)
    rho = pr.pack([rp])
    for _ in range(2):
        u = pr.interior_field(rho, pin, R=9, betas=[betas]).cpu().numpy()
        assert rel(u, ref) < 1e-11


def test_penetrable_time_reversal_matrix(P):
    """The mirror far-field matrix of three penetrable disks (the geometry of the
    time-reversal example, with k- = 2 k): F[i, j] = a(alpha_i + pi; alpha_j)
    against the oracle's block solve, F complex symmetric (reciprocity), and the
    eigenvalues of T = conj(F)^T F against LAPACK."""
    from paper_1409_8186_amd import tro, tro_eigh
    cl = synth.dort_example(64)
    ki = np.full(3, 2 * cl.k)
    n_alpha = 64
    al = 2 * np.pi * np.arange(n_alpha) / n_alpha
    rp, _ = pen.solve(cl.centers, cl.radii, cl.n_modes, cl.k, ki, al)
    Fo = pen.farfield(cl.centers, cl.radii, cl.n_modes, cl.k, rp, al + np.pi).T   # [receiver, incidence]
    pr = P.from_cluster(cl)
    pr.set_penetrable(ki)
    X, flag, relres, iters = pr.mirror_farfield(n_alpha, restart=30, tol=1e-13, maxit=500)
    assert np.all(flag.cpu().numpy() == 0)
    F = X.cpu().numpy().T
    assert rel(F, Fo) < 1e-10
    assert rel(F, F.T) < 1e-10
    w, ev, sweeps = tro_eigh(X)
    wo = np.sort(np.linalg.eigvalsh(Fo.conj().T @ Fo))[::-1]
    assert np.max(np.abs(w.cpu().numpy() - wo)) < 1e-10 * wo[0]
    say("penetrable T: leading eigenvalues", w.cpu().numpy()[:4])

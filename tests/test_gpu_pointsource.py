"""GPU parity of point-source incidence (Prop. 5) against the CPU oracle,
through the C ABI via the binding: right-hand sides, solves (sound-soft EFIE,
MFIE, penetrable disks), far and near fields with the point-source total field.

Tolerances: coefficients 1e-12 (H_m(k r) by upward recurrence from H_0, H_1:
relative error a few ulp per step where Y dominates); solves at tol 1e-13 and
the fields built on them 1e-10.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import farfield, nearfield, operator, operators as ops, penetrable as pen, pointsource as ps

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


def _two():
    c1 = synth.small_random(111, 6, 0.3, 0.8, 6.0, 0.3, 3.0, 5)
    c2 = synth.small_random(112, 5, 0.3, 0.9, 6.0, 0.3, 4.5, 9)
    # sources: one near a disk (k r below the asymptotic switch), one far
    # (k r above 25, 50 and 100), one inside the cluster box
    s1 = np.array([c1.centers[0] + (c1.radii[0] + 0.05) * np.array([1.0, 0.0]), [40.0, -25.0], [3.1, 3.3]])
    s2 = np.array([[-30.0, 2.0], c2.centers[2] + (c2.radii[2] + 0.02) * np.array([0.0, -1.0]), [2.9, 3.2]])
    return c1, c2, s1, s2


def test_point_source_rhs_matches_oracle(P):
    c1, c2, s1, s2 = _two()
    for cl, s in ((c1, s1), (c2, s2)):
        for c, a in zip(cl.centers, cl.radii):
            assert np.all(np.hypot(*(s - c).T) > a), "test sources must lie outside the disks"
    pr = P.from_clusters([c1, c2])
    src = np.stack([s1, s2])
    U = pr.split(pr.rhs(sources=src), R=3)
    f = pr.split(pr.rhs(sources=src, precond=True), R=3)
    for b, (cl, s) in enumerate([(c1, s1), (c2, s2)]):
        Uo = ps.point_source(cl.centers, cl.radii, cl.n_modes, cl.k, s)
        D = np.diag(operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k))
        say("instance", b, "U rel", rel(U[b].cpu().numpy(), Uo))
        assert rel(U[b].cpu().numpy(), Uo) < 1e-12
        assert rel(f[b].cpu().numpy(), -Uo / D[None, :]) < 1e-12


def test_point_source_efie_solve_and_fields_match_oracle(P):
    c1, c2, s1, s2 = _two()
    pr = P.from_clusters([c1, c2])
    rho, flag, relres, _, _ = pr.gmres(sources=np.stack([s1, s2]), restart=30, tol=1e-13, maxit=3000)
    assert np.all(flag.cpu().numpy() == 0), relres
    parts = pr.split(rho, R=3)
    th = synth.uniform_angles(40)
    af = pr.farfield(rho, th, R=3).cpu().numpy().reshape(2, 3, -1)
    g = np.linspace(-3.0, 9.0, 25)
    pts = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    ut = pr.nearfield(rho, pts, R=3, sources=np.stack([s1, s2])).cpu().numpy().reshape(2, 3, -1)
    for b, (cl, s) in enumerate([(c1, s1), (c2, s2)]):
        L = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
        ro = np.linalg.solve(L, -ps.point_source(cl.centers, cl.radii, cl.n_modes, cl.k, s).T).T
        say("instance", b, "rho rel", rel(parts[b].cpu().numpy(), ro))
        assert rel(parts[b].cpu().numpy(), ro) < 1e-10
        assert rel(af[b], ro @ farfield.farfield_rows(cl.centers, cl.radii, cl.n_modes, cl.k, th).T) < 1e-10
        ref = nearfield.potential(cl.centers, cl.radii, cl.n_modes, cl.k, ro, pts) + ps.incident(cl.k, s, pts)
        inside = np.zeros(len(pts), bool)
        for c, a in zip(cl.centers, cl.radii):
            inside |= np.hypot(*(pts - c).T) < a
        ref[:, inside] = 0.0
        assert rel(ut[b], ref) < 1e-10


def test_point_source_mfie_and_penetrable_match_oracle(P):
    """Formulations whose right-hand side takes dU (MFIE) and the penetrable
    transmission problem, with point sources."""
    cl = synth.small_random(113, 6, 0.3, 0.8, 6.0, 0.3, 3.4, 6)
    s = np.array([[-2.0, 1.0], [8.0, 7.5]])
    U = ps.point_source(cl.centers, cl.radii, cl.n_modes, cl.k, s)
    dU = ps.point_source_dn(cl.centers, cl.radii, cl.n_modes, cl.k, s)
    pr = P.from_cluster(cl)
    pr.set_operator("mfie")
    rho, flag, _, _, _ = pr.gmres(sources=[s], restart=30, tol=1e-13, maxit=3000)
    A = ops.combination({"I": 0.5, "N": 1.0}, cl.centers, cl.radii, cl.n_modes, cl.k)
    ro = np.linalg.solve(A, -dU.T).T
    assert rel(rho.cpu().numpy().reshape(2, -1), ro) < 1e-10
    ki, mu = np.linspace(0.5, 2.2, 6) * cl.k, np.linspace(0.7, 1.8, 6)
    pr.set_penetrable(ki, mu)
    rho, flag, _, _, _ = pr.gmres(sources=[s], restart=30, tol=1e-13, maxit=3000)
    rp, _ = pen.solve_coefficients(cl.centers, cl.radii, cl.n_modes, cl.k, ki, U, dU, mu)
    assert rel(rho.cpu().numpy().reshape(2, -1), rp) < 1e-10


def test_point_source_reciprocity_on_the_gpu(P):
    """u^s(x; s) = u^s(s; x) from two GPU solves (sound-soft, one-lane kernel)."""
    cl = synth.Cluster(*synth.random_disks(np.random.default_rng(114), 12, 0.3, 0.7, 0.0, 8.0, 0.3),
                       np.full(12, 10, np.int32), 3.0)
    sa, sb = np.array([-1.0, 4.0]), np.array([9.5, 2.0])
    pr = P.from_cluster(cl)
    rho, flag, _, _, _ = pr.gmres(sources=[[sa, sb]], restart=40, tol=1e-13, maxit=3000)
    u = pr.nearfield(rho, np.stack([sb, sa]), R=2).cpu().numpy()
    assert abs(u[0, 0] - u[1, 1]) < 1e-10 * abs(u[0, 0])


def test_point_source_inside_a_disk_is_flagged(P):
    """A source inside a disk has no expansion on that circle: NaN coefficients
    for that disk and GMRES flag 2 for its column; other columns solve."""
    cl = synth.small_random(115, 4, 0.3, 0.8, 5.0, 0.3, 3.0, 5)
    bad = cl.centers[1] + 0.2 * cl.radii[1]
    good = np.array([-2.0, -2.0])
    pr = P.from_cluster(cl)
    U = pr.rhs(sources=[[good, bad]]).cpu().numpy().reshape(2, -1)
    assert np.all(np.isfinite(U[0]))
    n0 = 2 * int(cl.n_modes[0]) + 1
    n1 = 2 * int(cl.n_modes[1]) + 1
    assert np.all(np.isfinite(U[1, :n0])) and np.all(np.isnan(U[1, n0:n0 + n1]))
    rho, flag, _, _, _ = pr.gmres(sources=[[good, bad]], restart=20, tol=1e-12, maxit=500)
    assert flag.cpu().numpy().tolist() == [0, 2]


def test_point_source_penetrable_graph_replay_matches_eager(P):
    """Restart cycles replayed as HIP graphs give the eager solve bit for bit,
    also with the penetrable tables and point sources (uniform N: one-lane
    kernel; 9 sources: FP64 MFMA)."""
    cl = synth.Cluster(*synth.random_disks(np.random.default_rng(116), 10, 0.3, 0.7, 0.0, 8.0, 0.3),
                       np.full(10, 9, np.int32), 3.0)
    ang = 2 * np.pi * np.arange(9) / 9
    src = np.stack([4.0 + 7.5 * np.cos(ang), 4.0 + 7.5 * np.sin(ang)], 1)
    pr = P.from_cluster(cl)
    pr.set_penetrable(1.6 * cl.k, 1.2)
    for s in (src[:1], src):
        r_e, f_e, _, it_e, _ = pr.gmres(sources=[s], restart=20, tol=1e-12, maxit=400, graph=False)
        r_g, f_g, _, it_g, _ = pr.gmres(sources=[s], restart=20, tol=1e-12, maxit=400, graph=True)
        assert np.all(f_e.cpu().numpy() == 0)
        assert torch.equal(it_e, it_g) and torch.equal(r_e, r_g)


def test_mixed_reciprocity_on_the_gpu(P):
    """GPU only: the far field at theta of the point-source solve equals
    e^{i pi/4} / sqrt(8 pi k) times the plane-wave (direction -theta) scattered
    field at the source, for sound-soft and penetrable disks."""
    cl = synth.Cluster(*synth.random_disks(np.random.default_rng(132), 12, 0.3, 0.7, 0.0, 8.0, 0.3),
                       np.full(12, 10, np.int32), 3.0)
    src = np.array([[-1.0, 4.0], [9.5, 2.0], [4.0, 10.0]])
    th = np.array([0.2, 2.1, 3.9, 5.5])
    gam = np.exp(0.25j * np.pi) / np.sqrt(8 * np.pi * cl.k)
    pr = P.from_cluster(cl)
    for pen_on in (False, True):
        if pen_on:
            pr.set_penetrable(1.7 * cl.k, 1.4)
        r_ps, f1, _, _, _ = pr.gmres(sources=[src], restart=40, tol=1e-13, maxit=3000)
        a_ps = pr.farfield(r_ps, th, R=3).cpu().numpy()                       # [source, theta]
        r_pw, f2, _, _, _ = pr.gmres(betas=[th + np.pi], restart=40, tol=1e-13, maxit=3000)
        u_pw = pr.nearfield(r_pw, src, R=4).cpu().numpy()                      # [theta, source]
        assert np.all(f1.cpu().numpy() == 0) and np.all(f2.cpu().numpy() == 0)
        assert rel(a_ps, gam * u_pw.T) < 1e-10

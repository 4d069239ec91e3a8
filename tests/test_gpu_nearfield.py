"""GPU parity of the near field (sec. 4.4) against the CPU oracle through the C ABI.

The densities come from the oracle's dense solve, so the near-field kernel is
tested on its own; tolerance 1e-11 of the largest value (a sum of H_m(k r)
e^{i m theta} terms: the upward recurrence for H_m keeps eps |H_m| where the Y
part dominates)."""
import numpy as np
import pytest
import torch
from scipy import special as sp

import synth
from oracle import nearfield, operator, operators as ops, rhs, solve

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def P():
    from paper_1409_8186_amd import Problem
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return Problem


def _points(cl, n, rng, spread=3.0):
    """Points around the cluster: uniform in its box, some just outside a circle
    (arguments below and above the asymptotic switch), some inside disks."""
    lo = cl.centers.min(0) - spread
    hi = cl.centers.max(0) + spread
    u = rng.uniform(lo, hi, size=(n, 2))
    p = rng.integers(0, len(cl.radii), n // 4)
    t = rng.uniform(0, 2 * np.pi, n // 4)
    f = rng.uniform(1.0 + 1e-9, 1.3, n // 4)
    near = cl.centers[p] + (cl.radii[p] * f)[:, None] * np.stack([np.cos(t), np.sin(t)], 1)
    ins = cl.centers[p[:8]] + 0.5 * cl.radii[p[:8], None] * np.stack([np.cos(t[:8]), np.sin(t[:8])], 1)
    return np.concatenate([u, near, ins])


def _close(got, ref, tol=1e-11):
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref)), np.max(np.abs(got - ref)) / np.max(np.abs(ref))


def test_nearfield_single_layer_matches_oracle(P):
    cl = synth.small_random(71, 7, 0.3, 1.0, 8.0, 0.3, 4.5, 5)
    L = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    U = rhs.planewave(cl.centers, cl.radii, cl.n_modes, cl.k, [0.4, 2.2, 3.7, 5.0, 0.1])
    rho = solve.efie_solve_lu(L, U)                        # [5, N]
    pts = _points(cl, 400, np.random.default_rng(1))
    pr = P.from_cluster(cl)
    rd = torch.tensor(rho.reshape(-1), device="cuda")
    u = pr.nearfield(rd, pts, R=5).cpu().numpy()
    ref = nearfield.potential(cl.centers, cl.radii, cl.n_modes, cl.k, rho, pts)
    _close(u, ref)
    betas = np.array([[0.4, 2.2, 3.7, 5.0, 0.1]])
    ut = pr.nearfield(rd, pts, R=5, betas=betas).cpu().numpy()
    _close(ut, nearfield.total_field(cl.centers, cl.radii, cl.n_modes, cl.k, rho, pts, betas[0]))
    inside = np.zeros(len(pts), bool)
    for c, a in zip(cl.centers, cl.radii):
        inside |= np.hypot(*(pts - c).T) < a
    assert inside.sum() >= 8 and np.all(u[:, inside] == 0) and np.all(ut[:, inside] == 0)


def test_nearfield_with_double_layer_weights(P):
    """After set_operator('bwie'): u = -(eta L + M) psi."""
    cl = synth.small_random(72, 5, 0.3, 0.9, 7.0, 0.3, 3.5, 5)
    eta = 1j * cl.k
    dens, _ = ops.solve_farfield("bwie", cl.centers, cl.radii, cl.n_modes, cl.k, [0.7], [0.0], eta=eta)
    pts = _points(cl, 200, np.random.default_rng(2))
    pr = P.from_cluster(cl)
    pr.set_operator("bwie", eta=eta)
    u = pr.nearfield(torch.tensor(dens.reshape(-1), device="cuda"), pts).cpu().numpy()[0]
    ref = nearfield.potential(cl.centers, cl.radii, cl.n_modes, cl.k, dens[0], pts, -eta, -1.0)
    _close(u, ref)


def test_nearfield_single_disk_total_field_mie(P):
    """GPU solve + near field of one sound-soft disk against the textbook total field."""
    O, a, k, N, beta = np.array([0.4, -0.3]), 0.8, 3.5, 16, 0.9
    cl = synth.Cluster(O[None, :], np.array([a]), np.array([N], np.int32), k)
    pr = P.from_cluster(cl)
    rho, flag, _, _, _ = pr.gmres(betas=[[beta]], restart=20, tol=1e-14, maxit=300)
    rng = np.random.default_rng(4)
    rr = rng.uniform(1.05 * a, 4.0, 50)
    tt = rng.uniform(0, 2 * np.pi, 50)
    pts = np.stack([O[0] + rr * np.cos(tt), O[1] + rr * np.sin(tt)], 1)
    ut = pr.nearfield(rho, pts, betas=[[beta]]).cpu().numpy()[0]
    m = np.arange(-40, 41)
    ref = np.exp(1j * k * (np.cos(beta) * O[0] + np.sin(beta) * O[1])) * np.sum(
        (1j ** m)[None, :] * (sp.jv(m[None, :], k * rr[:, None])
                              - sp.jv(m, k * a)[None, :] * sp.hankel1(m[None, :], k * rr[:, None])
                              / sp.hankel1(m, k * a)[None, :])
        * np.exp(1j * m[None, :] * (tt[:, None] - beta)), axis=1)
    assert np.max(np.abs(ut - ref)) < 1e-10


def test_nearfield_full_size_sampled(P):
    """The one-RHS geometry (M = 400, N_p = 12): GPU solve to 1e-12, total field
    on a 120 x 120 grid over the cluster; a 300-point sample against the oracle
    potential of the GPU density."""
    cl = synth.one_rhs()
    pr = P.from_cluster(cl)
    rho, flag, _, _, _ = pr.gmres(betas=[[np.pi / 4]], restart=50, tol=1e-12, maxit=20000, graph=True)
    assert int(flag[0]) == 0
    g = np.linspace(-5.0, 65.0, 120)
    pts = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    ut = pr.nearfield(rho, pts, betas=[[np.pi / 4]]).cpu().numpy()[0]
    idx = np.random.default_rng(5).choice(len(pts), 300, replace=False)
    ref = nearfield.total_field(cl.centers, cl.radii, cl.n_modes, cl.k, rho.cpu().numpy()[None, :],
                                pts[idx], [np.pi / 4])[0]
    _close(ut[idx], ref)
    say("max |u_t| on the grid", float(np.max(np.abs(ut))))

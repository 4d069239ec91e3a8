"""GPU parity of s-step GMRES (MUDIFF_SSTEP): after a first cycle of the
one-vector process, each cycle builds its basis ss Newton vectors at a time
(shifts: the first cycle's Ritz values in Leja order) and orthogonalises them
in one block.  The iterates are those of GMRES up to rounding, so every column
must equal its dense LU solution (the oracle) to the parity bar, 1e-10, at
tol 1e-12, with nearly the iteration count of the one-vector solver, on the
one-lane apply (uniform N_p, R = 1), the generic apply (uneven N_p, R = 3) and
the multi-right-hand-side applies (FP64-MFMA direct form, R = 8; circulant form,
R = 13), eager and replayed as graphs, with and without the preconditioner."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import operator, rhs, solve

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


def _dense_uniform(seed=61, M=60, N=10):
    """A crowded lattice-like cluster (about 25% area fraction) that needs a few
    hundred iterations: several s-step cycles at restart 30."""
    cl = synth.small_random(seed, M, 0.5, 0.5, 14.0, 0.2, 2 * np.pi, 0)
    return synth.Cluster(cl.centers, cl.radii, np.full(cl.M, N, np.int32), cl.k)


def _lu(cl, betas, precond=True):
    L = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    U = rhs.planewave(cl.centers, cl.radii, cl.n_modes, cl.k, betas)
    return solve.efie_solve_lu(L, U)


@pytest.mark.parametrize("ss", [4, 8, 16])
def test_sstep_one_lane_matches_lu(P, ss):
    cl = _dense_uniform()
    pr = P.from_cluster(cl)
    betas = [[np.pi / 4]]
    say("s-step one-lane, ss", ss)
    rho1, flag1, _, it1, _ = pr.gmres(betas=betas, restart=30, tol=1e-12, maxit=5000)
    rho, flag, relres, iters, resvec = pr.gmres(betas=betas, restart=30, tol=1e-12, maxit=5000,
                                                sstep=ss, want_resvec=True)
    n1, n = int(it1[0]), int(iters[0])
    say("  iterations: one-vector", n1, "s-step", n)
    assert int(flag[0]) == 0 and float(relres[0]) <= 1e-12
    assert n > 60  # several s-step cycles ran
    assert abs(n - n1) <= max(3, n1 // 50)
    assert rel(rho.cpu().numpy(), _lu(cl, betas[0])[0]) < 1e-10
    # the estimates decrease within every cycle (minimisation over a growing space)
    e = resvec.cpu().numpy()[0, :n + 1]
    for c0 in range(0, n, 30):
        blk = e[c0 + 1:min(n, c0 + 30) + 1]
        assert np.all(np.diff(blk) <= 1e-12 * blk[:-1] + 1e-16)


def test_sstep_generic_path_graph_and_options(P):
    """Uneven orders (the generic apply), three incidences, a ragged last block
    (restart 20, ss 8), graph replays equal to the eager solve, and the solve
    without the preconditioner."""
    cl = synth.small_random(62, 40, 0.3, 0.9, 13.0, 0.15, 6.0, 3)
    betas = [[0.3, 1.7, 4.0]]
    pr = P.from_cluster(cl)
    say("s-step generic path")
    rho, flag, _, iters, _ = pr.gmres(betas=betas, restart=20, tol=1e-12, maxit=5000, sstep=8)
    say("  iterations", iters.cpu().numpy().tolist())
    assert torch.all(flag == 0) and int(iters.min()) > 40
    ref = _lu(cl, betas[0])
    assert rel(pr.split(rho, 3)[0].cpu().numpy(), ref) < 1e-10
    for rep in range(3):
        rho_g, flag_g, _, it_g, _ = pr.gmres(betas=betas, restart=20, tol=1e-12, maxit=5000, sstep=8,
                                             graph=True)
        torch.cuda.synchronize()
        assert torch.equal(it_g, iters) and torch.equal(flag_g, flag) and torch.equal(rho_g, rho), rep
    # without the preconditioner (L rho = -U itself), on a sparser cluster where
    # restarted GMRES converges: the same iterations as the one-vector solver
    cs = synth.small_random(64, 16, 0.3, 0.9, 16.0, 0.3, 4.0, 3)
    ps = P.from_cluster(cs)
    _, flag1, _, it1, _ = ps.gmres(betas=betas, restart=30, tol=1e-12, maxit=20000, precond=False)
    rho3, flag3, _, it3, _ = ps.gmres(betas=betas, restart=30, tol=1e-12, maxit=20000, sstep=8,
                                      precond=False)
    say("  no preconditioner: one-vector", it1.cpu().numpy().tolist(), "s-step", it3.cpu().numpy().tolist())
    assert torch.all(flag1 == 0) and torch.all(flag3 == 0)
    assert int((it3 - it1).abs().max()) <= max(3, int(it1.max()) // 50)
    assert rel(ps.split(rho3, 3)[0].cpu().numpy(), _lu(cs, betas[0])) < 1e-10


def test_sstep_mfma_direct_matches_lu(P):
    """R = 8 on the FP64-MFMA direct form: the shift is applied in its epilogue;
    every column equals LU and needs about the lockstep solver's iterations."""
    cl = _dense_uniform()
    R = 8
    betas = [synth.uniform_angles(R) + 0.05]
    pr = P.from_cluster(cl)
    say("s-step MFMA direct form")
    _, flag1, _, it1, _ = pr.gmres(betas=betas, restart=30, tol=1e-12, maxit=5000)
    rho, flag, relres, iters, _ = pr.gmres(betas=betas, restart=30, tol=1e-12, maxit=5000, sstep=10)
    assert pr.apply_config(R)["kind"] == "mfma"
    n1, n = it1.cpu().numpy(), iters.cpu().numpy()
    say("  iterations: lockstep", n1.tolist(), "s-step", n.tolist())
    assert torch.all(flag1 == 0) and torch.all(flag == 0) and torch.all(relres <= 1e-12)
    assert n.min() > 60
    assert np.abs(n - n1).max() <= max(3, int(n1.max()) // 50)
    assert rel(pr.split(rho, R)[0].cpu().numpy(), _lu(cl, betas[0])) < 1e-10


def test_sstep_many_columns_wide_sweeps(P):
    """R = 32 (320 Gram-Schmidt chunks): the sweeps run as their wide variants
    (LDS-staged row tiles, one thread per row); LU parity for every column,
    the lockstep solver's iterations, graph replays equal to the eager solve."""
    cl = _dense_uniform()
    R = 32
    betas = [synth.uniform_angles(R) + 0.02]
    pr = P.from_cluster(cl)
    say("s-step wide sweeps, R", R)
    _, _, _, it1, _ = pr.gmres(betas=betas, restart=30, tol=1e-12, maxit=5000)
    rho, flag, relres, iters, _ = pr.gmres(betas=betas, restart=30, tol=1e-12, maxit=5000, sstep=15)
    n1, n = it1.cpu().numpy(), iters.cpu().numpy()
    say("  iterations: lockstep", int(n1.max()), "s-step", int(n.max()), int(n.min()))
    assert torch.all(flag == 0) and torch.all(relres <= 1e-12)
    assert n.min() > 60
    assert np.abs(n - n1).max() <= max(3, int(n1.max()) // 50)
    ref = _lu(cl, betas[0])
    assert rel(pr.split(rho, R)[0].cpu().numpy(), ref) < 1e-10
    rho_g, flag_g, _, it_g, _ = pr.gmres(betas=betas, restart=30, tol=1e-12, maxit=5000, sstep=15,
                                         graph=True)
    torch.cuda.synchronize()
    assert torch.equal(it_g, iters) and torch.equal(flag_g, flag) and torch.equal(rho_g, rho)


def test_sstep_circulant_graph_matches_lu(P):
    """Two instances in the circulant form at R = 13 (ragged 8-column tiles),
    restart 22 with blocks of 5 (a ragged last block of 2): LU parity for every
    column, graph replays equal to the eager solve bit for bit."""
    cls = [synth.small_random(501, 30, 0.3, 1.0, 3.6 * math.sqrt(30), 0.1, 6.0, 4),
           synth.small_random(502, 18, 0.2, 0.8, 16.0, 0.1, 9.0, 3)]
    R = 13
    betas = np.stack([synth.uniform_angles(R), synth.uniform_angles(R) + 0.05])
    pr = P.from_clusters(cls, circulant=True)
    pr.set_circulant(R, 1)
    say("s-step circulant form")
    _, _, _, it1, _ = pr.gmres(betas=betas, restart=22, tol=1e-12, maxit=3000)
    rho, flag, _, iters, _ = pr.gmres(betas=betas, restart=22, tol=1e-12, maxit=3000, sstep=5)
    assert pr.apply_config(R)["kind"] == "circulant"
    n1, n = it1.cpu().numpy(), iters.cpu().numpy()
    say("  iterations: lockstep", n1.tolist(), "s-step", n.tolist())
    assert torch.all(flag == 0)
    assert n.max() > 44  # s-step cycles ran
    assert np.abs(n - n1).max() <= max(3, int(n1.max()) // 50)
    for b, (c, Y) in enumerate(zip(cls, pr.split(rho, R))):
        assert rel(Y.cpu().numpy(), _lu(c, betas[b])) < 1e-10, b
    for rep in range(3):
        rho_g, flag_g, _, it_g, _ = pr.gmres(betas=betas, restart=22, tol=1e-12, maxit=3000, sstep=5,
                                             graph=True)
        torch.cuda.synchronize()
        assert torch.equal(it_g, iters) and torch.equal(flag_g, flag) and torch.equal(rho_g, rho), rep


def test_sstep_first_cycle_only_and_invalid(P):
    """A problem that converges inside the first cycle never reaches the s-step
    cycles; invalid sizes are refused."""
    cl = synth.small_random(63, 4, 0.4, 0.6, 10.0, 0.5, 2.0, 2)
    pr = P.from_cluster(cl)
    rho, flag, _, iters, _ = pr.gmres(betas=[[0.5]], restart=50, tol=1e-12, maxit=2000, sstep=8)
    assert int(flag[0]) == 0 and int(iters[0]) < 50
    assert rel(rho.cpu().numpy(), _lu(cl, [0.5])[0]) < 1e-10
    from paper_1409_8186_amd import _lib
    for kw in ({"sstep": 1}, {"sstep": 17}, {"sstep": 8, "restart": 200}, {"sstep": 8, "block": 4}):
        args = {"restart": 30, **kw}
        with pytest.raises(_lib.MudiffError):
            pr.gmres(betas=[[0.5]], tol=1e-8, maxit=10, **args)


def test_sstep_guard_on_a_hard_instance(P):
    """Instance 93 of the uneven workload (62 disks, N_p up to 28, 8 incidences)
    at restart 64 with blocks of 16: the Newton basis from its first cycle's
    Ritz values loses orthogonality, and without the cycle guard the s-step
    solve stalls near 1e-2.  With it, a cycle that raises a true residual is
    undone and the solve goes on with one-vector cycles: it converges like the
    lockstep solver, and the oracle's dense operator confirms the residual."""
    cl = synth.uneven_instances()[93]
    R = len(cl.betas)
    pr = P.from_cluster(cl)
    say("s-step guard, hard instance: M", cl.M, "unknowns", cl.n_tot)
    _, flag1, _, it1, _ = pr.gmres(betas=[cl.betas], restart=64, tol=1e-8, maxit=4000)
    rho, flag, relres, iters, _ = pr.gmres(betas=[cl.betas], restart=64, tol=1e-8, maxit=4000, sstep=16)
    n1, n = int(it1.max()), int(iters.max())
    say("  iterations: lockstep", n1, "s-step", n, "relres", float(relres.max()))
    assert torch.all(flag1 == 0) and torch.all(flag == 0)
    assert n <= 1.2 * n1
    L = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    D = operator.efie_diagonal(cl.radii, cl.n_modes, cl.k)
    A = operator.preconditioned(L, D)
    F = -rhs.planewave(cl.centers, cl.radii, cl.n_modes, cl.k, cl.betas) / D[None, :]
    X = pr.split(rho, R)[0].cpu().numpy()
    res = np.linalg.norm(X @ A.T - F, axis=1) / np.linalg.norm(F, axis=1)
    say("  oracle residual of D^-1 L rho = -D^-1 U", float(res.max()))
    assert res.max() < 1.01e-8

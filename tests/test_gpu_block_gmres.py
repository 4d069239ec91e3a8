"""GPU parity of block GMRES (MUDIFF_BLOCK): blocks of consecutive incidences of
an instance share one block Krylov space; every column must still equal its
dense LU solution (the oracle) to the parity bar for solutions, 1e-10, at
tol 1e-12, whatever the block size (full, ragged, one column), the operator
path (one-lane, MFMA, circulant form), the initial guess, the preconditioner
or the incidence (plane waves, point sources).  Also: graph replays equal the
eager solve bit for bit, repeated incidences inside a block (a rank-deficient
block) are dropped from the basis without harm, the per-step residual
estimates never increase within a cycle, and maxit ends a solve with flag 1.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import operator, pointsource as ps, rhs, solve

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


def _cluster(seed, M):
    return synth.small_random(seed, M, 0.3, 1.0, 9.0, 0.15, 6.0, 4)


def _lu(cl, betas):
    L = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    U = rhs.planewave(cl.centers, cl.radii, cl.n_modes, cl.k, betas)
    return solve.efie_solve_lu(L, U)


def _check(pr, cls, betas, rho, flag, R, bar=1e-10):
    assert torch.all(flag == 0), flag
    for b, (c, Y) in enumerate(zip(cls, pr.split(rho, R))):
        e = rel(Y.cpu().numpy(), _lu(c, betas[b]))
        assert e < bar, (b, e)


@pytest.mark.parametrize("block", [8, 3, 1])
def test_block_gmres_matches_lu(P, block):
    """Two instances x 8 incidences through the MFMA apply: one block of 8,
    blocks 3 + 3 + 2, and blocks of one column (plain GMRES per column)."""
    cls = [_cluster(90 + i, M=6 + 2 * i) for i in range(2)]
    R = 8
    betas = np.stack([synth.uniform_angles(R), synth.uniform_angles(R) + 0.1])
    say("block gmres, block", block)
    pr = P.from_clusters(cls)
    rho, flag, relres, iters, resvec = pr.gmres(betas=betas, restart=30, tol=1e-12, maxit=3000,
                                                block=block, want_resvec=True)
    it = iters.cpu().numpy()
    say("  iterations", it.tolist())
    _check(pr, cls, betas, rho, flag, R)
    assert torch.all(relres <= 1e-12)
    # estimates never increase inside the first cycle (minimisation over a
    # growing space), and the first one is 1 (x0 = 0)
    rv = resvec.cpu().numpy()
    for c in range(rv.shape[0]):
        n = min(int(it[c]), 30)
        e = rv[c, :n + 1]
        assert abs(e[0] - 1.0) < 1e-12
        assert np.all(np.diff(e) <= 1e-12 * e[:-1] + 1e-15), (c, e)
    # within one cycle a column's residual over the block space is at most its
    # residual over its own Krylov space: the full block needs no more steps
    _, flag1, _, it1, _ = pr.gmres(betas=betas, restart=30, tol=1e-12, maxit=3000)
    assert torch.all(flag1 == 0)
    say("  lockstep iterations", it1.cpu().numpy().tolist())
    if block == 8:
        assert it.max() <= it1.cpu().numpy().max()


def test_block_gmres_one_lane_path_and_options(P):
    """Uniform orders at R < 8 (the one-lane apply), with an initial guess,
    without the preconditioner, and from point sources."""
    cl = synth.small_random(33, 7, 0.5, 0.5, 8.0, 0.3, 5.0, 0)
    cl = synth.Cluster(cl.centers, cl.radii, np.full(cl.M, 7, np.int32), cl.k)
    R = 3
    betas = np.array([[0.2, 1.4, 3.0]])
    pr = P.from_cluster(cl)
    say("block gmres, one-lane path")
    rho, flag, _, iters, _ = pr.gmres(betas=betas, restart=20, tol=1e-12, maxit=2000, block=3)
    _check(pr, [cl], betas, rho, flag, R)
    # from the solution: no step
    rho2, flag2, _, it2, _ = pr.gmres(betas=betas, restart=20, tol=1e-10, maxit=2000, block=3,
                                      x0=rho)
    assert torch.all(flag2 == 0) and torch.all(it2 == 0)
    # without the preconditioner
    rho3, flag3, _, _, _ = pr.gmres(betas=betas, restart=20, tol=1e-12, maxit=4000, block=3,
                                    precond=False)
    _check(pr, [cl], betas, rho3, flag3, R)
    # point sources outside the cluster
    src = np.array([[[-6.0, -5.0], [25.0, 3.0], [4.0, 30.0]]])
    rho4, flag4, _, _, _ = pr.gmres(sources=src, restart=20, tol=1e-12, maxit=2000, block=2)
    assert torch.all(flag4 == 0)
    L = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    U = ps.point_source(cl.centers, cl.radii, cl.n_modes, cl.k, src[0])
    ref = np.linalg.solve(L, -U.T).T
    assert rel(pr.split(rho4, R)[0].cpu().numpy(), ref) < 1e-10


def test_block_gmres_circulant_graph_and_repeated_columns(P):
    """The circulant form at R = 13 (blocks 7 + 6), graph replays equal to the
    eager solve, and a block holding the same incidence three times."""
    cls = [synth.small_random(501, 30, 0.3, 1.0, 3.6 * math.sqrt(30), 0.1, 6.0, 4),
           synth.small_random(502, 18, 0.2, 0.8, 16.0, 0.1, 9.0, 3)]
    R = 13
    betas = np.stack([synth.uniform_angles(R), synth.uniform_angles(R) + 0.05])
    betas[1, 3] = betas[1, 2]
    betas[1, 4] = betas[1, 2]
    pr = P.from_clusters(cls, circulant=True)
    pr.set_circulant(R, 1)
    say("block gmres, circulant form")
    rho, flag, _, iters, _ = pr.gmres(betas=betas, restart=25, tol=1e-12, maxit=3000, block=7)
    assert pr.apply_config(R)["kind"] == "circulant"
    say("  iterations", iters.cpu().numpy().tolist())
    _check(pr, cls, betas, rho, flag, R)
    Y = pr.split(rho, R)[1].cpu().numpy()
    assert rel(Y[3], Y[2]) < 1e-10 and rel(Y[4], Y[2]) < 1e-10
    for rep in range(3):
        rho_g, flag_g, _, it_g, _ = pr.gmres(betas=betas, restart=25, tol=1e-12, maxit=3000,
                                             block=7, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(it_g, iters) and torch.equal(flag_g, flag), rep
        assert torch.equal(rho_g, rho), rep


def test_block_gmres_maxit_and_invalid_sizes(P):
    cl = _cluster(90, 6)
    pr = P.from_cluster(cl)
    betas = synth.uniform_angles(4)[None, :]
    _, flag, relres, iters, _ = pr.gmres(betas=betas, restart=30, tol=1e-14, maxit=3, block=4)
    assert torch.all(flag == 1) and torch.all(iters == 3) and torch.all(relres > 1e-14)
    from paper_1409_8186_amd import _lib
    with pytest.raises(_lib.MudiffError):  # block size above 16
        pr.gmres(betas=betas, restart=30, tol=1e-8, maxit=10, block=17)
    with pytest.raises(_lib.MudiffError):  # restart * block size above 2048
        pr.gmres(betas=synth.uniform_angles(8)[None, :], restart=512, tol=1e-8, maxit=10, block=8)

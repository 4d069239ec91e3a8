"""GPU parity of the transposed single-layer apply (L^T = P L P, P the mode
flip m -> -m) and of GMRES without the single-scattering preconditioner (sec. 5
system L rho = -U itself), against the CPU oracle through the C ABI.

Tolerances: applies 1e-12 (norm-wise); solves at tol 1e-13: 1e-10."""
import numpy as np
import pytest
import torch

import synth
from oracle import operator, operators as ops, rhs, solve

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.fixture(scope="module")
def P():
    from paper_1409_8186_amd import Problem
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return Problem


CLUSTERS = {
    "uniform": lambda: synth.Cluster(*synth.random_disks(np.random.default_rng(121), 9, 0.3, 0.7, 0.0, 7.0, 0.3),
                                     np.full(9, 8, np.int32), 3.5),
    "uneven": lambda: synth.small_random(122, 7, 0.3, 0.9, 7.0, 0.3, 4.0, 4),
}


@pytest.mark.parametrize("cname", ["uniform", "uneven"])
@pytest.mark.parametrize("R", [1, 9])
def test_transposed_apply_matches_oracle(P, cname, R):
    from paper_1409_8186_amd import _lib as L
    cl = CLUSTERS[cname]()
    Lm = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    rng = np.random.default_rng(R + 5)
    x = rng.standard_normal((R, Lm.shape[0])) + 1j * rng.standard_normal((R, Lm.shape[0]))
    pr = P.from_cluster(cl)
    y = pr.matvec(torch.tensor(x.reshape(-1), device="cuda"), R=R, op=L.OP_LT).cpu().numpy().reshape(R, -1)
    assert rel(y, x @ Lm) < 1e-12          # (L^T x^T)^T = x L
    pr.set_operator("mfie")
    with pytest.raises(L.MudiffError):
        pr.matvec(torch.tensor(x.reshape(-1), device="cuda"), R=R, op=L.OP_LT)


@pytest.mark.parametrize("R", [1, 9])
def test_gmres_without_preconditioner(P, R):
    """L rho = -U without D^{-1}: the same solution as LU, more iterations than
    the preconditioned solve; also from a given right-hand side and for the
    MFIE operator tables."""
    cl = CLUSTERS["uniform"]()
    betas = 2 * np.pi * np.arange(R) / R
    Lm = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    U = rhs.planewave(cl.centers, cl.radii, cl.n_modes, cl.k, betas)
    ref = solve.efie_solve_lu(Lm, U)
    pr = P.from_cluster(cl)
    r0, f0, _, it0, _ = pr.gmres(betas=[betas], restart=30, tol=1e-13, maxit=3000)
    r1, f1, res1, it1, _ = pr.gmres(betas=[betas], restart=30, tol=1e-13, maxit=3000, precond=False)
    assert np.all(f1.cpu().numpy() == 0) and np.all(res1.cpu().numpy() <= 1e-13)
    assert rel(r1.cpu().numpy().reshape(R, -1), ref) < 1e-10
    assert int(it1.max()) >= int(it0.max())
    r2, f2, _, _, _ = pr.gmres(rhs=torch.tensor(U.reshape(-1), device="cuda"), R=R, restart=30, tol=1e-13,
                               maxit=3000, precond=False)
    assert rel(r2.cpu().numpy().reshape(R, -1), ref) < 1e-10
    A = ops.combination({"I": 0.5, "N": 1.0}, cl.centers, cl.radii, cl.n_modes, cl.k)
    dU = ops.planewave_dn(cl.centers, cl.radii, cl.n_modes, cl.k, betas)
    pr.set_operator("mfie")
    r3, f3, _, _, _ = pr.gmres(betas=[betas], restart=30, tol=1e-13, maxit=3000, precond=False)
    assert rel(r3.cpu().numpy().reshape(R, -1), np.linalg.solve(A, -dU.T).T) < 1e-10

"""GPU parity of the operators M, N, D and the formulations built from them
(EFIE, MFIE, CFIE, Brakhage-Werner for a sound-soft boundary; single- and
double-layer equations for a sound-hard one) against the CPU oracle, through
the C ABI via the binding.

Tolerances: operator applies 1e-12 (norm-wise, as for the single layer);
far fields of solves at tol 1e-12: 1e-10; single-disk far fields against the
textbook Mie series: 1e-10.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import operators as ops

pytestmark = pytest.mark.gpu

FORMS = [("efie", False), ("mfie", False), ("cfie", False), ("bwie", False),
         ("neumann_sl", True), ("neumann_dl", True)]


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def P():
    from paper_1409_8186_amd import Problem
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return Problem


def _oracle_weights(name, k):
    return ops.formulation(name, alpha=0.5, eta=1j * k, k=k)


def _dense(cl, w):
    return ops.combination(w, cl.centers, cl.radii, cl.n_modes, cl.k)


CLUSTERS = {
    # uniform N <= 12: one-lane kernel for R = 1, MFMA for R >= 8
    "uniform": lambda: synth.Cluster(*synth.random_disks(np.random.default_rng(41), 9, 0.3, 0.7, 0.0, 7.0, 0.3),
                                     np.full(9, 8, np.int32), 3.5),
    # uneven N: generic kernel for R = 1
    "uneven": lambda: synth.small_random(42, 7, 0.3, 0.9, 7.0, 0.3, 4.0, 4),
}


@pytest.mark.parametrize("cname", ["uniform", "uneven"])
@pytest.mark.parametrize("R", [1, 9])
def test_operator_applies_match_oracle(P, cname, R):
    """op x and D^{-1} op x for every formulation's operator, on the one-lane,
    generic and MFMA kernels."""
    cl = CLUSTERS[cname]()
    pr = P.from_cluster(cl)
    rng = np.random.default_rng(7)
    X = rng.standard_normal((R, cl.n_tot)) + 1j * rng.standard_normal((R, cl.n_tot))
    xd = torch.tensor(X.reshape(-1), device="cuda")
    for name, _ in FORMS:
        say("apply", cname, "R", R, name, pr.apply_config(R)["kind"])
        w, _, _ = _oracle_weights(name, cl.k)
        A = _dense(cl, w)
        D = np.diag(A).copy()
        pr.set_operator(name)
        Y = pr.matvec(xd, R=R, op=0).cpu().numpy().reshape(R, -1)
        YA = pr.matvec(xd, R=R, op=1).cpu().numpy().reshape(R, -1)
        for r in range(R):
            assert rel(Y[r], A @ X[r]) < 1e-12, (name, r)
            assert rel(YA[r], (A @ X[r]) / D) < 1e-12, (name, r)
    pr.set_operator(None)


@pytest.mark.parametrize("name,hard", FORMS)
def test_formulation_solves_match_oracle(P, name, hard):
    """Preconditioned GMRES on each formulation (incidence-built right-hand
    side, far field with the formulation's weights) against the dense oracle
    solve, for R = 1 and R = 9 incidences."""
    cl = synth.small_random(43, 6, 0.3, 0.9, 7.0, 0.3, 4.0, 5)
    th = synth.uniform_angles(32)
    for R in (1, 9):
        betas = synth.uniform_angles(R) + 0.3
        say("solve", name, "R", R)
        pr = P.from_cluster(cl)
        pr.set_operator(name)
        rho, flag, relres, iters, _ = pr.gmres(betas=betas[None, :], restart=40, tol=1e-13, maxit=4000)
        assert int(flag.max()) == 0
        a = pr.farfield(rho, th, R=R).cpu().numpy()
        dens, a_ref = ops.solve_farfield(name, cl.centers, cl.radii, cl.n_modes, cl.k, betas, th,
                                         alpha=0.5, eta=1j * cl.k)
        assert rel(rho.cpu().numpy().reshape(R, -1), dens) < 1e-10
        assert rel(a, a_ref) < 1e-10


def _mie(center, a, k, beta, thetas, N, hard):
    from scipy import special as sp
    m = np.arange(-N, N + 1)
    ratio = (sp.jvp(m, k * a) / sp.h1vp(m, k * a)) if hard else (sp.jv(m, k * a) / sp.hankel1(m, k * a))
    O = np.asarray(center)
    ph = np.exp(1j * k * ((np.cos(beta) - np.cos(thetas)) * O[0] + (np.sin(beta) - np.sin(thetas)) * O[1]))
    s = np.sum(ratio[None, :] * np.exp(1j * m[None, :] * (thetas[:, None] - beta)), axis=1)
    return -np.exp(-0.25j * np.pi) * np.sqrt(2.0 / (np.pi * k)) * ph * s


@pytest.mark.parametrize("name,hard", FORMS)
def test_formulation_single_disk_mie(P, name, hard):
    c, a, k, N, beta = (0.7, -0.4), 0.9, 4.0, 14, 0.6
    cl = synth.Cluster(np.array([c]), np.array([a]), np.array([N], np.int32), k)
    pr = P.from_cluster(cl)
    pr.set_operator(name)
    rho, flag, _, _, _ = pr.gmres(betas=[[beta]], restart=20, tol=1e-14, maxit=200)
    th = synth.uniform_angles(40)
    af = pr.farfield(rho, th).cpu().numpy()[0]
    assert rel(af, _mie(c, a, k, beta, th, N, hard)) < 1e-10


def test_reset_restores_the_single_layer_bits(P):
    """Setting a formulation and returning to the built-in single layer gives
    the single-layer results bit for bit (solve and apply)."""
    cl = synth.small_random(44, 5, 0.3, 0.9, 6.0, 0.3, 4.0, 4)
    pr = P.from_cluster(cl)
    x = torch.randn(cl.n_tot, dtype=torch.complex128, device="cuda")
    y0 = pr.matvec(x, op=1).clone()
    rho0 = pr.gmres(betas=[[0.2]], restart=30, tol=1e-12, maxit=500)[0].clone()
    pr.set_operator("bwie")
    pr.matvec(x, op=1)
    pr.set_operator(None)
    assert torch.equal(pr.matvec(x, op=1), y0)
    assert torch.equal(pr.gmres(betas=[[0.2]], restart=30, tol=1e-12, maxit=500)[0], rho0)


def test_invalid_combination_and_gradient_guard(P):
    from paper_1409_8186_amd import MudiffError
    cl = synth.small_random(45, 4, 0.3, 0.9, 6.0, 0.3, 4.0, 3)
    pr = P.from_cluster(cl)
    with pytest.raises(MudiffError):
        pr.set_operator(ops={"L": 1.0, "D": 1.0}, rhs={"U": -1.0}, far={"L": 1.0})
    pr.set_operator("mfie")
    th = synth.uniform_angles(8)
    with pytest.raises(MudiffError):
        pr.grad([[0.1]], th, np.zeros(8, np.complex128), restart=20, tol=1e-10, maxit=200)

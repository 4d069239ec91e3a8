"""GPU parity: every step of the HIP path against the CPU oracle, element by
element, on the same seeded inputs (through the C ABI via the binding).

Tolerances (relative, norm-wise per column unless stated):
  * tables: componentwise |t - t_ref| <= 1e-11 |t_ref| (AMOS itself is good
    to ~1e-13 relative to |H|; arguments up to ~2e3 move the phase by x*eps);
  * operator apply: 1e-12 (a sum of N_tot products of O(1) terms in FP64);
  * right-hand side, far field of a given density: 1e-13;
  * solutions / far fields of solves at tol 1e-12: 1e-10 (the parity bar for solutions).
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import bessel, farfield, geometry, operator, rhs, solve

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def P():
    from paper_1409_8186_amd import Problem
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return Problem


def _uneven(seed=21, M=9):
    return synth.small_random(seed, M, 0.3, 1.0, 9.0, 0.15, 6.0, 4)


def _wide():
    """Pairs spanning small and large k b, uneven N_p up to 30."""
    centers = np.array([[0.0, 0.0], [0.9, 0.1], [40.0, 3.0], [-120.0, 250.0], [2.3, -0.4]])
    radii = np.array([0.3, 0.5, 1.5, 0.7, 0.2])
    n_modes = np.array([3, 6, 30, 12, 1])
    return synth.Cluster(centers, radii, n_modes, 4.7)


# ------------------------------------------------------------------ tables
@pytest.mark.parametrize("name", ["tiny", "uneven", "wide"])
def test_tables(P, tiny, name):
    cl = {"tiny": tiny, "uneven": _uneven(), "wide": _wide()}[name]
    say("tables", name)
    pr = P.from_cluster(cl)
    J, H = pr.disk_tables()
    J, H = J.cpu().numpy(), H.cpu().numpy()
    o = 0
    for p in range(cl.M):
        m = np.arange(cl.n_modes[p] + 2)
        x = cl.k * cl.radii[p]
        Jr = bessel.besselj(m, x)
        Hr = bessel.hankel1(m, x)
        assert np.all(np.abs(J[o:o + len(m)] - Jr) <= 1e-13 * np.abs(Hr) + 1e-300), (p, J[o:o + len(m)], Jr)
        assert np.all(np.abs(H[o:o + len(m)] - Hr) <= 1e-12 * np.abs(Hr)), p
        o += len(m)
    t = pr.pair_tables().cpu().numpy()
    b, al = geometry.pair_geometry(cl.centers)
    o = 0
    worst = 0.0
    for p in range(cl.M):
        for q in range(p + 1, cl.M):
            S = cl.n_modes[p] + cl.n_modes[q]
            s = np.arange(-S, S + 1)
            ref = bessel.hankel1(s, cl.k * b[p, q]) * np.exp(1j * s * al[p, q])
            err = np.abs(t[o:o + 2 * S + 1] - ref) / np.abs(ref)
            worst = max(worst, float(err.max()))
            o += 2 * S + 1
    say("  worst symbol rel err", worst)
    assert o == t.shape[0]
    assert worst < 1e-11


# ------------------------------------------------------------------ operator
def _dense(cl):
    L = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    D = operator.efie_diagonal(cl.radii, cl.n_modes, cl.k)
    return L, operator.preconditioned(L, D)


@pytest.mark.parametrize("name,R", [("tiny", 1), ("uneven", 1), ("uneven", 3), ("wide", 2)])
def test_matvec(P, tiny, name, R):
    cl = {"tiny": tiny, "uneven": _uneven(), "wide": _wide()}[name]
    say("matvec", name, "R", R)
    L, A = _dense(cl)
    rng = np.random.default_rng(5)
    X = rng.normal(size=(R, cl.n_tot)) + 1j * rng.normal(size=(R, cl.n_tot))
    pr = P.from_cluster(cl)
    x = torch.tensor(X.ravel(), device="cuda")
    yA = pr.matvec(x, R=R, op=1).cpu().numpy().reshape(R, -1)
    yL = pr.matvec(x, R=R, op=0).cpu().numpy().reshape(R, -1)
    for r in range(R):
        assert rel(yA[r], A @ X[r]) < 1e-12, (r, rel(yA[r], A @ X[r]))
        assert rel(yL[r], L @ X[r]) < 1e-12


def test_matvec_batched_instances(P):
    """B uneven instances in one handle: each column equals its own dense apply."""
    cls = [_uneven(30 + i, M=3 + 2 * i) for i in range(4)]
    say("matvec batched B=4")
    pr = P.from_clusters(cls)
    R = 2
    rng = np.random.default_rng(9)
    Xs = [rng.normal(size=(R, c.n_tot)) + 1j * rng.normal(size=(R, c.n_tot)) for c in cls]
    y = pr.matvec(pr.pack(Xs), R=R, op=1)
    for c, X, Y in zip(cls, Xs, pr.split(y, R)):
        _, A = _dense(c)
        Y = Y.cpu().numpy()
        for r in range(R):
            assert rel(Y[r], A @ X[r]) < 1e-12


@pytest.mark.parametrize("N", [1, 5, 8, 12])
def test_matvec_uniform_n_batches(P, N):
    """Uniform-N batches (the one-lane-per-pair path): instances of M = 2, 65
    and 130 disks (ragged 64-pair chunks, several waves per row), R = 1 and 3;
    close and distant pairs (k b from ~2 to ~200)."""
    cls = [synth.Cluster(*synth.random_disks(np.random.default_rng(60 + M), M, 0.4, 0.6, 0.0,
                                             4.0 * math.sqrt(M), 0.15),
                         np.full(M, N), 5.0) for M in (2, 65, 130)]
    say("matvec uniform N", N)
    pr = P.from_clusters(cls)
    rng = np.random.default_rng(70 + N)
    for R in (1, 3):
        Xs = [rng.normal(size=(R, c.n_tot)) + 1j * rng.normal(size=(R, c.n_tot)) for c in cls]
        for op in (0, 1):
            y = pr.matvec(pr.pack(Xs), R=R, op=op)
            for c, X, Y in zip(cls, Xs, pr.split(y, R)):
                L, A = _dense(c)
                Mref = A if op == 1 else L
                Y = Y.cpu().numpy()
                for r in range(R):
                    assert rel(Y[r], Mref @ X[r]) < 1e-12, (c.M, R, op, r)


def test_matvec_single_disk_and_repeat(P):
    """M = 1 (no pairs): A = I exactly; repeated applies give identical bits."""
    cl = synth.Cluster(np.array([[0.5, -1.0]]), np.array([0.8]), np.array([7]), 3.0)
    say("matvec M=1")
    pr = P.from_cluster(cl)
    x = torch.randn(cl.n_tot, dtype=torch.complex128, device="cuda")
    y = pr.matvec(x, op=1)
    assert torch.equal(y, x)
    cl2 = _uneven()
    pr2 = P.from_cluster(cl2)
    x2 = torch.randn(cl2.n_tot, dtype=torch.complex128, device="cuda")
    a = pr2.matvec(x2, op=1).clone()
    b = pr2.matvec(x2, op=1)
    assert torch.equal(a, b)


# ------------------------------------------------------------------ rhs
def test_rhs(P, tiny):
    cl = _uneven()
    say("rhs")
    pr = P.from_cluster(cl)
    betas = np.array([0.0, 0.7, 2.9, 5.1])
    U = pr.rhs(betas[None, :]).cpu().numpy().reshape(4, -1)
    Ur = rhs.planewave(cl.centers, cl.radii, cl.n_modes, cl.k, betas)
    assert rel(U, Ur) < 1e-13
    f = pr.rhs(betas[None, :], precond=True).cpu().numpy().reshape(4, -1)
    D = operator.efie_diagonal(cl.radii, cl.n_modes, cl.k)
    assert rel(f, -Ur / D[None, :]) < 1e-13


# ------------------------------------------------------------------ solve
def _lu(cl, betas):
    L = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    U = rhs.planewave(cl.centers, cl.radii, cl.n_modes, cl.k, betas)
    return solve.efie_solve_lu(L, U)


@pytest.mark.parametrize("graph", [False, True])
def test_gmres_tiny_vs_lu(P, tiny, graph):
    say("gmres tiny graph", graph)
    pr = P.from_cluster(tiny)
    rho, flag, relres, iters, resvec = pr.gmres(betas=[[0.0]], restart=30, tol=1e-12, maxit=2000,
                                                graph=graph, want_resvec=True)
    ref = _lu(tiny, [0.0])[0]
    assert int(flag[0]) == 0 and float(relres[0]) <= 1e-12
    assert rel(rho.cpu().numpy(), ref) < 1e-10
    it = int(iters[0])
    rv = resvec[0].cpu().numpy()
    assert rv[0] == 1.0 and 0 < rv[it] <= 1e-12
    # far field at 360 angles against the oracle's LU far field
    th = synth.uniform_angles(360)
    a = pr.farfield(rho, th).cpu().numpy()[0]
    aref = farfield.farfield(tiny.centers, tiny.radii, tiny.n_modes, tiny.k, th, ref)
    assert rel(a, aref) < 1e-10


def test_gmres_lane_path_graph_replay(P):
    """Uniform N = 8 (one lane per pair, the chunk sums finished inside the
    first Gram-Schmidt kernel): graph replay gives the eager result bit for
    bit on repeated solves, and both equal LU."""
    c = synth.Cluster(*synth.random_disks(np.random.default_rng(77), 40, 0.5, 0.5, 0.0, 25.0, 0.2),
                      np.full(40, 8), 2.0 * math.pi)
    say("gmres lane path graph replay")
    pr = P.from_cluster(c)
    rho, flag, _, iters, _ = pr.gmres(betas=[[0.4]], restart=20, tol=1e-12, maxit=3000)
    assert int(flag[0]) == 0
    assert rel(rho.cpu().numpy(), _lu(c, [0.4])[0]) < 1e-10
    for rep in range(3):
        rho_g, flag_g, _, iters_g, _ = pr.gmres(betas=[[0.4]], restart=20, tol=1e-12, maxit=3000,
                                                graph=True)
        torch.cuda.synchronize()
        assert torch.equal(iters_g, iters) and torch.equal(rho_g, rho), rep


def test_gmres_matches_oracle_gmres_iterations(P, tiny):
    """Same restart / tolerance: the iteration counts of the oracle's MGS GMRES
    and the device CGS2 GMRES agree to within a few (orthogonalisation
    rounding differs)."""
    say("gmres iteration count")
    pr = P.from_cluster(tiny)
    _, flag, _, iters, _ = pr.gmres(betas=[[0.0]], restart=30, tol=1e-8, maxit=2000)
    L, A = _dense(tiny)
    D = operator.efie_diagonal(tiny.radii, tiny.n_modes, tiny.k)
    U = rhs.planewave(tiny.centers, tiny.radii, tiny.n_modes, tiny.k, [0.0])[0]
    _, fl, _, it_ref, _ = solve.gmres(lambda v: A @ v, -U / D, 30, 1e-8, 2000)
    assert int(flag[0]) == 0 and fl == 0
    assert abs(int(iters[0]) - it_ref) <= 3, (int(iters[0]), it_ref)


def test_gmres_long_restart_matches_oracle(P):
    """A dense low-frequency cluster (M = 150, k = 1, ~20% area fraction) where
    GMRES needs ~170 inner steps in one cycle: the residual history matches the
    oracle's step by step past 128 steps, the iteration counts agree, and the
    solution's residual under the oracle's matrix is at the tolerance."""
    c = synth.small_random(7, 150, 0.2, 1.0, 28.0, 0.05, 1.0, 8, R=1)
    say("gmres restart 300: N_tot", c.n_tot)
    pr = P.from_cluster(c)
    rho, flag, relres, iters, resvec = pr.gmres(betas=[[0.0]], restart=300, tol=1e-10,
                                                maxit=1000, want_resvec=True)
    L, A = _dense(c)
    D = operator.efie_diagonal(c.radii, c.n_modes, c.k)
    f = -rhs.planewave(c.centers, c.radii, c.n_modes, c.k, [0.0])[0] / D
    _, fl, _, it_ref, rv_ref = solve.gmres(lambda v: A @ v, f, 300, 1e-10, 1000)
    it = int(iters[0])
    say("  iterations", it, "oracle", it_ref)
    assert int(flag[0]) == 0 and fl == 0
    assert abs(it - it_ref) <= 3
    rv = resvec[0].cpu().numpy()
    n = min(it, it_ref) - 10
    assert n > 140
    # estimates agree while well above the rounding floor of the basis
    assert np.max(np.abs(rv[:n] - rv_ref[:n]) / rv_ref[:n]) < 1e-4
    x = rho.cpu().numpy().reshape(-1)
    assert np.linalg.norm(A @ x - f) / np.linalg.norm(f) < 2e-10


def test_gmres_weak_coupling_second_pass(P):
    """Six far-apart disks: A = I + K with small K, so each new Krylov direction
    cancels most of A v_j and the second Gram-Schmidt pass runs on most steps
    (8 of 12 in a CPU replay of the device algorithm).  Solution vs LU and the
    iteration count vs the oracle's MGS GMRES."""
    centers = np.array([[0, 0], [40, 3], [-35, 20], [10, -45], [60, 50], [-50, -40]], float)
    radii = np.array([0.3, 0.5, 0.4, 0.35, 0.6, 0.45])
    cl = synth.Cluster(centers, radii, np.array([4, 6, 5, 5, 7, 6]), 2.0)
    say("gmres weak coupling")
    pr = P.from_cluster(cl)
    rho, flag, relres, iters, _ = pr.gmres(betas=[[0.3]], restart=30, tol=1e-12, maxit=200)
    assert int(flag[0]) == 0 and float(relres[0]) <= 1e-12
    ref = _lu(cl, [0.3])[0]
    assert rel(rho.cpu().numpy(), ref) < 1e-10
    L, A = _dense(cl)
    D = operator.efie_diagonal(cl.radii, cl.n_modes, cl.k)
    U = rhs.planewave(cl.centers, cl.radii, cl.n_modes, cl.k, [0.3])[0]
    _, fl, _, it_ref, _ = solve.gmres(lambda v: A @ v, -U / D, 30, 1e-12, 200)
    assert fl == 0 and abs(int(iters[0]) - it_ref) <= 2, (int(iters[0]), it_ref)


@pytest.mark.parametrize("B,R", [(64, 1), (32, 8)])
def test_gmres_straggler_phase(P, B, R):
    """Many easy instances and one hard one (≈10 against ≈265 GMRES(10) steps):
    once at most 1/32 of the columns still run, the Gram-Schmidt kernels run
    over their chunks only and the MFMA apply (R = 8) over their tiles with
    short column segments.  Every column must still equal LU."""
    easy = [synth.small_random(300 + i, 4, 0.3, 0.5, 60.0, 5.0, 2.0, 3) for i in range(B - 1)]
    hard = synth.small_random(201, 14, 0.6, 0.9, 9.0, 0.05, 1.5, 5)
    cls = easy[:B // 2] + [hard] + easy[B // 2:]
    betas = np.tile(synth.uniform_angles(R), (B, 1))
    say("gmres straggler phase B", B, "R", R)
    pr = P.from_clusters(cls)
    rho, flag, relres, iters, _ = pr.gmres(betas=betas, restart=10, tol=1e-12, maxit=3000)
    it = iters.cpu().numpy().reshape(B, R)
    say("  iterations easy max", int(np.delete(it, B // 2, axis=0).max()), "hard", it[B // 2].tolist())
    assert torch.all(flag == 0)
    assert it[B // 2].min() > 20 * np.delete(it, B // 2, axis=0).max() // 2
    for c, b, Y in zip(cls, betas, pr.split(rho, R)):
        assert rel(Y.cpu().numpy(), _lu(c, b)) < 1e-10


def test_gmres_batched_lockstep(P):
    """B = 3 uneven instances x R = 3 angles in one solve; every column equals LU."""
    cls = [_uneven(40 + i, M=4 + 3 * i) for i in range(3)]
    betas = np.array([[0.0, 1.0, 2.5], [0.3, 3.3, 6.0], [1.1, 1.2, 1.3]])
    say("gmres batched")
    pr = P.from_clusters(cls)
    rho, flag, relres, iters, _ = pr.gmres(betas=betas, restart=20, tol=1e-12, maxit=3000)
    assert torch.all(flag == 0), flag
    for b, (c, R) in enumerate(zip(cls, pr.split(rho, 3))):
        ref = _lu(c, betas[b])
        assert rel(R.cpu().numpy(), ref) < 1e-10


def test_gmres_flags_and_warm_start(P, tiny):
    say("gmres maxit / x0")
    pr = P.from_cluster(tiny)
    _, flag, relres, iters, _ = pr.gmres(betas=[[0.0]], restart=30, tol=1e-12, maxit=3)
    assert int(flag[0]) == 1 and int(iters[0]) == 3 and float(relres[0]) > 1e-12
    ref = _lu(tiny, [0.0])[0]
    x0 = torch.tensor(ref, device="cuda")
    rho, flag, relres, iters, _ = pr.gmres(betas=[[0.0]], restart=30, tol=1e-8, maxit=100, x0=x0)
    assert int(flag[0]) == 0 and int(iters[0]) == 0


def test_gmres_general_rhs(P):
    """rhs given instead of angles: solves L rho = -rhs."""
    cl = _uneven()
    say("gmres rhs")
    pr = P.from_cluster(cl)
    rng = np.random.default_rng(3)
    U = rng.normal(size=cl.n_tot) + 1j * rng.normal(size=cl.n_tot)
    rho, flag, _, _, _ = pr.gmres(rhs=torch.tensor(U, device="cuda"), R=1, restart=30, tol=1e-12,
                                  maxit=3000)
    L = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    assert int(flag[0]) == 0
    assert rel(rho.cpu().numpy(), np.linalg.solve(L, -U)) < 1e-10


def test_farfield_given_density(P):
    cl = _uneven()
    say("farfield")
    pr = P.from_cluster(cl)
    rng = np.random.default_rng(4)
    R = 2
    X = rng.normal(size=(R, cl.n_tot)) + 1j * rng.normal(size=(R, cl.n_tot))
    th = np.linspace(0, 2 * np.pi, 97)
    a = pr.farfield(torch.tensor(X.ravel(), device="cuda"), th, R=R).cpu().numpy()
    aref = farfield.farfield(cl.centers, cl.radii, cl.n_modes, cl.k, th, X)
    assert rel(a, aref) < 1e-13


# ------------------------------------------------------------------ full size
def test_one_rhs_full_size(P):
    """M = 400, N_p = 12 (10,000 unknowns): apply on random x vs the dense
    oracle, GMRES(50) at tol 1e-12 vs LU, far field at 720 angles."""
    cl = synth.one_rhs()
    say("one_rhs full size: assembling the dense oracle")
    L = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    D = operator.efie_diagonal(cl.radii, cl.n_modes, cl.k)
    pr = P.from_cluster(cl)
    rng = np.random.default_rng(8)
    X = rng.normal(size=cl.n_tot) + 1j * rng.normal(size=cl.n_tot)
    y = pr.matvec(torch.tensor(X, device="cuda"), op=1).cpu().numpy()
    assert rel(y, X + (L @ X - D * X) / D) < 1e-12
    say("one_rhs: gmres tol 1e-12")
    rho, flag, relres, iters, _ = pr.gmres(betas=[[math.pi / 4]], restart=50, tol=1e-12, maxit=20000)
    say("  iters", int(iters[0]), "relres", float(relres[0]))
    assert int(flag[0]) == 0
    U = rhs.planewave(cl.centers, cl.radii, cl.n_modes, cl.k, [math.pi / 4])[0]
    say("one_rhs: LU")
    ref = solve.solve_lu(L, -U)
    assert rel(rho.cpu().numpy(), ref) < 1e-10
    a = pr.farfield(rho, cl.thetas).cpu().numpy()[0]
    aref = farfield.farfield(cl.centers, cl.radii, cl.n_modes, cl.k, cl.thetas, ref)
    assert rel(a, aref) < 1e-10


# ------------------------------------------------------------------ multi-RHS (MFMA path)
@pytest.mark.parametrize("R", [8, 19, 40])
def test_matvec_multi_rhs(P, R):
    """R >= 8 runs the FP64-MFMA kernel; ragged R exercises partial tiles."""
    cls = [_uneven(80 + i, M=4 + 3 * i) for i in range(3)]
    say("matvec multi-RHS R", R)
    pr = P.from_clusters(cls)
    rng = np.random.default_rng(R)
    Xs = [rng.normal(size=(R, c.n_tot)) + 1j * rng.normal(size=(R, c.n_tot)) for c in cls]
    x = pr.pack(Xs)
    for op in (1, 0):
        y = pr.matvec(x, R=R, op=op)
        for c, X, Y in zip(cls, Xs, pr.split(y, R)):
            L, A = _dense(c)
            M_ = A if op == 1 else L
            assert rel(Y.cpu().numpy(), X @ M_.T) < 1e-12, (op, rel(Y.cpu().numpy(), X @ M_.T))


def _mfma_candidates(R):
    out = []
    ctmax = max(1, min(4, (R + 7) // 8))
    for waves in (4, 8):
        for ct in (1, 2, 4):
            if ct > ctmax and ct > 1:
                continue
            for qs in (0, 32):
                out.append((ct, waves // ct, qs, 64 * waves))
    return out


@pytest.mark.parametrize("R", [8, 19])
def test_matvec_every_mfma_tile(P, R):
    """Every tile the autotuner may pick, forced in turn, on uneven instances
    (non-uniform N_p from 5 to 26, so that rows need one to four 16-row tiles;
    M up to 40, so that 32-disk segments split rows; a ragged RHS count): each
    equals the dense oracle apply."""
    cls = [synth.small_random(80 + i, M, 0.3, 1.0, 3.0 * math.sqrt(M), 0.1, 8.0, 6)
           for i, M in enumerate((40, 7, 33))]
    cls.append(synth.small_random(83, 12, 0.1, 1.5, 14.0, 0.1, 12.0, 8))  # n_p from 19 to 53
    say("every MFMA tile R", R)
    pr = P.from_clusters(cls)
    rng = np.random.default_rng(90 + R)
    Xs = [rng.normal(size=(R, c.n_tot)) + 1j * rng.normal(size=(R, c.n_tot)) for c in cls]
    refs = [(_dense(c)[1] @ X.T).T for c, X in zip(cls, Xs)]
    x = pr.pack(Xs)
    for ct, rp, qs, th in _mfma_candidates(R):
        pr.set_apply_config(R, ct, rp, qs, th)
        cfg = pr.apply_config(R)
        assert (cfg["kind"], cfg["ct"], cfg["rp"], cfg["qs"], cfg["threads"]) == ("mfma", ct, rp, qs, th)
        y = pr.matvec(x, R=R, op=1)
        for Y, ref in zip(pr.split(y, R), refs):
            assert rel(Y.cpu().numpy(), ref) < 1e-12, (ct, rp, qs, th)


def test_apply_config_kinds(P, tiny):
    """The path each apply takes: one lane per pair for uniform N <= 12 and few
    RHS, the generic kernel otherwise, MFMA (autotuned on first use) for R >= 8."""
    one = synth.Cluster(np.array([[0.0, 0.0], [3.0, 0.5], [1.0, 4.0]]), np.array([0.5] * 3),
                        np.array([12] * 3), 6.0)
    assert P.from_cluster(one).apply_config(1)["kind"] == "lane"
    pr = P.from_cluster(tiny)                       # N_p = 15
    assert pr.apply_config(1)["kind"] == "generic"
    x = torch.randn(8 * tiny.n_tot, dtype=torch.complex128, device="cuda")
    pr.matvec(x, R=8, op=1)
    cfg = pr.apply_config(8)
    assert cfg["kind"] == "mfma" and cfg["tuned_ms"] > 0.0


def test_gmres_multi_rhs_lockstep(P):
    """8 incidences x 2 instances: the MFMA apply inside lockstep GMRES; every
    column equals its LU solution."""
    cls = [_uneven(90 + i, M=6 + 2 * i) for i in range(2)]
    betas = np.stack([synth.uniform_angles(8), synth.uniform_angles(8) + 0.1])
    say("gmres multi-RHS")
    pr = P.from_clusters(cls)
    rho, flag, relres, iters, _ = pr.gmres(betas=betas, restart=30, tol=1e-12, maxit=3000)
    assert torch.all(flag == 0), flag
    for b, (c, Rv) in enumerate(zip(cls, pr.split(rho, 8))):
        assert rel(Rv.cpu().numpy(), _lu(c, betas[b])) < 1e-10
    # restart cycles replayed as HIP graphs (persistent MFMA queue, its counter
    # reset and the finishing pass inside the graph): identical results, on
    # repeated solves with host work in between
    for rep in range(3):
        rho_g, flag_g, relres_g, iters_g, _ = pr.gmres(betas=betas, restart=30, tol=1e-12,
                                                       maxit=3000, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(iters_g, iters) and torch.equal(flag_g, flag), rep
        assert torch.equal(rho_g, rho), rep

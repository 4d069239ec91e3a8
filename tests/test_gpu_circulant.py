"""GPU parity of the circulant-embedded form of the well-separated blocks
(MUDIFF_TABLES_CIRCULANT; the FFT Toeplitz products of the paper's sec. 5)
against the dense CPU oracle, element by element, on seeded clusters whose
pairs straddle the gate k b_pq = N_p + N_q (close pairs stay in the direct
form).  The bar is the operator apply's: 1e-12 relative per column; solves at
tol 1e-12 against LU: 1e-10.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import geometry, operator, rhs, solve

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


def _dense(cl):
    L = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    D = operator.efie_diagonal(cl.radii, cl.n_modes, cl.k)
    return L, operator.preconditioned(L, D)


def _near_pairs(cl):
    """Ordered pairs below the gate, counted from the geometry alone."""
    b, _ = geometry.pair_geometry(cl.centers)
    S = cl.n_modes[:, None] + cl.n_modes[None, :]
    near = cl.k * b < S
    np.fill_diagonal(near, False)
    return int(near.sum())


def _mixed(seed, M=30):
    """Radii 0.3..1, k = 6, N_p = ceil(k a_p) + 4 (7..10): about one pair in
    ten below the gate."""
    return synth.small_random(seed, M, 0.3, 1.0, 3.6 * math.sqrt(M), 0.1, 6.0, 4)


def _embed_len(n_modes):
    """Embedding length the tables pick: L_min = 2 (N' + N'') + 1 over the two
    largest orders, raised to the shortest 2^i 3^j >= L_min when that is at most
    128 and at most 1.2 L_min (fast transforms), else L_min itself."""
    n = np.sort(np.asarray(n_modes))[::-1]
    lmin = 2 * (int(n[0]) + int(n[1])) + 1
    smooth = min(2 ** i * 3 ** j for i in range(9) for j in range(6) if 2 ** i * 3 ** j >= lmin)
    return smooth if smooth <= 128 and 5 * smooth <= 6 * lmin else lmin


def _batch():
    """A mixed instance, a dense low-frequency one (mostly close pairs: it stays
    in the direct form), another mixed one with other orders, and one disk."""
    one = synth.Cluster(np.array([[0.5, -0.2]]), np.array([0.7]), np.array([6]), 6.0)
    low = synth.small_random(505, 10, 0.5, 0.9, 6.0, 0.1, 1.0, 6)
    return [_mixed(501), low, synth.small_random(502, 18, 0.2, 0.8, 16.0, 0.1, 9.0, 3), one]


def test_circulant_classification(P):
    cls = _batch()
    pr = P.from_clusters(cls, circulant=True)
    info = pr.circulant_info()
    near = sum(_near_pairs(c) for c in cls)
    total = sum(c.M * (c.M - 1) for c in cls)
    say("circulant info", info, "near (host count)", near, "of", total)
    assert info["near_pairs"] == near and info["far_pairs"] == total - near
    assert 0 < near < total
    Ns = [np.sort(c.n_modes)[::-1] for c in cls if c.M > 1]
    assert info["L_max"] == max(_embed_len(c.n_modes) for c in cls if c.M > 1)
    assert P.from_clusters(cls).circulant_info() == {"far_pairs": 0, "near_pairs": 0, "L_max": 0}


@pytest.mark.parametrize("R", [8, 13, 32, 40, 64])
def test_circulant_matvec(P, R):
    """Every product tile of the per-frequency step (R picks it: 8, 16, 32 or
    64 columns) with ragged column counts, on instances in and out of the form,
    for A = D^-1 L, L and L^T."""
    cls = _batch()
    say("circulant matvec R", R)
    pr = P.from_clusters(cls, circulant=True)
    pr.set_circulant(R, 1)
    rng = np.random.default_rng(700 + R)
    Xs = [rng.normal(size=(R, c.n_tot)) + 1j * rng.normal(size=(R, c.n_tot)) for c in cls]
    x = pr.pack(Xs)
    for op in (1, 0, 2):
        y = pr.matvec(x, R=R, op=op)
        assert pr.apply_config(R)["kind"] == "circulant"
        for c, X, Y in zip(cls, Xs, pr.split(y, R)):
            L, A = _dense(c)
            Mx = {1: A, 0: L, 2: L.T}[op]
            e = rel(Y.cpu().numpy(), X @ Mx.T)
            assert e < 1e-12, (op, c.M, e)
    # every per-frequency product tile the autotuner may pick for R
    for tile in pr.circulant_tiles(R):
        pr.set_circulant_tile(R, *tile)
        y = pr.matvec(x, R=R, op=1)
        assert pr.circulant_tile(R) == tile
        for c, X, Y in zip(cls, Xs, pr.split(y, R)):
            assert rel(Y.cpu().numpy(), X @ _dense(c)[1].T) < 1e-12, tile
    # the direct form on the same handle agrees
    pr.set_circulant(R, 0)
    y = pr.matvec(x, R=R, op=1)
    assert pr.apply_config(R)["kind"] == "mfma"
    for c, X, Y in zip(cls, Xs, pr.split(y, R)):
        assert rel(Y.cpu().numpy(), X @ _dense(c)[1].T) < 1e-12


def test_circulant_close_pair_lists_every_tile(P):
    """Denser clusters (13-50% of the pairs close, up to 43 close neighbours per
    group of 8 rows, so that 32-entry segments split the lists; the 9-disk one
    falls below half far work and stays direct) under every MFMA tile the
    autotuner may pick, with the circulant form on."""
    cls = [synth.small_random(510 + i, M, 0.4, 1.0, 2.2 * math.sqrt(M), 0.1, 7.0, 9)
           for i, M in enumerate((60, 9, 45))]
    R = 19
    pr = P.from_clusters(cls, circulant=True)
    info = pr.circulant_info()
    say("close-pair lists: info", info)
    rng = np.random.default_rng(77)
    Xs = [rng.normal(size=(R, c.n_tot)) + 1j * rng.normal(size=(R, c.n_tot)) for c in cls]
    refs = [X @ _dense(c)[1].T for c, X in zip(cls, Xs)]
    x = pr.pack(Xs)
    pr.set_circulant(R, 1)
    ctmax = max(1, min(4, (R + 7) // 8))
    for waves in (4, 8):
        for ct in (1, 2, 4):
            if ct > ctmax and ct > 1:
                continue
            for qs in (0, 32):
                pr.set_apply_config(R, ct, waves // ct, qs, 64 * waves)
                assert pr.apply_config(R)["kind"] == "circulant"
                y = pr.matvec(x, R=R, op=1)
                for Y, ref in zip(pr.split(y, R), refs):
                    assert rel(Y.cpu().numpy(), ref) < 1e-12, (ct, waves, qs)


def _fixed_orders(seed, M, box, k, first, rest):
    """small_random placement with order `first` on disk 3 and `rest` elsewhere."""
    c = synth.small_random(seed, M, 0.3, 0.8, box, 0.2, k, 2)
    n = np.full(c.M, rest, np.int32)
    n[3] = first
    return synth.Cluster(c.centers, c.radii, n, k)


def _fft_batch():
    """Embedding lengths of every kind in one launch: L = 27 and 81 (radix 3),
    L_min = 41 raised to 48 = 2^4 3 (radix 3 then radix 2), L_min = 37 kept
    (48 would add 30% to the products: direct sums), and an instance outside
    the form."""
    c27 = _fixed_orders(540, 24, 30.0, 6.0, 7, 6)
    c81 = synth.small_random(541, 16, 0.8, 1.0, 40.0, 0.2, 10.0, 10)
    c81 = synth.Cluster(c81.centers, c81.radii, np.full(c81.M, 20, np.int32), c81.k)
    c37 = _fixed_orders(542, 20, 32.0, 6.0, 10, 8)
    low = synth.small_random(505, 10, 0.5, 0.9, 6.0, 0.1, 1.0, 6)
    return [c27, _mixed(501), c81, c37, low]


def _wide_batch():
    """A length above 81 (L_min = 97 raised to 108 = 2^2 3^3: the launch then
    runs the transforms of both length classes, 108 in the 128-length kernels
    and 27, 48 in the 81-length ones) beside L = 27 and L = 48."""
    c108 = synth.small_random(543, 14, 0.8, 1.0, 46.0, 0.2, 9.0, 10)
    c108 = synth.Cluster(c108.centers, c108.radii, np.full(c108.M, 24, np.int32), c108.k)
    return [_fixed_orders(540, 24, 30.0, 6.0, 7, 6), c108, _mixed(503)]


@pytest.mark.parametrize("R", [8, 16, 40])
def test_circulant_fft_lengths(P, R):
    """Fast transforms of lengths 27, 81 (radix 3) and 48 (radix 3, 2) beside
    direct sums (L = 37) and an instance outside the form, in one launch: A, L
    and L^T against the dense oracle, every product tile."""
    cls = _fft_batch()
    assert [_embed_len(c.n_modes) for c in cls[:4]] == [27, 48, 81, 37]
    pr = P.from_clusters(cls, circulant=True)
    info = pr.circulant_info()
    say("fft lengths R", R, info)
    assert info["L_max"] == 81
    pr.set_circulant(R, 1)
    rng = np.random.default_rng(900 + R)
    Xs = [rng.normal(size=(R, c.n_tot)) + 1j * rng.normal(size=(R, c.n_tot)) for c in cls]
    x = pr.pack(Xs)
    dense = [_dense(c) for c in cls]
    for op in (1, 0, 2):
        y = pr.matvec(x, R=R, op=op)
        assert pr.apply_config(R)["kind"] == "circulant"
        for (L, A), X, Y in zip(dense, Xs, pr.split(y, R)):
            Mx = {1: A, 0: L, 2: L.T}[op]
            e = rel(Y.cpu().numpy(), X @ Mx.T)
            assert e < 1e-12, (op, e)
    for tile in pr.circulant_tiles(R):
        pr.set_circulant_tile(R, *tile)
        y = pr.matvec(x, R=R, op=1)
        for (_, A), X, Y in zip(dense, Xs, pr.split(y, R)):
            assert rel(Y.cpu().numpy(), X @ A.T) < 1e-12, tile


@pytest.mark.parametrize("R", [8, 19])
def test_circulant_lengths_above_81(P, R):
    """L = 108 (2^2 3^3) in a launch with L = 27 and 48: the fast transforms
    of the launch run in two length classes (up to 81, and 128); A, L and L^T
    against the dense oracle, and lockstep GMRES against LU."""
    cls = _wide_batch()
    assert [_embed_len(c.n_modes) for c in cls] == [27, 108, 48]
    pr = P.from_clusters(cls, circulant=True)
    info = pr.circulant_info()
    say("lengths above 81, R", R, info)
    assert info["L_max"] == 108 and info["far_pairs"] > 0
    pr.set_circulant(R, 1)
    rng = np.random.default_rng(960 + R)
    Xs = [rng.normal(size=(R, c.n_tot)) + 1j * rng.normal(size=(R, c.n_tot)) for c in cls]
    x = pr.pack(Xs)
    dense = [_dense(c) for c in cls]
    for op in (1, 0, 2):
        y = pr.matvec(x, R=R, op=op)
        assert pr.apply_config(R)["kind"] == "circulant"
        for (L, A), X, Y in zip(dense, Xs, pr.split(y, R)):
            Mx = {1: A, 0: L, 2: L.T}[op]
            e = rel(Y.cpu().numpy(), X @ Mx.T)
            assert e < 1e-12, (op, e)
    betas = np.stack([synth.uniform_angles(R) + 0.1 * i for i in range(len(cls))])
    rho, flag, _, iters, _ = pr.gmres(betas=betas, restart=30, tol=1e-12, maxit=3000)
    say("  gmres iterations", iters.cpu().numpy().tolist())
    assert torch.all(flag == 0)
    for b, (c, Y) in enumerate(zip(cls, pr.split(rho, R))):
        assert rel(Y.cpu().numpy(), _lu(c, betas[b])) < 1e-10


def _close_counts(cl):
    """Close neighbours of each disk (k b_pq < N_p + N_q), from the geometry."""
    b, _ = geometry.pair_geometry(cl.centers)
    near = cl.k * b < cl.n_modes[:, None] + cl.n_modes[None, :]
    np.fill_diagonal(near, False)
    return near.sum(axis=1)


def _crowded27(seed):
    """L = 27 (N_p = 6, one disk 7) with disk 0 ringed by ten close neighbours
    at distance 1.6 (k b = 9.6 < 13) and 30 disks spread far from the ring."""
    ring = [[1.6 * math.cos(2 * math.pi * j / 10), 1.6 * math.sin(2 * math.pi * j / 10)]
            for j in range(10)]
    far, fr = synth.random_disks(np.random.default_rng(seed), 30, 0.3, 0.5, 6.0, 40.0, 0.3)
    centers = np.vstack([[[0.0, 0.0]], ring, far])
    radii = np.concatenate([[0.4], np.full(10, 0.3), fr])
    n = np.full(len(radii), 6, np.int32)
    n[5] = 7
    return synth.Cluster(centers, radii, n, 6.0)


def _sparse_and_crowded_batch():
    """Two L = 27 instances: one with at most a few close neighbours per disk
    and one whose ringed disk has ten (a close-pair list longer than a row
    group's mask of 8); and an L = 81 one with a few close pairs."""
    c27 = synth.small_random(560, 30, 0.3, 0.6, 16.0, 0.2, 6.0, 2)
    n27 = np.full(c27.M, 6, np.int32)
    n27[0] = 7
    c27 = synth.Cluster(c27.centers, c27.radii, n27, 6.0)
    c81 = synth.small_random(561, 20, 0.8, 1.0, 28.0, 0.2, 10.0, 10)
    c81 = synth.Cluster(c81.centers, c81.radii, np.full(c81.M, 20, np.int32), 10.0)
    return [c27, _crowded27(562), c81]


@pytest.mark.parametrize("R", [8, 24])
def test_circulant_radix3_close_pairs(P, R):
    """Radix-3 instances with sparse and crowded close pairs beside each other
    in one launch, ragged 16-column blocks of the output pass: A, L and L^T
    against the dense oracle, every product tile, and lockstep GMRES (columns
    that stop early are skipped by the output pass) against LU."""
    cls = _sparse_and_crowded_batch()
    counts = [_close_counts(c) for c in cls]
    say("close neighbours per disk (max)", [int(c.max()) for c in counts],
        "close ordered pairs", [int(c.sum()) for c in counts])
    assert counts[0].sum() > 0 and counts[0].max() <= 8
    assert counts[1].max() > 8
    assert counts[2].sum() > 0 and counts[2].max() <= 8
    pr = P.from_clusters(cls, circulant=True)
    info = pr.circulant_info()
    assert info["L_max"] == 81 and info["near_pairs"] == sum(int(c.sum()) for c in counts)
    pr.set_circulant(R, 1)
    rng = np.random.default_rng(950 + R)
    Xs = [rng.normal(size=(R, c.n_tot)) + 1j * rng.normal(size=(R, c.n_tot)) for c in cls]
    x = pr.pack(Xs)
    dense = [_dense(c) for c in cls]
    for op in (1, 0, 2):
        y = pr.matvec(x, R=R, op=op)
        assert pr.apply_config(R)["kind"] == "circulant"
        for (L, A), X, Y in zip(dense, Xs, pr.split(y, R)):
            Mx = {1: A, 0: L, 2: L.T}[op]
            e = rel(Y.cpu().numpy(), X @ Mx.T)
            assert e < 1e-12, (op, e)
    for tile in pr.circulant_tiles(R):
        pr.set_circulant_tile(R, *tile)
        y = pr.matvec(x, R=R, op=1)
        for (_, A), X, Y in zip(dense, Xs, pr.split(y, R)):
            assert rel(Y.cpu().numpy(), X @ A.T) < 1e-12, tile
    betas = np.stack([synth.uniform_angles(R) + 0.1 * i for i in range(len(cls))])
    rho, flag, _, iters, _ = pr.gmres(betas=betas, restart=30, tol=1e-12, maxit=3000)
    say("  gmres iterations", iters.cpu().numpy().tolist())
    assert torch.all(flag == 0), flag
    assert len(set(iters.cpu().numpy().tolist())) > 1  # columns stop at different steps
    for b, (c, Y) in enumerate(zip(cls, pr.split(rho, R))):
        assert rel(Y.cpu().numpy(), _lu(c, betas[b])) < 1e-10


def _lu(cl, betas):
    L = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    U = rhs.planewave(cl.centers, cl.radii, cl.n_modes, cl.k, betas)
    return solve.efie_solve_lu(L, U)


def test_circulant_gmres_graph_and_stragglers(P):
    """Lockstep GMRES on the circulant form: every column equals LU, graph
    replays are bit-identical to the eager solve, and a batch with one hard
    instance runs its straggler phase (short close-pair segments, product
    tiles of the running columns only) to the same LU solutions."""
    cls = [_mixed(520), _mixed(521, M=22)]
    R = 8
    betas = np.stack([synth.uniform_angles(R), synth.uniform_angles(R) + 0.2])
    pr = P.from_clusters(cls, circulant=True)
    pr.set_circulant(R, 1)
    rho, flag, relres, iters, _ = pr.gmres(betas=betas, restart=30, tol=1e-12, maxit=3000)
    say("circulant gmres iterations", iters.cpu().numpy().tolist())
    assert pr.apply_config(R)["kind"] == "circulant"
    assert torch.all(flag == 0), flag
    for b, (c, Y) in enumerate(zip(cls, pr.split(rho, R))):
        assert rel(Y.cpu().numpy(), _lu(c, betas[b])) < 1e-10
    for rep in range(3):
        rho_g, flag_g, _, iters_g, _ = pr.gmres(betas=betas, restart=30, tol=1e-12, maxit=3000,
                                                graph=True)
        torch.cuda.synchronize()
        assert torch.equal(iters_g, iters) and torch.equal(flag_g, flag) and torch.equal(rho_g, rho), rep
    B = 32
    easy = [synth.small_random(300 + i, 4, 0.3, 0.5, 60.0, 5.0, 2.0, 3) for i in range(B - 1)]
    hard = _mixed(530, M=26)
    allc = easy[:B // 2] + [hard] + easy[B // 2:]
    bet = np.tile(synth.uniform_angles(R), (B, 1))
    pr2 = P.from_clusters(allc, circulant=True)
    pr2.set_circulant(R, 1)
    rho, flag, _, iters, _ = pr2.gmres(betas=bet, restart=10, tol=1e-12, maxit=5000)
    it = iters.cpu().numpy().reshape(B, R)
    say("  straggler: easy max", int(np.delete(it, B // 2, axis=0).max()), "hard", it[B // 2].tolist())
    assert torch.all(flag == 0)
    assert it[B // 2].min() > 4 * np.delete(it, B // 2, axis=0).max()
    for c, b, Y in zip(allc, bet, pr2.split(rho, R)):
        assert rel(Y.cpu().numpy(), _lu(c, b)) < 1e-10
    # replayed cycles with the straggler phase: the graph is captured again after
    # each compaction, and the solve is bit-identical to the eager one
    for rep in range(2):
        rho_g, flag_g, _, iters_g, _ = pr2.gmres(betas=bet, restart=10, tol=1e-12, maxit=5000, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(iters_g, iters) and torch.equal(flag_g, flag) and torch.equal(rho_g, rho), rep

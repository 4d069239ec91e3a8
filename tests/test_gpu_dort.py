"""GPU parity of the time-reversal (DORT) path of the paper's Example III
against the CPU oracle, through the C ABI via the binding.

Tolerances:
  * far-field matrix F from GMRES at tol 1e-13: 1e-10 of max |F| elementwise;
  * T = conj(F)^T F: 1e-10 of max |T| elementwise;
  * eigenvalues: significant ones (>= 1e-8 w_max) to 1e-10 relative, the rest
    (rounding-level, rank deficiency) below 1e-10 w_max in absolute value;
  * eigenvectors of significant simple eigenvalues: |v_gpu^H v_oracle| within
    1e-9 of 1 (eigenvectors are unique up to a phase);
  * Herglotz waves: 1e-12 of max |u| elementwise (a plain sum of unit phases).
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import dort

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def P():
    from paper_1409_8186_amd import Problem
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return Problem


def _check_eig(w, ev, w_ref, V_ref, T_ref):
    n = len(w_ref)
    wmax = w_ref[0]
    sig = w_ref >= 1e-8 * wmax
    np.testing.assert_allclose(w[sig], w_ref[sig], rtol=1e-10)
    assert np.max(np.abs(w[~sig])) <= 1e-10 * wmax if np.any(~sig) else True
    # unit, mutually orthogonal eigenvectors (rows of ev)
    G = ev @ ev.conj().T
    assert np.max(np.abs(G - np.eye(n))) < 1e-11
    # T v = w v for the significant ones
    for j in np.nonzero(sig)[0]:
        v = ev[j]
        assert np.linalg.norm(T_ref @ v - w[j] * v) <= 1e-10 * wmax
    # simple significant eigenvalues: same eigenvector up to a phase
    gaps = np.abs(np.diff(w_ref))
    for j in np.nonzero(sig)[0]:
        gap = min(gaps[j - 1] if j > 0 else np.inf, gaps[j] if j < n - 1 else np.inf)
        if gap > 1e-6 * wmax:
            assert abs(abs(np.vdot(V_ref[:, j], ev[j])) - 1.0) < 1e-9


@pytest.mark.parametrize("n_alpha", [24, 23])
def test_mirror_farfield_tro_and_eigh_match_oracle(P, n_alpha):
    """Random 5-disk cluster: F, T and the eigenpairs of T; an odd mirror size
    takes the padded pairing of the Jacobi rounds."""
    from paper_1409_8186_amd import tro, tro_eigh
    cl = synth.small_random(21, 5, 0.3, 0.8, 6.0, 0.3, 4.0, 4)
    say("dort small: n_alpha", n_alpha, "N_tot", cl.n_tot)
    pr = P.from_cluster(cl)
    X, flag, relres, iters = pr.mirror_farfield(n_alpha, restart=30, tol=1e-13, maxit=2000)
    assert int(flag.max()) == 0
    F_ref = dort.farfield_matrix(cl.centers, cl.radii, cl.n_modes, cl.k, n_alpha)
    Xh = X.cpu().numpy()
    assert np.max(np.abs(Xh - F_ref.T)) <= 1e-10 * np.max(np.abs(F_ref))
    T = tro(X).cpu().numpy()
    T_ref = dort.time_reversal(F_ref)
    assert np.max(np.abs(T - T_ref)) <= 1e-10 * np.max(np.abs(T_ref))
    assert np.max(np.abs(T - T.conj().T)) <= 1e-13 * np.max(np.abs(T_ref))
    w, ev, sweeps = tro_eigh(X)
    say("  jacobi sweeps", sweeps)
    assert 1 <= sweeps <= 30
    w_ref, V_ref = dort.eig_desc(T_ref)
    _check_eig(w.cpu().numpy(), ev.cpu().numpy(), w_ref, V_ref, T_ref)
    # X itself is left unchanged by tro_eigh
    assert np.array_equal(X.cpu().numpy(), Xh)


def test_tro_eigh_single_disk_closed_form(P):
    """One disk: the 2N+1 nonzero eigenvalues N_alpha^2 |c_m|^2 from the Mie
    far-field coefficients, the rest zero."""
    from scipy import special as sp
    from paper_1409_8186_amd import tro_eigh
    center, a, k, N, n_alpha = (0.8, -0.3), 0.7, 5.0, 6, 32
    cl = synth.Cluster(np.array([center]), np.array([a]), np.array([N], np.int32), k)
    pr = P.from_cluster(cl)
    X, flag, _, _ = pr.mirror_farfield(n_alpha, restart=20, tol=1e-13, maxit=500)
    w, ev, sweeps = tro_eigh(X)
    w = w.cpu().numpy()
    m = np.arange(-N, N + 1)
    c = -np.exp(-0.25j * np.pi) * np.sqrt(2.0 / (np.pi * k)) * sp.jv(m, k * a) / sp.hankel1(m, k * a)
    ref = np.sort(n_alpha ** 2 * np.abs(c) ** 2)[::-1]
    np.testing.assert_allclose(w[:2 * N + 1], ref, rtol=1e-10)
    assert np.max(np.abs(w[2 * N + 1:])) < 1e-11 * w[0]


@pytest.mark.parametrize("n,m", [(1, 7), (18, 40), (257, 120), (300, 700), (600, 300), (40, 1500),
                                 (24, 2100), (40, 5)])
def test_tro_eigh_random_matrix(P, n, m):
    """Eigenpairs of T = conj(X) X^T for a seeded complex Gaussian X against the
    oracle's dense eigen-decomposition.  Rows of at most 1024 entries take
    blocks of 4 columns, one (n = 1, 18), two (n = 257) or two per 512 threads
    (n = 300, 600) entries per thread, with a partial last block and the padding
    block for n = 18 and 257; longer rows take one column pair per workgroup,
    held in registers (m = 1500) or streamed (m = 2100).  n = 40, m = 5: rank 5,
    35 eigenvalues at the rounding level (the eps |F|^2 stopping rule)."""
    from paper_1409_8186_amd import tro_eigh
    rng = np.random.default_rng(1000 + n)
    Xh = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    say("tro_eigh random: n", n, "m", m)
    w, ev, sweeps = tro_eigh(torch.tensor(Xh, device="cuda"))
    say("  jacobi sweeps", sweeps)
    assert 1 <= sweeps <= 30
    T_ref = dort.time_reversal(Xh.T)
    w_ref, V_ref = dort.eig_desc(T_ref)
    _check_eig(w.cpu().numpy(), ev.cpu().numpy(), w_ref, V_ref, T_ref)


def test_tro_eigh_zero_matrix(P):
    """F = 0: no pair is rotated, one sweep, all eigenvalues 0 and V = I."""
    from paper_1409_8186_amd import tro_eigh
    w, ev, sweeps = tro_eigh(torch.zeros((9, 4), dtype=torch.complex128, device="cuda"))
    assert sweeps == 1
    assert np.array_equal(w.cpu().numpy(), np.zeros(9))
    assert np.array_equal(ev.cpu().numpy(), np.eye(9))


@pytest.mark.parametrize("m", [0, 2, -5])
def test_herglotz_matches_oracle_and_jacobi_anger(P, m):
    from scipy import special as sp
    from paper_1409_8186_amd import herglotz
    k, n_alpha = 2 * math.pi, 128
    al = dort.mirror_angles(n_alpha)
    rng = np.random.default_rng(9)
    pts = rng.uniform(-4, 4, size=(300, 2))
    f = np.stack([np.exp(-1j * m * al), rng.standard_normal(n_alpha) + 1j * rng.standard_normal(n_alpha)])
    u = herglotz(al, torch.tensor(f, device="cuda"), k, pts).cpu().numpy()
    for t in range(2):
        ref = dort.herglotz(n_alpha, f[t], k, pts)
        assert np.max(np.abs(u[t] - ref)) <= 1e-12 * np.max(np.abs(ref))
    r, phi = np.hypot(pts[:, 0], pts[:, 1]), np.arctan2(pts[:, 1], pts[:, 0])
    closed = 2 * np.pi * (1j ** m) * sp.jv(m, k * r) * np.exp(-1j * m * phi)
    assert np.max(np.abs(u[0] - closed)) < 1e-11


def test_dort_example_full_size(P):
    """The paper's example at 512 mirror cells: three significant eigenvalues
    equal to the oracle's, the rest orders of magnitude below, and the
    Herglotz wave of each of the three eigenvectors focusing on its obstacle,
    equal to the oracle's values at the obstacle centers."""
    from paper_1409_8186_amd import herglotz, tro, tro_eigh
    n_alpha = 512
    cl = synth.dort_example(n_alpha)
    say("dort example: N_tot", cl.n_tot, "n_alpha", n_alpha)
    pr = P.from_cluster(cl)
    X, flag, relres, iters = pr.mirror_farfield(n_alpha, restart=30, tol=1e-13, maxit=2000)
    assert int(flag.max()) == 0
    F_ref = dort.farfield_matrix(cl.centers, cl.radii, cl.n_modes, cl.k, n_alpha)
    assert np.max(np.abs(X.cpu().numpy() - F_ref.T)) <= 1e-10 * np.max(np.abs(F_ref))
    T_ref = dort.time_reversal(F_ref)
    T = tro(X).cpu().numpy()
    assert np.max(np.abs(T - T_ref)) <= 1e-10 * np.max(np.abs(T_ref))
    w, ev, sweeps = tro_eigh(X)
    say("  jacobi sweeps", sweeps)
    w, ev = w.cpu().numpy(), ev.cpu().numpy()
    w_ref, V_ref = dort.eig_desc(T_ref)
    np.testing.assert_allclose(w[:3], w_ref[:3], rtol=1e-10)
    assert w[2] > 100 * w[3]
    al = dort.mirror_angles(n_alpha)
    u = herglotz(al, torch.tensor(ev[:3], device="cuda"), cl.k, cl.centers).cpu().numpy()
    for j in range(3):
        a = np.abs(u[j])
        assert np.argmax(a) == j and a[j] > 2 * np.max(np.delete(a, j))
        # same as the oracle's wave up to the eigenvector's phase
        ref = np.abs(dort.herglotz(n_alpha, V_ref[:, j], cl.k, cl.centers))
        np.testing.assert_allclose(a, ref, rtol=1e-8)

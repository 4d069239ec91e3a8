"""Host helpers of s-step GMRES (paper_1409_8186_amd/csrc/ritz.h): eigenvalues
of complex upper Hessenberg matrices against numpy.linalg.eigvals, and the Leja
ordering of the shifts (first the value of largest modulus, then each the
maximiser of the product of distances to those before it), checked by brute
force, and the scales of the Newton steps (largest distance from the shift to
a Ritz value).  Built with g++ (plain C++, no device code)."""
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
EXE = os.path.join(HERE, "native", "_build", "ritz_driver")


@pytest.fixture(scope="module")
def driver():
    os.makedirs(os.path.dirname(EXE), exist_ok=True)
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_1409_8186_amd", "csrc"),
                    os.path.join(HERE, "native", "ritz_driver.cpp"), "-o", EXE], check=True)
    return EXE


def _run(exe, mats, s):
    txt = []
    for H in mats:
        n = H.shape[0]
        txt.append(f"{n} {s}")
        txt.extend(f"{float(z.real)!r} {float(z.imag)!r}" for z in H.T.ravel())
    out = subprocess.run([exe], input="\n".join(txt) + "\n", capture_output=True, text=True,
                         check=True).stdout.split("\n")
    res, i = [], 0
    for H in mats:
        ok, m = map(int, out[i].split())
        i += 1
        ev = np.array([complex(*map(float, out[i + k].split())) for k in range(m)])
        i += m
        lj = np.array([complex(*map(float, out[i + k].split())) for k in range(s)])
        i += s
        sg = np.array([float(out[i + k]) for k in range(s)])
        i += s
        res.append((ok, ev, lj, sg))
    return res


def _match(a, b):
    """Largest distance after pairing each eigenvalue of a with the nearest unused one of b."""
    b = list(b)
    worst = 0.0
    for z in a:
        k = int(np.argmin([abs(z - w) for w in b]))
        worst = max(worst, abs(z - b.pop(k)))
    return worst


def test_hessenberg_eigenvalues_match_numpy(driver):
    rng = np.random.default_rng(11)
    mats = []
    for n in (1, 2, 5, 20, 50):
        H = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
        mats.append(np.triu(H, -1))
    # an Arnoldi Hessenberg matrix of I + K (eigenvalues clustered around 1)
    n = 200
    A = np.eye(n) + 0.3 * (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) / np.sqrt(n)
    m = 50
    V = np.zeros((n, m + 1), complex)
    Hm = np.zeros((m + 1, m), complex)
    v = rng.normal(size=n) + 0j
    V[:, 0] = v / np.linalg.norm(v)
    for j in range(m):
        w = A @ V[:, j]
        for _ in range(2):
            h = V[:, :j + 1].conj().T @ w
            w -= V[:, :j + 1] @ h
            Hm[:j + 1, j] += h
        Hm[j + 1, j] = np.linalg.norm(w)
        V[:, j + 1] = w / Hm[j + 1, j]
    mats.append(Hm[:m, :m])
    # a matrix with a repeated eigenvalue (Jordan-like block) and a zero subdiagonal
    J = np.diag([2.0 + 1j] * 3 + [0.5, -1.0]).astype(complex) + np.diag([1.0, 0.0, 1.0, 1.0], 1)
    mats.append(J)
    for H, (ok, ev, _, _) in zip(mats, _run(driver, mats, 1)):
        assert ok and len(ev) == H.shape[0]
        ref = np.linalg.eigvals(H)
        tol = 1e-10 * max(1.0, np.abs(ref).max())
        if H is J:
            tol = 1e-4  # a defective eigenvalue is only determined to eps^(1/2)
        assert _match(ev, ref) < tol, (H.shape, _match(ev, ref))


def test_leja_order(driver):
    rng = np.random.default_rng(12)
    H = np.triu(rng.normal(size=(30, 30)) + 1j * rng.normal(size=(30, 30)), -1)
    (ok, ev, lj, sg), = _run(driver, [H], 8)
    assert ok
    vals = list(ev)
    k = int(np.argmax(np.abs(vals)))
    pick = [vals.pop(k)]
    while len(pick) < 8:
        score = [np.prod([abs(z - t) for t in pick]) for z in vals]
        pick.append(vals.pop(int(np.argmax(score))))
    assert np.allclose(lj, pick, rtol=0, atol=1e-12)
    # Newton scales: the largest distance from each shift to a Ritz value
    assert np.allclose(sg, [max(abs(z - t) for z in ev) for t in lj], rtol=1e-14, atol=0)
    # fewer values than shifts: the order repeats
    (_, ev2, lj2, sg2), = _run(driver, [np.array([[1.0 + 0j, 2.0], [0.0, 3.0]])], 5)
    assert np.allclose(lj2, [3, 1, 3, 1, 3])
    assert np.allclose(sg2, [2, 2, 2, 2, 2])
    # a single Ritz value: every distance is zero, the scale falls back to 1
    (_, _, lj3, sg3), = _run(driver, [np.array([[0.7 + 0.2j]])], 3)
    assert np.allclose(lj3, [0.7 + 0.2j] * 3) and np.allclose(sg3, [1, 1, 1])

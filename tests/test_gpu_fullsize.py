"""GPU parity at the full workload sizes, on sampled outputs the oracle can form
one by one (rows of the operator, single instances, single configurations),
and on properties that hold at any size.

  * multi_rhs: M = 1000 disks, uneven N_p = ceil(10 a_p) + 10, R = 256: sampled
    operator rows of the direct (FP64-MFMA tiles) and the circulant form
    against oracle row blocks; the GMRES solve of 8 of its 256 incidences at
    tol 1e-12 (circulant form): the true residual of every column from oracle
    rows of all 1000 disks against the reported one, the optical theorem and
    far-field reciprocity between the columns;
  * uneven instances: 512 seeded instances x 8 incidences solved together at
    the workload's tol 1e-8 (every column converges; the reported true
    residual against the oracle's on sampled instances), then the sampled
    instances, the largest and the slowest among them, re-solved at tol 1e-12
    against oracle LU to 1e-10;
  * differentiation: 32 configurations x 64 incidences x 64 receivers, adjoint
    gradient (tol 1e-12): sampled configurations against the oracle gradient.
"""
import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import synth
from oracle import farfield, geometry, gradient, operator, rhs, solve

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.fixture(scope="module")
def P():
    from paper_1409_8186_amd import Problem
    assert torch.cuda.is_available()
    return Problem


@pytest.mark.parametrize("form", ["direct", "circulant"])
def test_multi_rhs_full_size_apply(P, form):
    cl = synth.multi_rhs()
    R = 256
    say("multi_rhs: M", cl.M, "N_tot", cl.n_tot, "R", R, "form", form)
    pr = P.from_cluster(cl, circulant=form == "circulant")
    if form == "circulant":
        pr.set_circulant(R, 1)
    rng = np.random.default_rng(33)
    X = rng.normal(size=(R, cl.n_tot)) + 1j * rng.normal(size=(R, cl.n_tot))
    y = pr.matvec(torch.tensor(X.ravel(), device="cuda"), R=R, op=1).cpu().numpy().reshape(R, -1)
    assert pr.apply_config(R)["kind"] == ("circulant" if form == "circulant" else "mfma")
    off, _ = geometry.mode_offsets(cl.n_modes)
    D = operator.efie_diagonal(cl.radii, cl.n_modes, cl.k)
    b, _ = geometry.pair_geometry(cl.centers)
    near = (cl.k * b < cl.n_modes[:, None] + cl.n_modes[None, :]).sum(1) - 1
    # rows with the most close pairs (direct part of the circulant form) and others
    sample = sorted(set([0, 17, 500, 998, 999, int(np.argmax(near))] + list(rng.integers(0, cl.M, 5))))
    worst = 0.0
    for p in sample:
        blk = operator.efie_row_block(cl.centers, cl.radii, cl.n_modes, cl.k, int(p))
        rows = slice(off[p], off[p + 1])
        ref = (X @ blk.T) / D[rows][None, :]            # rows of A = D^-1 L, all 256 columns
        worst = max(worst, rel(y[:, rows], ref))
    say("  worst sampled-row rel err", worst, "close pairs of the sampled rows", near[sample].tolist())
    assert worst < 1e-12


def test_multi_rhs_full_size_solve(P):
    """8 of the workload's 256 incidences (beta_j, j = 0, 32, ..., 224: pairs
    j, j + 128 opposite) solved at tol 1e-12 on the circulant form, the launch
    configuration of the bench line with R = 8.  Checks: (1) the true
    residual ||A x - f|| / ||f|| of every column from oracle rows of all 1000
    disks (the oracle's own assembly, threaded over disks) is below 1e-11 and
    equals the reported one; (2) the optical theorem per column (exact for the
    truncated system, trapezoid rule on 4608 far-field angles, more than
    2 (k max|O_p| + max N_p) + 64); (3) reciprocity a_j(beta_i + pi) =
    a_i(beta_j + pi) between all pairs of columns."""
    cl = synth.multi_rhs()
    idx = np.arange(0, 256, 32)
    betas = synth.uniform_angles(256)[idx]
    R = len(idx)
    pr = P.from_cluster(cl, circulant=True)
    rho, flag, relres, iters, _ = pr.gmres(betas=betas[None, :], restart=50, tol=1e-12, maxit=20000)
    say("multi_rhs solve: iterations", iters.cpu().numpy().tolist(), "form", pr.apply_config(R)["kind"])
    assert torch.all(flag == 0), flag
    x = rho.cpu().numpy().reshape(R, -1)
    relres = relres.cpu().numpy()
    D = operator.efie_diagonal(cl.radii, cl.n_modes, cl.k)
    U = rhs.planewave(cl.centers, cl.radii, cl.n_modes, cl.k, betas)
    f = -U / D[None, :]
    off, _ = geometry.mode_offsets(cl.n_modes)

    def resid_rows(p):
        blk = operator.efie_row_block(cl.centers, cl.radii, cl.n_modes, cl.k, p)
        rows = slice(off[p], off[p + 1])
        return p, (x @ blk.T) / D[rows][None, :] - f[:, rows]
    r = np.zeros_like(x)
    with ThreadPoolExecutor(16) as ex:
        for p, rr in ex.map(resid_rows, range(cl.M)):
            r[:, off[p]:off[p + 1]] = rr
    res = np.linalg.norm(r, axis=1) / np.linalg.norm(f, axis=1)
    say("  true residual (oracle rows)", res.max(), "reported", relres.max())
    assert np.all(res < 1e-11)
    assert np.all(np.abs(res - relres) <= 1e-6 * relres + 5e-14)
    nth = 4608
    th = synth.uniform_angles(nth)
    a = pr.farfield(rho, th, R=R).cpu().numpy()
    lhs = (2 * np.pi / nth) * np.sum(np.abs(a) ** 2, axis=1)
    at_beta = a[np.arange(R), (idx * (nth // 256))]
    opt = -math.sqrt(8 * math.pi / cl.k) * np.real(np.exp(0.25j * math.pi) * at_beta)
    say("  optical theorem worst rel", np.max(np.abs(lhs - opt) / lhs))
    assert np.all(np.abs(lhs - opt) <= 1e-10 * lhs)
    sh = nth // 2
    rec = max(abs(a[j, (idx[i] * (nth // 256) + sh) % nth] - a[i, (idx[j] * (nth // 256) + sh) % nth])
              / abs(a[i, (idx[j] * (nth // 256) + sh) % nth]) for i in range(R) for j in range(R))
    say("  reciprocity worst rel", rec)
    assert rec < 1e-10


def test_uneven_instances_full_size_gmres(P):
    """All 512 instances x 8 incidences in one solve, the documentation run's
    launch configuration (circulant form where it pays, GMRES(300), tol 1e-8):
    every column converges, and on sampled instances the reported true
    residual equals the oracle's ||A x - f|| / ||f|| of the returned iterate.
    The sampled instances (the largest, the smallest, the three slowest and
    two seeded ones) are then re-solved together at tol 1e-13 and compared
    with oracle LU at the parity bar, 1e-10."""
    insts = synth.uneven_instances()
    R = 8
    say("uneven: instances", len(insts), "unknowns", sum(c.n_tot for c in insts))
    pr = P.from_clusters(insts, circulant=True)
    betas = np.stack([c.betas for c in insts])
    rho, flag, relres, iters, _ = pr.gmres(betas=betas, restart=300, tol=1e-8, maxit=20000)
    flag = flag.cpu().numpy().reshape(len(insts), R)
    relres = relres.cpu().numpy().reshape(len(insts), R)
    it = iters.cpu().numpy().reshape(len(insts), R)
    say("  form", pr.apply_config(R)["kind"], "converged columns", int((flag == 0).sum()), "of",
        flag.size, "iterations", int(it.min()), "..", int(it.max()))
    assert np.all(flag == 0)
    parts = pr.split(rho, R)
    Ms = np.array([c.M for c in insts])
    nts = np.array([c.n_tot for c in insts])
    rng = np.random.default_rng(12)
    slow = np.argsort(it.max(axis=1))[-3:]
    sample = sorted(set([int(np.argmin(Ms)), int(np.argmax(nts))] + [int(b) for b in slow]
                        + rng.choice(len(insts), 2, replace=False).tolist()))
    mats = {}
    for b in sample:
        c = insts[b]
        L = operator.efie_matrix(c.centers, c.radii, c.n_modes, c.k)
        D = operator.efie_diagonal(c.radii, c.n_modes, c.k)
        U = rhs.planewave(c.centers, c.radii, c.n_modes, c.k, c.betas)
        mats[b] = (L, U)
        x = parts[b].cpu().numpy().reshape(R, -1)
        f = -U / D[None, :]
        res = np.array([np.linalg.norm((L @ x[r]) / D + U[r] / D) / np.linalg.norm(f[r])
                        for r in range(R)])
        dev = np.abs(res - relres[b])
        say("  instance", b, "M", c.M, "k %.2f" % c.k, "iterations", it[b].tolist(),
            "relres gpu/oracle max %.3e / %.3e, worst difference %.2e" % (relres[b].max(),
                                                                         res.max(), dev.max()))
        # the residual of an iterate is itself computed to ~eps ||A|| ||x|| / ||f||
        assert np.all(dev <= 1e-6 * relres[b] + 5e-14)
        assert np.all(res <= 1.0000001e-8)
    # the low-frequency dense instances (k ~ 1.6-2.4, M ~ 160-200) are ill
    # conditioned: at tol 1e-12 their iterates differ from LU by ~2e-10, so the
    # re-solve runs to tol 1e-13
    sub = [insts[b] for b in sample]
    ps = P.from_clusters(sub, circulant=True)
    rho2, flag2, relres2, iters2, _ = ps.gmres(betas=np.stack([c.betas for c in sub]), restart=300,
                                               tol=1e-13, maxit=40000)
    say("  tol 1e-13 re-solve of", sample, "iterations",
        iters2.cpu().numpy().reshape(len(sub), R).max(axis=1).tolist())
    assert torch.all(flag2 == 0), flag2
    errs = {}
    for b, Y in zip(sample, ps.split(rho2, R)):
        L, U = mats[b]
        errs[b] = rel(Y.cpu().numpy(), solve.efie_solve_lu(L, U))
    say("    LU rel per instance", errs)
    assert max(errs.values()) < 1e-10


def test_differentiation_full_size(P):
    pairs = synth.differentiation()
    say("differentiation: configs", len(pairs), "unknowns", pairs[0][0].n_tot)
    sample = [0, 31]
    targets = []
    for i, (base, tgt) in enumerate(pairs):
        if i in sample:
            targets.append(gradient.forward(tgt.centers, tgt.radii, tgt.n_modes, tgt.k,
                                            base.betas, base.thetas))
        else:   # any seeded target is a valid misfit; zeros keep the test short
            targets.append(np.zeros((len(base.betas), len(base.thetas)), complex))
    bases = [b for b, _ in pairs]
    pr = P.from_clusters(bases)
    betas = np.stack([b.betas for b in bases])
    tg = np.concatenate([t.reshape(-1) for t in targets])
    loss, dc, da, dk = pr.grad(betas, bases[0].thetas, tg, restart=50, tol=1e-12, maxit=20000)
    loss, dc, da, dk = loss.cpu().numpy(), dc.cpu().numpy(), da.cpu().numpy(), dk.cpu().numpy()
    o = np.concatenate([[0], np.cumsum([b.M for b in bases])])
    for i in sample:
        b = bases[i]
        l0, dc0, da0, dk0 = gradient.misfit_grad(b.centers, b.radii, b.n_modes, b.k, b.betas,
                                                 b.thetas, targets[i])
        g = np.concatenate([dc[o[i]:o[i + 1]].ravel(), da[o[i]:o[i + 1]], [dk[i]]])
        g0 = np.concatenate([dc0.ravel(), da0, [dk0]])
        say("  config", i, "loss", loss[i], l0, "grad rel", rel(g, g0))
        assert abs(loss[i] - l0) <= 1e-10 * l0
        assert rel(g, g0) < 1e-10

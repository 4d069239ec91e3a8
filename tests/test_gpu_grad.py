"""GPU parity of the adjoint gradient (mudiff_grad) against the oracle's adjoint
gradient (1e-10) and the oracle's central differences (1e-6), single and
batched instances, and the torch.autograd.Function wrapper."""
import numpy as np
import pytest
import torch

import synth
from oracle import gradient

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _case(seed, M=5, R=3, n_rec=6):
    base = synth.small_random(seed, M, 0.4, 0.7, 6.0, 0.3, 3.0, 4, R=R, n_theta=n_rec)
    rng = np.random.default_rng(seed + 100)
    tgt = synth.perturb(rng, base)
    target = gradient.forward(tgt.centers, tgt.radii, tgt.n_modes, tgt.k, base.betas, base.thetas)
    return base, target


@pytest.fixture(scope="module")
def P():
    from paper_1409_8186_amd import Problem
    assert torch.cuda.is_available()
    return Problem


def _gpu_grad(P, cls, targets):
    pr = P.from_clusters(cls)
    betas = np.stack([c.betas for c in cls])
    tg = np.concatenate([t.reshape(-1) for t in targets])
    loss, dc, da, dk = pr.grad(betas, cls[0].thetas, tg, restart=40, tol=1e-13, maxit=5000)
    return (loss.cpu().numpy(), dc.cpu().numpy(), da.cpu().numpy(), dk.cpu().numpy())


def test_grad_vs_oracle_adjoint(P):
    base, target = _case(51)
    say("grad single")
    loss, dc, da, dk = _gpu_grad(P, [base], [target])
    args = (base.centers, base.radii, base.n_modes, base.k, base.betas, base.thetas, target)
    l0, dc0, da0, dk0 = gradient.misfit_grad(*args)
    say("  loss", loss[0], l0)
    assert abs(loss[0] - l0) <= 1e-10 * l0
    g = np.concatenate([dc.ravel(), da, dk])
    g0 = np.concatenate([dc0.ravel(), da0, [dk0]])
    say("  rel", rel(g, g0))
    assert rel(g, g0) < 1e-10


def test_grad_vs_central_differences(P):
    base, target = _case(52, M=4, R=2, n_rec=5)
    say("grad fd")
    _, dc, da, dk = _gpu_grad(P, [base], [target])
    args = (base.centers, base.radii, base.n_modes, base.k, base.betas, base.thetas, target)
    fc, fa, fk = gradient.misfit_fd(*args, h=1e-5)
    g = np.concatenate([dc.ravel(), da, dk])
    f = np.concatenate([fc.ravel(), fa, [fk]])
    assert rel(g, f) < 1e-6
    assert np.all(np.abs(g - f) <= 1e-6 * np.max(np.abs(f)) + 1e-6 * np.abs(f))


def test_grad_batched_instances(P):
    cases = [_case(60 + i, M=3 + i, R=3, n_rec=6) for i in range(3)]
    cls = [c for c, _ in cases]
    say("grad batched")
    loss, dc, da, dk = _gpu_grad(P, cls, [t for _, t in cases])
    o = 0
    for b, (c, t) in enumerate(cases):
        l0, dc0, da0, dk0 = gradient.misfit_grad(c.centers, c.radii, c.n_modes, c.k, c.betas,
                                                 c.thetas, t)
        M = c.M
        g = np.concatenate([dc[o:o + M].ravel(), da[o:o + M], [dk[b]]])
        g0 = np.concatenate([dc0.ravel(), da0, [dk0]])
        assert abs(loss[b] - l0) <= 1e-10 * l0
        assert rel(g, g0) < 1e-10, (b, rel(g, g0))
        o += M


def test_autograd_function(P):
    from paper_1409_8186_amd import FarFieldMisfit
    cases = [_case(70 + i, M=4, R=2, n_rec=5) for i in range(2)]
    cls = [c for c, _ in cases]
    say("autograd")
    centers = torch.tensor(np.concatenate([c.centers for c in cls]), dtype=torch.float64,
                           device="cuda", requires_grad=True)
    radii = torch.tensor(np.concatenate([c.radii for c in cls]), dtype=torch.float64,
                         device="cuda", requires_grad=True)
    k = torch.tensor([c.k for c in cls], dtype=torch.float64, device="cuda", requires_grad=True)
    n_modes = np.concatenate([c.n_modes for c in cls])
    off = np.array([0, 4, 8])
    betas = np.stack([c.betas for c in cls])
    target = np.concatenate([t for _, t in cases])
    loss = FarFieldMisfit.apply(centers, radii, k, n_modes, off, betas, cls[0].thetas, target,
                                {"tol": 1e-13})
    w = torch.tensor([0.7, -1.3], dtype=torch.float64, device="cuda")
    (loss * w).sum().backward()
    _, dc, da, dk = _gpu_grad(P, cls, [t for _, t in cases])
    wi = np.repeat([0.7, -1.3], 4)
    assert rel(centers.grad.cpu().numpy(), dc * wi[:, None]) < 1e-12
    assert rel(radii.grad.cpu().numpy(), da * wi) < 1e-12
    assert rel(k.grad.cpu().numpy(), dk * np.array([0.7, -1.3])) < 1e-12


def test_grad_sstep_solves(P):
    """The forward and adjoint solves as s-step GMRES (flags MUDIFF_SSTEP with
    size 4, restart 8, so that several s-step cycles run), two instances of 8
    incidences (the FP64-MFMA apply): the oracle's adjoint gradient to 1e-10."""
    from paper_1409_8186_amd import _lib as L
    cases = [_case(70 + i, M=5 + i, R=8, n_rec=6) for i in range(2)]
    cls = [c for c, _ in cases]
    pr = P.from_clusters(cls)
    betas = np.stack([c.betas for c in cls])
    tg = np.concatenate([t.reshape(-1) for _, t in cases])
    say("grad s-step")
    loss, dc, da, dk = pr.grad(betas, cls[0].thetas, tg, restart=8, tol=1e-13, maxit=5000,
                               flags=L.SSTEP | L.sstep_size(4))
    loss, dc, da, dk = (x.cpu().numpy() for x in (loss, dc, da, dk))
    o = 0
    for b, (c, t) in enumerate(cases):
        l0, dc0, da0, dk0 = gradient.misfit_grad(c.centers, c.radii, c.n_modes, c.k, c.betas,
                                                 c.thetas, t)
        assert abs(loss[b] - l0) <= 1e-10 * l0
        g = np.concatenate([dc[o:o + c.M].ravel(), da[o:o + c.M], [dk[b]]])
        g0 = np.concatenate([dc0.ravel(), da0, [dk0]])
        say("  instance", b, "rel", rel(g, g0))
        assert rel(g, g0) < 1e-10
        o += c.M

"""torch.autograd.Function around mudiff_grad: the far-field misfit of B disk
clusters as a differentiable function of their centers, radii and wavenumbers.

The forward pass rebuilds the device tables from the current parameters (the
Hankel tables are recomputed, not stored across calls), runs the forward and
adjoint solves in mudiff_grad and keeps the gradient; backward scales it by
the incoming gradient of each instance's loss.  Truncation orders N_p are
fixed inputs (not differentiated).
"""
from __future__ import annotations

import numpy as np
import torch

from .api import Problem


class FarFieldMisfit(torch.autograd.Function):
    """loss[b] = sum_{r, j} |a_b(theta_j; beta_{b,r}) - target_{b,r,j}|^2.

    Arguments: centers [M,2] float64, radii [M] float64, k [B] float64 (the
    differentiable inputs), then n_modes [M] (int), disk_off [B+1] (int),
    betas [B,R], thetas [n_rec], target [B*R, n_rec] complex128 and a dict of
    solver options (restart, tol, maxit)."""

    @staticmethod
    def forward(ctx, centers, radii, k, n_modes, disk_off, betas, thetas, target, opts=None):
        opts = dict(opts or {})
        c = centers.detach().cpu().numpy()
        a = radii.detach().cpu().numpy()
        kk = k.detach().cpu().numpy().reshape(-1)
        nm = np.asarray(n_modes)
        off = np.asarray(disk_off)
        inst = [(c[off[b]:off[b + 1]], a[off[b]:off[b + 1]], nm[off[b]:off[b + 1]], kk[b])
                for b in range(len(off) - 1)]
        dev = centers.device if centers.is_cuda else torch.device("cuda")
        P = Problem(inst, device=str(dev))
        loss, dc, da, dk = P.grad(betas, thetas, target, restart=opts.get("restart", 50),
                                  tol=opts.get("tol", 1e-10), maxit=opts.get("maxit", 20000))
        P.close()
        inst_of = torch.as_tensor(np.repeat(np.arange(len(off) - 1), np.diff(off)), device=dev)
        ctx.save_for_backward(dc, da, dk, inst_of)
        return loss.to(centers.device)

    @staticmethod
    def backward(ctx, gl):
        dc, da, dk, inst_of = ctx.saved_tensors
        g = gl.to(dc.device)
        gi = g[inst_of]
        return (dc * gi[:, None]).to(gl.device), (da * gi).to(gl.device), (dk * g).to(gl.device), \
            None, None, None, None, None, None

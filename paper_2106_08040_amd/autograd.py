"""torch.autograd.Function around the solver: harmonics as a differentiable function of the
particle parameters (D, K, alpha, easy-axis polar and azimuth angles).

Forward runs fpn_solve; backward runs fpn_adjoint, which integrates the parameter tangents of the
discrete solve and contracts them with the incoming gradient in FP64.  Superposition weights,
data misfits and every other part of a loss are ordinary torch operations on the returned tensor.

Instances the solver flags (status other than OK or TOL_UNMET, e.g. UNRESOLVED: the degree does not
resolve the particle) have NaN harmonics; a loss has to leave them out (torch.where on
torch.isfinite), and their parameter gradient is returned as 0, the gradient of such a loss.
"""
from __future__ import annotations

import numpy as np


def _torch():
    import torch
    return torch


def axis_from_angles(theta, phi):
    torch = _torch()
    return torch.stack([torch.sin(theta) * torch.cos(phi), torch.sin(theta) * torch.sin(phi), torch.cos(theta)], -1)


class Harmonics:
    """Binds a context, a drive and the solve options; call it with the parameters."""

    def __init__(self, ctx, drive, samples, settle, n_harm, L, substeps=0, tol=0.0):
        self.ctx, self.drive = ctx, drive
        self.samples, self.settle, self.n_harm = samples, settle, n_harm
        self.L, self.substeps, self.tol = L, substeps, tol

    def __call__(self, params, Ms, T, offset):
        """params [n, 5] float64 (D [m], K [J/m^3], alpha, theta, phi) with requires_grad as needed;
        Ms, T [n]; offset [n, 3] (mu0 H, T).  Returns Phi as a real tensor [n, 2, n_harm + 1, 2]."""
        return _HarmonicsFn.apply(params, self, Ms, T, offset)


def _inst(params, Ms, T, offset):
    torch = _torch()
    p = params.detach().to(torch.float64)
    return dict(D=p[:, 0], K=p[:, 1], alpha=p[:, 2], Ms=Ms, T=T, easy_axis=axis_from_angles(p[:, 3], p[:, 4]),
                offset=offset)


class _HarmonicsFn(_torch().autograd.Function):
    @staticmethod
    def forward(fctx, params, h, Ms, T, offset):
        torch = _torch()
        inst = _inst(params, Ms, T, offset)
        n = params.shape[0]
        L = np.broadcast_to(np.asarray(h.L, np.int32), (n,))
        _, harm, st = h.ctx.solve(inst, L, h.drive, h.samples, h.settle, h.n_harm, substeps=h.substeps,
                                  want_m=False, tol=h.tol)
        fctx.h = h
        fctx.inst = inst
        fctx.L = L
        fctx.save_for_backward(params)
        return torch.view_as_real(harm).clone()

    @staticmethod
    def backward(fctx, grad_out):
        h = fctx.h
        (params,) = fctx.saved_tensors
        torch = _torch()
        grad, _, st = h.ctx.adjoint(fctx.inst, fctx.L, h.drive, h.samples, h.settle, h.n_harm,
                                    grad_out.contiguous(), substeps=h.substeps, tol=h.tol, want_harm=False)
        from . import FPN_INST_OK, FPN_INST_TOL_UNMET
        failed = (st != FPN_INST_OK) & (st != FPN_INST_TOL_UNMET)
        grad = torch.where(failed[:, None], torch.zeros_like(grad), grad)
        return grad.to(params.dtype), None, None, None, None

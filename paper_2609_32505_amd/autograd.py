"""torch.autograd.Function wrappers: the forward and the backward both run
in the library (Algorithm 4 for the SVD, Algorithm 2 for the polar factors,
the EVD pseudo-gradient theorem for the symmetric eigendecomposition).
"""
from __future__ import annotations

import torch

from . import api


class SVD(torch.autograd.Function):
    """(U, S, Vh) like ``torch.linalg.svd(A, full_matrices=False)``."""

    @staticmethod
    def forward(ctx, A, opts):
        U, S, V, info = api.svd_fwd(A.contiguous(), **opts)
        ctx.save_for_backward(U, S, V)
        ctx.opts = {k: v for k, v in opts.items() if k in ("eps_K", "eps_R", "eps_T")}
        ctx.squeeze = A.dim() == 2
        Vh = V.transpose(-1, -2)
        if ctx.squeeze:
            return U[0], S[0], Vh[0]
        return U, S, Vh

    @staticmethod
    def backward(ctx, dU, dS, dVh):
        U, S, V = ctx.saved_tensors
        sq = ctx.squeeze
        def bat(t):
            return None if t is None else (t.unsqueeze(0) if sq else t).contiguous()
        dU, dS, dVh = bat(dU), bat(dS), bat(dVh)
        # the forward returns V^T: its incoming gradient is transposed to dV
        dV = None if dVh is None else dVh.transpose(-1, -2).contiguous()
        dA = api.svd_bwd(U, S, V, dU, dS, dV, **ctx.opts)
        return (dA[0] if sq else dA), None


class Polar(torch.autograd.Function):
    """(W, H) with A = W H."""

    @staticmethod
    def forward(ctx, A, opts):
        A = A.contiguous()
        W, H, S, V, info = api.polar_fwd(A, cache=True, **opts)
        ctx.save_for_backward(A if A.dim() == 3 else A.unsqueeze(0), S, V)
        ctx.opts = {k: v for k, v in opts.items() if k in ("eps_R", "eps_T")}
        ctx.squeeze = A.dim() == 2
        if ctx.squeeze:
            return W[0], H[0]
        return W, H

    @staticmethod
    def backward(ctx, dW, dH):
        A, S, V = ctx.saved_tensors
        sq = ctx.squeeze
        def bat(t):
            return None if t is None else (t.unsqueeze(0) if sq else t).contiguous()
        dA = api.polar_bwd(A, None, S, V, bat(dW), bat(dH), **ctx.opts)
        return (dA[0] if sq else dA), None


class Eigh(torch.autograd.Function):
    """(lam, V) with H = V diag(lam) V^T, lam descending."""

    @staticmethod
    def forward(ctx, H, opts):
        H = H.contiguous()
        lam, V, info = api.eigh(H, **opts)
        ctx.save_for_backward(lam, V)
        ctx.opts = {k: v for k, v in opts.items() if k == "eps_K"}
        ctx.squeeze = H.dim() == 2
        if ctx.squeeze:
            return lam[0], V[0]
        return lam, V

    @staticmethod
    def backward(ctx, dlam, dV):
        lam, V = ctx.saved_tensors
        sq = ctx.squeeze
        def bat(t):
            return None if t is None else (t.unsqueeze(0) if sq else t).contiguous()
        dH = api.eigh_bwd(lam, V, bat(dlam), bat(dV), **ctx.opts)
        return (dH[0] if sq else dH), None


def svd(A, **opts):
    """Differentiable thin SVD of A (m >= n): returns (U, S, Vh)."""
    return SVD.apply(A, opts)


def polar(A, **opts):
    """Differentiable polar decomposition A = W H: returns (W, H)."""
    return Polar.apply(A, opts)


def eigh(H, **opts):
    """Differentiable symmetric eigendecomposition: returns (lam, V)."""
    return Eigh.apply(H, opts)

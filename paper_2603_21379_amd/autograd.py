"""torch.autograd.Functions for the core projection and the reconstruction.

Forward and backward both run in libtkmi's kernels: the backward passes
call the hand-written vector-Jacobian products (tucker_core_vjp,
tucker_reconstruct_vjp), which recontract X instead of storing unfoldings.
Tensors of FP64 or FP32 are supported (factors in the same dtype).
"""
from __future__ import annotations

import torch

from . import binding as B


def _cols(F):
    return [int(f.shape[1]) for f in F]


class TuckerCore(torch.autograd.Function):
    """G = X x_1 F_1^T ... x_d F_d^T."""

    @staticmethod
    def forward(ctx, X, *F):
        X = X.contiguous()
        F = [f.contiguous() for f in F]
        G = torch.empty(_cols(F), dtype=B.factor_torch_dtype(X.dtype), device=X.device)
        B.tucker_core(X, F, G)
        ctx.save_for_backward(X, *F)
        return G

    @staticmethod
    def backward(ctx, Gbar):
        X, *F = ctx.saved_tensors
        Gbar = Gbar.contiguous().to(F[0].dtype)
        Xbar = torch.empty_like(X) if ctx.needs_input_grad[0] else None
        Fbar = [torch.empty_like(f) if ctx.needs_input_grad[1 + k] else None
                for k, f in enumerate(F)]
        if Xbar is not None or any(f is not None for f in Fbar):
            B.tucker_core_vjp(X, F, Gbar, Xbar=Xbar, Fbar=Fbar)
        return (Xbar, *Fbar)


class TuckerReconstruct(torch.autograd.Function):
    """X_hat = G x_1 F_1 ... x_d F_d (dims taken from the factors)."""

    @staticmethod
    def forward(ctx, G, *F):
        G = G.contiguous()
        F = [f.contiguous() for f in F]
        dims = [int(f.shape[0]) for f in F]
        Xh = torch.empty(dims, dtype=G.dtype, device=G.device)
        B.tucker_reconstruct(dims, G, F, Xhat=Xh)
        ctx.save_for_backward(G, *F)
        return Xh

    @staticmethod
    def backward(ctx, H):
        G, *F = ctx.saved_tensors
        H = H.contiguous().to(G.dtype)
        dims = [int(f.shape[0]) for f in F]
        Gbar = torch.empty_like(G) if ctx.needs_input_grad[0] else None
        Fbar = [torch.empty_like(f) if ctx.needs_input_grad[1 + k] else None
                for k, f in enumerate(F)]
        if Gbar is not None or any(f is not None for f in Fbar):
            B.tucker_reconstruct_vjp(dims, G, F, H, Gbar=Gbar, Fbar=Fbar)
        return (Gbar, *Fbar)


def tucker_core(X, F):
    return TuckerCore.apply(X, *F)


def tucker_reconstruct(G, F):
    return TuckerReconstruct.apply(G, *F)


def projection_loss(X, F):
    """||X - R(C(X, F), F)||_F^2 with both maps differentiable."""
    Xh = tucker_reconstruct(tucker_core(X, F), F)
    return ((X - Xh) ** 2).sum()

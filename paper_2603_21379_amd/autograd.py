"""torch.autograd.Functions for the core projection, the reconstruction and
the full tensor of an H-Tucker format.

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


class ProjectionLoss(torch.autograd.Function):
    """L = ||X - R(C(X, F), F)||_F^2 (C the core projection, R the
    reconstruction), as an FP64 device scalar.  Forward: tucker_core and the
    residual pass of tucker_reconstruct; backward: tucker_projection_loss_vjp,
    which keeps the loss's adjoint in the output gradient of X (no other
    X-sized buffer)."""

    @staticmethod
    def forward(ctx, X, *F):
        X = X.contiguous()
        F = [f.contiguous() for f in F]
        G = torch.empty(_cols(F), dtype=B.factor_torch_dtype(X.dtype), device=X.device)
        B.tucker_core(X, F, G)
        r2 = torch.empty(2, dtype=torch.float64, device=X.device)
        B.tucker_reconstruct(list(X.shape), G, F, Xref=X, resid2=r2)
        ctx.save_for_backward(X, G, *F)
        return r2[0]

    @staticmethod
    def backward(ctx, Lbar):
        X, G, *F = ctx.saved_tensors
        if Lbar.dtype != torch.float64:
            Lbar = Lbar.to(torch.float64)
        Lbar = Lbar.contiguous()
        Xbar = torch.empty_like(X) if ctx.needs_input_grad[0] else None
        Fbar = [torch.empty_like(f) if ctx.needs_input_grad[1 + k] else None
                for k, f in enumerate(F)]
        if Xbar is not None or any(f is not None for f in Fbar):
            B.tucker_projection_loss_vjp(X, F, G, Lbar, Xbar=Xbar, Fbar=Fbar)
        return (Xbar, *Fbar)


def projection_loss(X, F):
    """||X - R(C(X, F), F)||_F^2 with both maps differentiable (FP64 scalar)."""
    return ProjectionLoss.apply(X, *F)


class HTuckerFull(torch.autograd.Function):
    """Full tensor of an H-Tucker format (root relation and nested bases,
    Section 4) from its leaf bases and transfer tensors; gradients flow to
    every leaf basis and every transfer tensor."""

    @staticmethod
    def forward(ctx, spec, out_dtype, *params):
        dims, tree, ranks, leaves, internal = spec
        U = {t: p.contiguous() for t, p in zip(leaves, params[:len(leaves)])}
        Bd = {t: p.contiguous() for t, p in zip(internal, params[len(leaves):])}
        rk = [0] + [int(ranks[t]) for t in range(1, tree.num_nodes)]
        n = tree.num_nodes
        Ul = [U.get(t) for t in range(n)]
        Bl = [Bd.get(t) for t in range(n)]
        Xhat = torch.empty(tuple(dims), dtype=out_dtype, device=params[0].device)
        B.htucker_reconstruct(list(dims), tree, rk, Ul, Bl, Xhat=Xhat)
        ctx.spec = spec
        ctx.save_for_backward(*params)
        return Xhat

    @staticmethod
    def backward(ctx, H):
        dims, tree, ranks, leaves, internal = ctx.spec
        params = ctx.saved_tensors
        n = tree.num_nodes
        Ul = [None] * n
        Bl = [None] * n
        for t, p in zip(leaves, params[:len(leaves)]):
            Ul[t] = p
        for t, p in zip(internal, params[len(leaves):]):
            Bl[t] = p
        rk = [0] + [int(ranks[t]) for t in range(1, n)]
        Bbar = [torch.empty_like(b) if b is not None else None for b in Bl]
        Ubar = [torch.empty_like(u) if u is not None else None for u in Ul]
        Hc = H.contiguous()
        if Hc.dtype not in (torch.float32, torch.float64):
            Hc = Hc.double()
        B.htucker_reconstruct_vjp(list(dims), tree, rk, Ul, Bl, Hc, Bbar, Ubar)
        return (None, None, *[Ubar[t] for t in leaves], *[Bbar[t] for t in internal])


def htucker_full(dims, tree, ranks, U: dict, Bd: dict, out_dtype=torch.float64):
    """Differentiable full tensor of the format (leaf bases U[t], transfer
    tensors Bd[t] for internal nodes including the root 0, FP64)."""
    leaves = [t for t in range(1, tree.num_nodes) if tree.is_leaf(t)]
    internal = [t for t in range(tree.num_nodes) if not tree.is_leaf(t)]
    spec = (tuple(dims), tree, dict(ranks), leaves, internal)
    return HTuckerFull.apply(spec, out_dtype, *[U[t] for t in leaves], *[Bd[t] for t in internal])


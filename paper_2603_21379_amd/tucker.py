"""Sub-R-HOSVD and Sub-R-RtL-HT pipelines over the C ABI.

These functions only allocate outputs (torch device memory) and call the
library entry points in order; every arithmetic step runs in libtkmi's HIP
kernels.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

from . import binding as B


def upload_sketches(sketches, device, fdtype: torch.dtype):
    """Host sketch operands (objects with .idx int64 [s], .omega [s x ell]) to
    device tensors (idx int64, omega in the factor dtype).  A sketch whose idx
    covers every column is passed as idx=None (the dense sketch)."""
    out = []
    for sk, ncols in sketches:
        idx = None if len(sk.idx) == ncols else torch.from_numpy(sk.idx).to(device)
        om = torch.from_numpy(sk.omega).to(device=device, dtype=fdtype).contiguous()
        out.append((idx, om))
    return out


def mode_sketches_to_device(sketches, dims, device, fdtype):
    N = math.prod(dims)
    return upload_sketches([(s, N // n) for s, n in zip(sketches, dims)], device, fdtype)


@dataclass
class TuckerResult:
    G: torch.Tensor
    F: list          # factors used for the core (U_k, or span-Q_k bases)
    Q: list          # FP64 orthonormal bases Q_k
    Y: list
    info: torch.Tensor


def sub_r_hosvd(X: torch.Tensor, ranks, sk_dev, core_factor: str = "U", ws=None) -> TuckerResult:
    """Algorithm 1 on the GPU.  core_factor "U": r_k columns; "Q": ell_k
    columns spanning Range(Q_k)."""
    dims = list(X.shape)
    d = len(dims)
    fdt = B.factor_torch_dtype(X.dtype)
    dev = X.device
    Z = [torch.empty(n, om.shape[1], dtype=torch.float64, device=dev)
         for n, (_, om) in zip(dims, sk_dev)]
    Y = [torch.empty(n, om.shape[0], dtype=X.dtype, device=dev) for n, (_, om) in zip(dims, sk_dev)]
    B.tucker_sketch_all_modes(X, sk_dev, Z, Y, ws=ws)
    cols = [int(r) if core_factor == "U" else z.shape[1] for r, z in zip(ranks, Z)]
    F = [torch.empty(n, c, dtype=fdt, device=dev) for n, c in zip(dims, cols)]
    info = torch.zeros(d, dtype=torch.int32, device=dev)
    B.tucker_qr(Z, Y, r=cols, U=F, info=info, ws=ws)
    G = torch.empty(cols, dtype=fdt, device=dev)
    B.tucker_core(X, F, G, ws=ws)
    return TuckerResult(G, F, Z, Y, info)


def residual(X: torch.Tensor, G: torch.Tensor, F, ws=None):
    """(||X - X_hat||^2, ||X||^2) in FP64, computed on the GPU."""
    r2 = torch.zeros(2, dtype=torch.float64, device=X.device)
    B.tucker_reconstruct(list(X.shape), G, F, Xref=X, resid2=r2, ws=ws)
    return r2


def rel_error(X, G, F, ws=None) -> float:
    r2 = residual(X, G, F, ws=ws).cpu()
    return math.sqrt(float(r2[0]) / float(r2[1]))


def reconstruct(dims, G, F, ws=None) -> torch.Tensor:
    out = torch.empty(dims, dtype=G.dtype, device=G.device)
    B.tucker_reconstruct(list(dims), G, F, Xhat=out, ws=ws)
    return out


@dataclass
class HTResult:
    U: dict
    B: dict
    info: torch.Tensor


def sub_r_rtl_ht(X: torch.Tensor, tree, ranks: dict, sk_dev: dict, ws=None) -> HTResult:
    """Algorithm 2 on the GPU.  ranks[t] and sk_dev[t] for every non-root node."""
    dims = list(X.shape)
    fdt = torch.float64  # H-Tucker bases and transfers are FP64 for every tensor dtype
    dev = X.device
    n = tree.num_nodes
    nS = {t: math.prod(dims[k] for k in tree.modes(t)) for t in range(n)}
    U = [None] + [torch.empty(nS[t], ranks[t], dtype=fdt, device=dev) for t in range(1, n)]
    Bt = [None] * n
    for t in range(n):
        if not tree.is_leaf(t):
            rt = 1 if t == 0 else ranks[t]
            Bt[t] = torch.empty(rt, ranks[tree.left[t]], ranks[tree.right[t]], dtype=fdt, device=dev)
    info = torch.zeros(n, dtype=torch.int32, device=dev)
    rk = [0] + [ranks[t] for t in range(1, n)]
    sk = [None] + [sk_dev[t] for t in range(1, n)]
    B.htucker_decompose(X, tree, rk, sk, U, Bt, info=info, ws=ws)
    return HTResult({t: U[t] for t in range(1, n)},
                    {t: Bt[t] for t in range(n) if Bt[t] is not None}, info)


def _ht_lists(tree, ranks, U: dict, Bd: dict):
    n = tree.num_nodes
    Ul = [U[t].contiguous() if tree.is_leaf(t) else None for t in range(n)]
    Bl = [Bd[t].contiguous() if not tree.is_leaf(t) else None for t in range(n)]
    return [0] + [int(ranks[t]) for t in range(1, n)], Ul, Bl


def ht_reconstruct(dims, tree, ranks: dict, U: dict, Bd: dict, Xref=None, out_dtype=None, ws=None):
    """Full tensor of an H-Tucker format (leaf bases U, transfers Bd, FP64 on
    the device) in out_dtype, and/or [||Xref - Xhat||^2, ||Xref||^2]."""
    rk, Ul, Bl = _ht_lists(tree, ranks, U, Bd)
    dev = Bl[0].device
    Xhat = torch.empty(tuple(dims), dtype=out_dtype, device=dev) if out_dtype is not None else None
    r2 = torch.empty(2, dtype=torch.float64, device=dev) if Xref is not None else None
    B.htucker_reconstruct(list(dims), tree, rk, Ul, Bl, Xref=Xref, Xhat=Xhat, resid2=r2, ws=ws)
    return Xhat, r2


def ht_rel_error(X, tree, ranks: dict, U: dict, Bd: dict, ws=None) -> float:
    _, r2 = ht_reconstruct(list(X.shape), tree, ranks, U, Bd, Xref=X, ws=ws)
    v = r2.cpu()
    return float(math.sqrt(v[0] / v[1]))


def ht_reconstruct_vjp(dims, tree, ranks: dict, U: dict, Bd: dict, H, ws=None):
    """(dL/dB_t for internal nodes, dL/dU_t for leaves) given H = dL/dXhat."""
    rk, Ul, Bl = _ht_lists(tree, ranks, U, Bd)
    Bbar = [torch.empty_like(b) if b is not None else None for b in Bl]
    Ubar = [torch.empty_like(u) if u is not None else None for u in Ul]
    B.htucker_reconstruct_vjp(list(dims), tree, rk, Ul, Bl, H.contiguous(), Bbar, Ubar, ws=ws)
    n = tree.num_nodes
    return ({t: Bbar[t] for t in range(n) if Bbar[t] is not None},
            {t: Ubar[t] for t in range(n) if Ubar[t] is not None})

"""Sub-R-RtL-HT (Algorithm 2 of the paper), FP64.

Leaves: the factor steps of Sub-R-HOSVD without the core.  Every internal
non-root node S (levels z-1 .. 1): sample w_S columns of X^(S), sketch with a
Gaussian, orthonormal basis Q_S, W_S from the SVD of Q_S^T Y_S, U_S = Q_S W_S,
and the transfer tensor B_S(i,j,k) = <U_S(:,i), U_Sl(:,j) kron U_Sr(:,k)>
(Section 4, transfer-tensor equation).  Root: B_R(1,j,k) = <vec X,
U_Rl(:,j) kron U_Rr(:,k)> (Section 4, root transfer equation).

The dimension tree is an input (heap-indexed nodes with contiguous mode
ranges; left child = first half of the modes).
"""
from __future__ import annotations

import math

import numpy as np

from .tucker import orth, range_sketch, w_step


def _node_dims(dims, tree, t):
    modes = tree.modes(t)
    A = int(np.prod(dims[:modes[0]], dtype=np.int64))
    nS = int(np.prod([dims[k] for k in modes], dtype=np.int64))
    B = int(np.prod(dims[modes[-1] + 1:], dtype=np.int64))
    return A, nS, B


def gather_node(X: np.ndarray, tree, t: int, idx: np.ndarray, to64=None) -> np.ndarray:
    """Y_S = X^(S) E_S for a node S of contiguous modes: column j of X^(S) is
    X[a, :, b] of X viewed as (n_before, n_S, n_after), (a, b) = divmod(j, n_after).
    The sampled fibers are taken first and then upcast exactly (`to64`)."""
    to64 = to64 or (lambda v: np.asarray(v, dtype=np.float64))
    A, nS, B = _node_dims(X.shape, tree, t)
    X3 = X.reshape(A, nS, B)
    a, b = np.divmod(np.asarray(idx, dtype=np.int64), B)
    return to64(X3[a, :, b].T.copy())


def kron_cols(V: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Columns v_j kron w_k ordered (j, k) C-order; (v kron w)[a n_w + b] = v_a w_b."""
    return np.einsum("aj,bk->abjk", V, W).reshape(V.shape[0] * W.shape[0], -1)


def transfer_tensor(US: np.ndarray, Ul: np.ndarray, Ur: np.ndarray) -> np.ndarray:
    """B_S(i,j,k) = <U_S(:,i), U_l(:,j) kron U_r(:,k)>, shape (r_S, r_l, r_r)."""
    B = US.T @ kron_cols(Ul, Ur)
    return B.reshape(US.shape[1], Ul.shape[1], Ur.shape[1])


def root_transfer(X: np.ndarray, tree, Ul: np.ndarray, Ur: np.ndarray) -> np.ndarray:
    """B_R(1,j,k) = <vec X, U_Rl(:,j) kron U_Rr(:,k)> = (U_Rl^T X^(Rl) U_Rr)[j,k]."""
    nl = Ul.shape[0]
    Xm = np.asarray(X, dtype=np.float64).reshape(nl, -1)
    return (Ul.T @ Xm @ Ur)[None]


def sub_r_rtl_ht(X: np.ndarray, tree, ranks: dict, sketches: dict):
    """Algorithm 2.  ranks[t] and sketches[t] for every non-root node t.
    Returns (explicit bases U[t], transfers B[t] for internal nodes incl. the
    root t=0, Q[t])."""
    X = np.asarray(X, dtype=np.float64)
    U, Q, B = {}, {}, {}
    # all node bases come from X directly (root-to-leaves scheme), leaves first
    order = sorted(range(1, tree.num_nodes), key=lambda t: -tree.level[t])
    for t in order:
        Y = gather_node(X, tree, t, sketches[t].idx)
        Z = range_sketch(Y, sketches[t].omega)
        Q[t] = orth(Z)
        _, U[t], _ = w_step(Q[t], Y, ranks[t])
    for t in order:
        if not tree.is_leaf(t):
            B[t] = transfer_tensor(U[t], U[tree.left[t]], U[tree.right[t]])
    B[0] = root_transfer(X, tree, U[tree.left[0]], U[tree.right[0]])
    return U, B, Q


def ht_bases(tree, leaf_bases: dict, B: dict) -> dict:
    """Nested bases U_S = (U_Sl kron U_Sr) (B_S^(1))^T for every non-root node."""
    out = {}

    def basis(t):
        if t in out:
            return out[t]
        if tree.is_leaf(t):
            out[t] = leaf_bases[t]
        else:
            Bt = B[t]
            out[t] = kron_cols(basis(tree.left[t]), basis(tree.right[t])) @ \
                Bt.reshape(Bt.shape[0], -1).T
        return out[t]

    for t in range(1, tree.num_nodes):
        basis(t)
    return out


def ht_full(dims, tree, leaf_bases: dict, B: dict) -> np.ndarray:
    """Full tensor of the H-Tucker format: X^(Rl) = U_Rl B_R(1,:,:) U_Rr^T with
    nested bases (Section 4, nestedness property)."""
    nb = ht_bases(tree, leaf_bases, B)
    Xm = nb[tree.left[0]] @ B[0][0] @ nb[tree.right[0]].T
    return Xm.reshape(dims)


def ht_rel_error(X: np.ndarray, tree, U: dict, B: dict) -> float:
    X = np.asarray(X, dtype=np.float64)
    leaves = {t: U[t] for t in U if tree.is_leaf(t)}
    Xh = ht_full(X.shape, tree, leaves, B)
    return float(math.sqrt(np.sum((X - Xh) ** 2) / np.sum(X ** 2)))


def ht_residuals_streamed(X: np.ndarray, tree, formats, to64=None, rows: int = 512):
    """Squared residuals ||X - X_hat_f||_F^2 of several H-Tucker formats
    f = (leaf bases, transfers) and ||X||_F^2, in one pass over row blocks of
    the root matricisation X^(Rl) (Section 4, root relation): a block of rows
    of X_hat_f^(Rl) is (U_Rl^nest[rows] B_R) (U_Rr^nest)^T with nested bases
    from `ht_bases`.  Blocks are upcast exactly with `to64`.  Returns
    (list of squared residuals, squared norm)."""
    to64 = to64 or (lambda a: np.asarray(a, dtype=np.float64))
    L, R = tree.left[0], tree.right[0]
    parts = []
    for U, B in formats:
        nb = ht_bases(tree, {t: U[t] for t in U if tree.is_leaf(t)}, B)
        parts.append((nb[L] @ B[0][0], nb[R]))
    nl = parts[0][0].shape[0]
    Xm = X.reshape(nl, -1)
    r2 = [0.0] * len(formats)
    n2 = 0.0
    for r0 in range(0, nl, rows):
        xb = to64(Xm[r0:r0 + rows])
        n2 += float(np.sum(xb * xb))
        for f, (Tl, Vr) in enumerate(parts):
            d = xb - Tl[r0:r0 + rows] @ Vr.T
            r2[f] += float(np.sum(d * d))
    return r2, n2


def ht_full_vjp(dims, tree, leaf_bases: dict, B: dict, H: np.ndarray):
    """Vector-Jacobian product of the H-Tucker format's full tensor (ht_full)
    with respect to its parameters, the leaf bases and the transfer tensors.

    The paper does not differentiate the format; this is the chain rule
    through its two defining relations (Section 4): at the root
    X^(Rl) = U_Rl B_R U_Rr^T, so with H^(Rl) the adjoint viewed the same way
        B_R_bar = U_Rl^T H U_Rr,  U_Rl_bar = H U_Rr B_R^T,  U_Rr_bar = H^T U_Rl B_R,
    and at an internal node U_S = (U_Sl kron U_Sr) (B_S^(1))^T (nestedness), so
    with K = U_Sl kron U_Sr (columns (j, k) C-order)
        B_S_bar^(1) = U_S_bar^T K,  K_bar = U_S_bar B_S^(1),
        U_Sl_bar[a, j] = sum_{b,k} K_bar[(a,b), (j,k)] U_Sr[b, k],
        U_Sr_bar[b, k] = sum_{a,j} K_bar[(a,b), (j,k)] U_Sl[a, j],
    applied from the root's children down to the leaves (each node's basis
    feeds only its parent, so every adjoint has one term).  Returns
    (B_bar for every internal node including the root 0, U_bar for the leaves),
    FP64."""
    nb = ht_bases(tree, leaf_bases, B)
    L, R = tree.left[0], tree.right[0]
    Hm = np.asarray(H, dtype=np.float64).reshape(nb[L].shape[0], nb[R].shape[0])
    BR = B[0][0]
    Bbar = {0: (nb[L].T @ Hm @ nb[R])[None]}
    Ubar = {L: Hm @ nb[R] @ BR.T, R: Hm.T @ nb[L] @ BR}
    order = sorted(range(1, tree.num_nodes), key=lambda t: tree.level[t])   # parents first
    for t in order:
        if tree.is_leaf(t):
            continue
        l, r = tree.left[t], tree.right[t]
        Ul, Ur = nb[l], nb[r]
        rS, rl, rr = B[t].shape
        K = kron_cols(Ul, Ur)
        B1 = B[t].reshape(rS, rl * rr)
        Bbar[t] = (Ubar[t].T @ K).reshape(rS, rl, rr)
        Kbar = (Ubar[t] @ B1).reshape(Ul.shape[0], Ur.shape[0], rl, rr)
        Ubar[l] = np.einsum("abjk,bk->aj", Kbar, Ur)
        Ubar[r] = np.einsum("abjk,aj->bk", Kbar, Ul)
    return Bbar, {t: Ubar[t] for t in Ubar if tree.is_leaf(t)}


"""Tensor primitives of Section 2.2 (unfoldings and TTM), plain NumPy, FP64."""
from __future__ import annotations

import numpy as np


def unfold(X: np.ndarray, k: int) -> np.ndarray:
    """Mode-k matricization (Section 2.2, Definition of unfolding).

    X^(k)(i_k, j) = X(i_1..i_d) with j the C-order linear index of the other
    modes; size n_k x n_{!=k}.
    """
    return np.moveaxis(X, k, 0).reshape(X.shape[k], -1)


def fold(M: np.ndarray, k: int, dims) -> np.ndarray:
    """Inverse of `unfold`."""
    dims = tuple(dims)
    rest = dims[:k] + dims[k + 1:]
    return np.moveaxis(M.reshape((dims[k],) + rest), 0, k)


def unfold_set(X: np.ndarray, S) -> np.ndarray:
    """Multi-mode matricization X^(S) (Section 2.2): rows C-ordered over the
    modes of S (ascending), columns C-ordered over the complement."""
    S = sorted(S)
    rest = [k for k in range(X.ndim) if k not in S]
    nS = int(np.prod([X.shape[k] for k in S]))
    return np.transpose(X, S + rest).reshape(nS, -1)


def ttm(X: np.ndarray, U: np.ndarray, k: int) -> np.ndarray:
    """TTM product X x_k U for U of size m x n_k (Section 2.2, TTM definition):
    B(.., j, ..) = sum_{i_k} X(.., i_k, ..) U(j, i_k), i.e. B^(k) = U X^(k)."""
    dims = list(X.shape)
    out = U @ unfold(X, k)
    dims[k] = U.shape[0]
    return fold(out, k, dims)


def multi_ttm(X: np.ndarray, Us) -> np.ndarray:
    """(U_1, .., U_d) X = X x_1 U_1 x_2 ... x_d U_d (Section 2.2)."""
    for k, U in enumerate(Us):
        X = ttm(X, U, k)
    return X

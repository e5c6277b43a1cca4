"""Deterministic brute-force references and the paper's error bounds.

Only for tiny inputs: full SVDs of unfoldings.
"""
from __future__ import annotations

import math

import numpy as np

from .htucker import root_transfer, transfer_tensor
from .tensor import unfold, unfold_set
from .tucker import canonical_signs, core


def t_hosvd(X: np.ndarray, ranks):
    """Truncated HOSVD (Section 3): U_k = dominant r_k left singular vectors
    of X^(k), core S = (U_1^T..U_d^T) X."""
    X = np.asarray(X, dtype=np.float64)
    Us = []
    for k, r in enumerate(ranks):
        U, _, _ = np.linalg.svd(unfold(X, k), full_matrices=False)
        U = U[:, :r]
        Us.append(U * canonical_signs(U))
    return core(X, Us), Us


def unfolding_tail(A: np.ndarray, c: int) -> float:
    """sqrt(sum_{i > c} sigma_i(A)^2)."""
    s = np.linalg.svd(A, compute_uv=False)
    return float(math.sqrt(np.sum(s[c:] ** 2)))


def lower_bound_sq(X: np.ndarray, cs) -> float:
    """Any Tucker approximation with c_k columns per mode has relative squared
    error >= max_k sum_{i>c_k} sigma_i(X^(k))^2 / ||X||^2 (Eckart-Young on
    each unfolding, since X_hat^(k) has rank <= c_k)."""
    X = np.asarray(X, dtype=np.float64)
    nx2 = float(np.sum(X ** 2))
    return max(unfolding_tail(unfold(X, k), c) ** 2 for k, c in enumerate(cs)) / nx2


def rhosvd_factor(d: int, ranks, p: int) -> float:
    """(d + sum r_k / (p - 1))^(1/2) of the R-HOSVD expectation bound (Section 3)."""
    return math.sqrt(d + sum(ranks) / (p - 1))


def rangefinder_factor(k: int, p: int) -> float:
    """(1 + k/(p-1))^(1/2) of the Gaussian range-finder bound (Section 2.3)."""
    return math.sqrt(1.0 + k / (p - 1))


def thm34_factor(ranks, p: int, deltas, etas) -> float:
    """(d + sum_k 3^(3/2) r_k (1+eta_k)(r_k+p) / ((1-delta_k)(p+1)))^(1/2),
    Theorem 3.4 (bound for Sub-R-HOSVD under the sampling event)."""
    d = len(ranks)
    s = sum(3 ** 1.5 * r * (1 + e) * (r + p) / ((1 - dl) * (p + 1))
            for r, dl, e in zip(ranks, deltas, etas))
    return math.sqrt(d + s)


def sampling_event(X: np.ndarray, k: int, r: int, idx: np.ndarray):
    """(delta_k, eta_k) realised by a fiber sample: from the right singular
    vectors V1 (first r) and V2 (rest) of X^(k) (Lemma 3.1 / event B_k):
    sigma_r(V1^T E) = sqrt((1-delta) s/m), sigma_1(V2^T E) = sqrt((1+eta) s/m)."""
    A = unfold(np.asarray(X, dtype=np.float64), k)
    m = A.shape[1]
    s = len(idx)
    _, _, Vt = np.linalg.svd(A, full_matrices=False)
    V1E = Vt[:r][:, idx]
    V2E = Vt[r:][:, idx]
    smin = np.linalg.svd(V1E, compute_uv=False)[-1]
    smax = np.linalg.svd(V2E, compute_uv=False)[0] if V2E.shape[0] else 0.0
    delta = 1.0 - smin ** 2 * m / s
    eta = max(0.0, smax ** 2 * m / s - 1.0)
    return delta, eta


def rtl_ht(X: np.ndarray, tree, ranks: dict):
    """Deterministic RtL-HT (Section 4): for every non-root node the dominant
    r_S left singular vectors of X^(S); transfers from the explicit bases;
    root from vec X."""
    X = np.asarray(X, dtype=np.float64)
    U = {}
    for t in range(1, tree.num_nodes):
        Ut, _, _ = np.linalg.svd(unfold_set(X, tree.modes(t)), full_matrices=False)
        Ut = Ut[:, :ranks[t]]
        U[t] = Ut * canonical_signs(Ut)
    B = {}
    for t in range(1, tree.num_nodes):
        if not tree.is_leaf(t):
            B[t] = transfer_tensor(U[t], U[tree.left[t]], U[tree.right[t]])
    B[0] = root_transfer(X, tree, U[tree.left[0]], U[tree.right[0]])
    return U, B


def ht_tails_sq(X: np.ndarray, tree, ranks: dict) -> list:
    """sum_{i > r_S} sigma_i(X^(S))^2 for every non-root node S."""
    X = np.asarray(X, dtype=np.float64)
    return [unfolding_tail(unfold_set(X, tree.modes(t)), ranks[t]) ** 2
            for t in range(1, tree.num_nodes)]

"""Closed-form gradients of the Tucker core projection and reconstruction.

The paper does not differentiate its method; this follows directly from the
TTM definition (Section 2.2): with C(X, F) = X x_1 F_1^T .. x_d F_d^T and
R(G, F) = G x_1 F_1 .. x_d F_d (F_k free n_k x c_k matrices) and
L = ||X - R(C(X, F), F)||_F^2:

  core VJP, given G_bar:     X_bar  = G_bar x_1 F_1 .. x_d F_d
                             F_bar_k = (X x_{j!=k} F_j^T)^(k) (G_bar^(k))^T
  reconstruct VJP, given H:  G_bar  = H x_1 F_1^T .. x_d F_d^T
                             F_bar_k = H^(k) ((G x_{j!=k} F_j)^(k))^T
  with H = dL/dX_hat = -2 (X - X_hat) and the direct term dL/dX = 2 (X - X_hat).
"""
from __future__ import annotations

import numpy as np

from .tensor import multi_ttm, ttm, unfold


def _all_but(X, mats, k):
    for j, M in enumerate(mats):
        if j != k:
            X = ttm(X, M, j)
    return X


def core_vjp(X: np.ndarray, Fs, Gbar: np.ndarray):
    Xbar = multi_ttm(Gbar, Fs)
    FT = [F.T for F in Fs]
    Fbar = [unfold(_all_but(X, FT, k), k) @ unfold(Gbar, k).T for k in range(X.ndim)]
    return Xbar, Fbar


def reconstruct_vjp(G: np.ndarray, Fs, H: np.ndarray):
    Gbar = multi_ttm(H, [F.T for F in Fs])
    Fbar = [unfold(H, k) @ unfold(_all_but(G, Fs, k), k).T for k in range(G.ndim)]
    return Gbar, Fbar


def loss_and_grads(X: np.ndarray, Fs):
    """L = ||X - R(C(X,F),F)||^2 and (dL/dX, [dL/dF_k])."""
    X = np.asarray(X, dtype=np.float64)
    G = multi_ttm(X, [F.T for F in Fs])
    Xh = multi_ttm(G, Fs)
    D = X - Xh
    L = float(np.sum(D * D))
    H = -2.0 * D
    Gbar, Fr = reconstruct_vjp(G, Fs, H)
    Xc, Fc = core_vjp(X, Fs, Gbar)
    dX = 2.0 * D + Xc
    dF = [a + b for a, b in zip(Fr, Fc)]
    return L, dX, dF

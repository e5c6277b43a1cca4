"""Sub-R-HOSVD (Algorithm 1 of the paper), step by step, FP64.

For every mode k: sample s_k mode-k fibers into Y_k = X^(k) E_k
(Section 3.1, fiber sampling without forming the unfolding), sketch with a
Gaussian Omega_k (s_k x (r_k+p)), orthonormal basis Q_k of Range(Y_k Omega_k),
W_k = dominant r_k left singular vectors of Q_k^T Y_k, U_k = Q_k W_k; then the
core S = (U_1^T, .., U_d^T) X.  The fiber indices and Omega_k are inputs
(drawn by the caller), so the oracle itself draws nothing.
"""
from __future__ import annotations

import math

import numpy as np

from .tensor import multi_ttm, unfold


def gather_fibers(X: np.ndarray, k: int, idx: np.ndarray, to64=None) -> np.ndarray:
    """Y_k = X^(k) E_k: the columns idx of the mode-k unfolding, taken as
    mode-k fibers of X (Section 3.1).  Column j of X^(k) is the fiber
    X[a, :, b] of X viewed as (n_{<k}, n_k, n_{>k}) with (a, b) = divmod(j, n_{>k}).
    `to64` upcasts stored values exactly (applied to the gathered fibers only)."""
    to64 = to64 or (lambda v: np.asarray(v, dtype=np.float64))
    dims = X.shape
    A = int(np.prod(dims[:k], dtype=np.int64))
    B = int(np.prod(dims[k + 1:], dtype=np.int64))
    X3 = X.reshape(A, dims[k], B)
    a, b = np.divmod(np.asarray(idx, dtype=np.int64), B)
    return to64(X3[a, :, b].T.copy())


def range_sketch(Y: np.ndarray, omega: np.ndarray) -> np.ndarray:
    """Z_k = Y_k Omega_k (Alg. 1, range finder of Section 2.3)."""
    return Y @ omega


def orth(Z: np.ndarray) -> np.ndarray:
    """Orthonormal basis of Range(Z): thin Householder QR with R_ii >= 0
    (Alg. 1, orthonormal basis step).  Always returns Z.shape[1] columns."""
    Q, R = np.linalg.qr(Z, mode="reduced")
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s


def canonical_signs(U: np.ndarray) -> np.ndarray:
    """+1/-1 per column so that each column's largest-magnitude entry (first
    one on ties) is positive.  The paper leaves singular-vector signs open."""
    j = np.argmax(np.abs(U), axis=0)
    s = np.sign(U[j, np.arange(U.shape[1])])
    s[s == 0] = 1.0
    return s


def w_step(Q: np.ndarray, Y: np.ndarray, r: int):
    """W_k = dominant r left singular vectors of Q^T Y, U_k = Q W_k (Alg. 1)."""
    M = Q.T @ Y
    Wfull, sv, _ = np.linalg.svd(M, full_matrices=False)
    W = Wfull[:, :r]
    U = Q @ W
    s = canonical_signs(U)
    return W * s, U * s, sv


def sub_r_hosvd(X: np.ndarray, ranks, sketches, core_factor: str = "U"):
    """Algorithm 1 on a float64 view of X.

    sketches[k] provides idx (sorted fiber indices) and omega (s_k x ell_k).
    core_factor "U" projects on U_k (r_k columns, Alg. 1); "Q" on Q_k
    (ell_k columns).  Returns (G, U list, Q list, Y list, Z list).
    """
    X = np.asarray(X, dtype=np.float64)
    Us, Qs, Ys, Zs = [], [], [], []
    for k in range(X.ndim):
        Y = gather_fibers(X, k, sketches[k].idx)
        Z = range_sketch(Y, sketches[k].omega)
        Q = orth(Z)
        _, U, _ = w_step(Q, Y, ranks[k])
        Us.append(U), Qs.append(Q), Ys.append(Y), Zs.append(Z)
    F = Us if core_factor == "U" else Qs
    return core(X, F), Us, Qs, Ys, Zs


def core(X: np.ndarray, Fs) -> np.ndarray:
    """G = (F_1^T, .., F_d^T) X (Alg. 1, core step)."""
    return multi_ttm(np.asarray(X, dtype=np.float64), [F.T for F in Fs])


def core_streamed(X: np.ndarray, Fs, to64=None, slab: int = 1) -> np.ndarray:
    """Same core, accumulated over slabs of mode 0: by linearity of the TTM,
    G = sum_slabs (F_1[slab]^T, F_2^T, .., F_d^T) X[slab].  Lets the oracle
    handle tensors whose FP64 copy does not fit in memory; `to64` upcasts a
    stored slab exactly."""
    to64 = to64 or (lambda a: np.asarray(a, dtype=np.float64))
    G = None
    for i in range(0, X.shape[0], slab):
        part = core(to64(X[i:i + slab]), [Fs[0][i:i + slab]] + list(Fs[1:]))
        G = part if G is None else G + part
    return G


def core_chunked(X: np.ndarray, Fs, to64=None, rows: int = 1 << 16) -> np.ndarray:
    """Same core, contracting the last mode first: X viewed as the
    (N / n_d) x n_d matrix times F_d (a matrix product over chunks of rows,
    each upcast exactly with `to64`), then the other modes of the much
    smaller result.  For tensors whose FP64 copy does not fit in memory."""
    to64 = to64 or (lambda a: np.asarray(a, dtype=np.float64))
    dims = X.shape
    Fd = np.asarray(Fs[-1], dtype=np.float64)
    M = X.reshape(-1, dims[-1])
    T = np.empty((M.shape[0], Fd.shape[1]))
    for r0 in range(0, M.shape[0], rows):
        T[r0:r0 + rows] = to64(M[r0:r0 + rows]) @ Fd
    T = T.reshape(dims[:-1] + (Fd.shape[1],))
    return multi_ttm(T, [F.T for F in Fs[:-1]] + [np.eye(Fd.shape[1])])


def reconstruct(G: np.ndarray, Fs) -> np.ndarray:
    """X_hat = (F_1, .., F_d) G (Tucker format, Section 3)."""
    return multi_ttm(G, Fs)


def rel_error(X: np.ndarray, G: np.ndarray, Fs, to64=None, slab: int | None = None) -> float:
    """||X - (F_1..F_d) G||_F / ||X||_F, formed explicitly (slab-wise along
    mode 0 when `slab` is given)."""
    to64 = to64 or (lambda a: np.asarray(a, dtype=np.float64))
    if slab is None:
        Xf = to64(X)
        return float(np.linalg.norm(Xf - reconstruct(G, Fs)) / np.linalg.norm(Xf))
    num = den = 0.0
    for i in range(0, X.shape[0], slab):
        xs = to64(X[i:i + slab])
        xh = reconstruct(G, [Fs[0][i:i + slab]] + list(Fs[1:]))
        num += float(np.sum((xs - xh) ** 2))
        den += float(np.sum(xs ** 2))
    return math.sqrt(num / den)


def sq_norm(X: np.ndarray, to64=None, rows: int = 1 << 22) -> float:
    """||X||_F^2 in FP64, summed over chunks of the flattened tensor (each
    chunk upcast exactly with `to64`)."""
    to64 = to64 or (lambda a: np.asarray(a, dtype=np.float64))
    v = X.reshape(-1)
    total = 0.0
    for i in range(0, v.shape[0], rows):
        c = to64(v[i:i + rows])
        total += float(np.dot(c, c))
    return total


def rel_error_orthonormal(G: np.ndarray, normX2: float) -> float:
    """||X - (F_1..F_d) G||_F / ||X||_F for G = (F_1^T..F_d^T) X with every
    F_k orthonormal (Tucker format, Section 3): X_hat is then the orthogonal
    projection of X onto the product of the factor ranges, so
    ||X - X_hat||^2 = ||X||^2 - ||G||^2.  The subtraction cancels about
    log10(1 / eps^2) digits: with FP64 sums the result carries a relative
    error of about 1e-15 / eps^2, so it is refused below eps = 1e-4."""
    g2 = float(np.sum(np.asarray(G, dtype=np.float64) ** 2))
    e2 = 1.0 - g2 / normX2
    if e2 < 1e-8:
        raise ValueError(f"relative error {max(e2, 0.0) ** 0.5:.2e} < 1e-4: use rel_error")
    return math.sqrt(e2)


def mode_errors(X: np.ndarray, Fs):
    """eps_k = ||X^(k) - F_k F_k^T X^(k)||_F / ||X||_F for every mode."""
    X = np.asarray(X, dtype=np.float64)
    nx = np.linalg.norm(X)
    out = []
    for k, F in enumerate(Fs):
        A = unfold(X, k)
        out.append(float(np.linalg.norm(A - F @ (F.T @ A)) / nx))
    return out


def projector_distance(F1: np.ndarray, F2: np.ndarray) -> float:
    """||F1 F1^T - F2 F2^T||_F / sqrt(2 c): sign- and rotation-invariant.

    For n > 8192 rows the n x n difference is not formed: for bases with
    orthonormal columns and the same c, ||F1 F1^T - F2 F2^T||_F^2 =
    2 ||F1 - F2 (F2^T F1)||_F^2 (twice the sum of the squared sines of the
    principal angles), a residual that is computed directly."""
    n, c = F1.shape
    if n <= 8192:
        P = F1 @ F1.T - F2 @ F2.T
        return float(np.linalg.norm(P) / math.sqrt(2 * c))
    R = F1 - F2 @ (F2.T @ F1)
    return float(np.linalg.norm(R) / math.sqrt(c))

"""Pins of the FP64 oracle for Sub-R-HOSVD (Algorithm 1) against what the
paper and the mathematics fix: definitions written out as loops, closed
forms, invariants, textbook special cases and the paper's error bounds."""
import itertools
import math

import numpy as np
import pytest

import oracle
import synthgen
from oracle import brute


def _lin(idx, dims):
    j = 0
    for i, n in zip(idx, dims):
        j = j * n + i
    return j


def test_unfold_matches_definition_loops():
    """X^(k)(i_k, j) = X(i), j = lexicographic index of the other modes (Section 2.2)."""
    rng = np.random.default_rng(0)
    dims = (2, 3, 4, 2)
    X = rng.standard_normal(dims)
    for k in range(4):
        A = oracle.unfold(X, k)
        rest = dims[:k] + dims[k + 1:]
        assert A.shape == (dims[k], math.prod(rest))
        for i in itertools.product(*[range(n) for n in dims]):
            j = _lin(i[:k] + i[k + 1:], rest)
            assert A[i[k], j] == X[i]


def test_unfold_set_matches_definition_loops():
    rng = np.random.default_rng(1)
    dims = (2, 3, 2, 3)
    X = rng.standard_normal(dims)
    for S in ([0, 1], [1, 2], [2, 3], [0, 1, 2]):
        A = oracle.unfold_set(X, S)
        rest = [k for k in range(4) if k not in S]
        for i in itertools.product(*[range(n) for n in dims]):
            r = _lin([i[k] for k in S], [dims[k] for k in S])
            c = _lin([i[k] for k in rest], [dims[k] for k in rest])
            assert A[r, c] == X[i]


def test_ttm_matches_definition_loops():
    rng = np.random.default_rng(2)
    dims = (3, 2, 4)
    X = rng.standard_normal(dims)
    U = rng.standard_normal((5, 2))
    B = oracle.ttm(X, U, 1)
    assert B.shape == (3, 5, 4)
    for a, j, c in itertools.product(range(3), range(5), range(4)):
        ref = sum(X[a, i, c] * U[j, i] for i in range(2))
        assert abs(B[a, j, c] - ref) < 1e-14


def test_gather_is_unfolding_columns_loops():
    rng = np.random.default_rng(3)
    dims = (3, 4, 2, 5)
    X = rng.standard_normal(dims)
    for k in range(4):
        ncols = math.prod(dims) // dims[k]
        idx = np.sort(rng.choice(ncols, 7, replace=False))
        Y = oracle.gather_fibers(X, k, idx)
        rest = dims[:k] + dims[k + 1:]
        for t, j in enumerate(idx):
            # invert the lexicographic index j of the other modes
            other, rem = [], int(j)
            for n in reversed(rest):
                other.append(rem % n)
                rem //= n
            other = other[::-1]
            for ik in range(dims[k]):
                full = tuple(other[:k]) + (ik,) + tuple(other[k:])
                assert Y[ik, t] == X[full]


def _run(X, ranks, p, s, seed, dense=False, core_factor="U"):
    dims = X.shape
    ells = synthgen.default_ell(dims, ranks, p)
    sk = synthgen.mode_sketches(dims, ells, s, cfg=100 + seed, omega_dtype="f64", dense=dense)
    return oracle.sub_r_hosvd(X, ranks, sk, core_factor=core_factor)


@pytest.mark.parametrize("core_factor", ["U", "Q"])
def test_exact_multilinear_rank_recovered(core_factor):
    """sigma = 0: Range(Y_k) = Range(X^(k)) (Section 3.1), so eps ~ 1e-12 (64^3, r = 8, p = 5)."""
    inp = synthgen.tucker_tensor((64, 64, 64), (8, 8, 8), 0.5, 0.0, cfg=1, dtype="f64")
    G, Us, Qs, _, _ = _run(inp.X, (8, 8, 8), 5, synthgen.default_s(inp.dims), 0,
                           core_factor=core_factor)
    F = Us if core_factor == "U" else Qs
    assert oracle.rel_error(inp.X, G, F) < 1e-12


def test_bases_orthonormal():
    inp = synthgen.tucker_tensor((64, 64, 64), (8, 8, 8), 0.5, 1e-6, cfg=1, dtype="f64")
    _, Us, Qs, _, _ = _run(inp.X, (8, 8, 8), 5, synthgen.default_s(inp.dims), 0)
    for F in Us + Qs:
        assert np.max(np.abs(F.T @ F - np.eye(F.shape[1]))) < 1e-13


def test_qr_is_a_qr():
    """Q R = Z with R upper triangular and R_ii > 0 (thin QR uniqueness)."""
    rng = np.random.default_rng(4)
    Z = rng.standard_normal((50, 9))
    Q = oracle.orth(Z)
    R = Q.T @ Z
    assert np.allclose(np.tril(R, -1), 0, atol=1e-13)
    assert np.all(np.diag(R) > 0)
    assert np.allclose(Q @ R, Z, atol=1e-13)


def test_order2_reduces_to_randomized_svd():
    """d = 2: the method is the randomized SVD of a matrix (Section 2.3); with a
    clear spectral gap U_1, U_2 span the dominant singular spaces."""
    rng = np.random.default_rng(5)
    m, n, r = 120, 90, 6
    Uo, _ = np.linalg.qr(rng.standard_normal((m, r)))
    Vo, _ = np.linalg.qr(rng.standard_normal((n, r)))
    A = Uo @ np.diag(np.geomspace(10, 1, r)) @ Vo.T + 1e-9 * rng.standard_normal((m, n))
    G, Us, _, _, _ = _run(A, (r, r), 6, [min(10 * m, n), min(10 * n, m)], 1)
    Ul, _, Vt = np.linalg.svd(A)
    assert oracle.projector_distance(Us[0], Ul[:, :r]) < 1e-6
    assert oracle.projector_distance(Us[1], Vt[:r].T) < 1e-6
    np.testing.assert_allclose(G, Us[0].T @ A @ Us[1], rtol=0, atol=1e-12)
    best = math.sqrt(np.sum(np.linalg.svd(A, compute_uv=False)[r:] ** 2))
    err = np.linalg.norm(A - Us[0] @ G @ Us[1].T)
    assert best * (1 - 1e-9) <= err <= brute.rhosvd_factor(2, (r, r), 6) * best


def test_full_basis_reconstructs_any_tensor():
    """ell_k = n_k with every fiber sampled: Q_k is a full basis, X_hat = X."""
    rng = np.random.default_rng(6)
    X = rng.standard_normal((6, 5, 7))
    G, _, Qs, _, _ = _run(X, (6, 5, 7), 0, [0, 0, 0], 2, dense=True, core_factor="Q")
    assert oracle.rel_error(X, G, Qs) < 1e-13


def test_dense_full_oversampling_equals_truncated_hosvd():
    """Every fiber sampled and ell_k = n_k: W_k picks the dominant left
    singular vectors of X^(k) exactly, i.e. the T-HOSVD (Section 3)."""
    inp = synthgen.tucker_tensor((10, 9, 8), (3, 3, 3), 0.5, 1e-3, cfg=7, dtype="f64")
    G, Us, _, _, _ = _run(inp.X, (3, 3, 3), 10, [0, 0, 0], 3, dense=True)
    Gt, Ut = brute.t_hosvd(inp.X, (3, 3, 3))
    for a, b in zip(Us, Ut):
        np.testing.assert_allclose(a, b, atol=1e-10)
    np.testing.assert_allclose(G, Gt, atol=1e-10)


def test_lower_bound_holds_on_every_draw():
    """Eckart-Young per unfolding: eps^2 >= max_k tail_k^2 / ||X||^2, any draw."""
    inp = synthgen.tucker_tensor((12, 11, 10), (4, 4, 4), 0.6, 3e-2, cfg=8, dtype="f64")
    lb = brute.lower_bound_sq(inp.X, (4, 4, 4))
    for seed in range(25):
        G, Us, _, _, _ = _run(inp.X, (4, 4, 4), 4, [40, 40, 40], seed)
        assert oracle.rel_error(inp.X, G, Us) ** 2 >= lb * (1 - 1e-12)


def test_mode_sum_inequality():
    """||X - X_hat||^2 <= sum_k ||(I - U_k U_k^T) X^(k)||^2 for orthonormal U_k
    (the lemma used in the proof of Theorem 3.4)."""
    inp = synthgen.tucker_tensor((12, 11, 10), (4, 4, 4), 0.6, 3e-2, cfg=8, dtype="f64")
    for seed in range(5):
        G, Us, _, _, _ = _run(inp.X, (4, 4, 4), 4, [40, 40, 40], seed)
        eps = oracle.rel_error(inp.X, G, Us)
        assert eps ** 2 <= sum(e ** 2 for e in oracle.mode_errors(inp.X, Us)) * (1 + 1e-12)


def _noisy(cfg=9):
    return synthgen.tucker_tensor((14, 13, 12), (4, 4, 4), 0.7, 5e-2, cfg=cfg, dtype="f64")


def test_dense_rangefinder_expectation_bound_q_core():
    """Dense Gaussian sketch, Q-core: E||X - X_hat||^2 <= sum_k (1 + r_k/(p-1)) tau_k^2
    (range-finder bound of Section 2.3 per mode, summed by the mode-sum lemma);
    mean over 25 draws as in the paper's protocol."""
    inp = _noisy()
    r, p = (4, 4, 4), 4
    X = inp.X
    taus = [brute.unfolding_tail(oracle.unfold(X, k), r[k]) ** 2 for k in range(3)]
    bound = sum(brute.rangefinder_factor(r[k], p) ** 2 * taus[k] for k in range(3))
    errs = []
    for seed in range(25):
        G, _, Qs, _, _ = _run(X, r, p, [0, 0, 0], seed, dense=True, core_factor="Q")
        errs.append(np.linalg.norm(X - oracle.reconstruct(G, Qs)) ** 2)
    assert np.mean(errs) <= bound


def test_rhosvd_expectation_bound_u_core():
    """Dense sketch, U-core (R-HOSVD): E||X - X_hat|| <= (d + sum r_k/(p-1))^(1/2)
    ||X - X*|| <= same factor times the T-HOSVD error (Section 3)."""
    inp = _noisy()
    r, p = (4, 4, 4), 4
    Gt, Ut = brute.t_hosvd(inp.X, r)
    ref = np.linalg.norm(inp.X - oracle.reconstruct(Gt, Ut))
    errs = []
    for seed in range(25):
        G, Us, _, _, _ = _run(inp.X, r, p, [0, 0, 0], seed, dense=True)
        errs.append(np.linalg.norm(inp.X - oracle.reconstruct(G, Us)))
    assert np.mean(errs) <= brute.rhosvd_factor(3, r, p) * ref
    # and the T-HOSVD itself is within sqrt(d) of its own error (sanity)
    assert min(errs) >= ref / math.sqrt(3) * 0.999


def test_sampled_theorem_3_4_bound():
    """Theorem 3.4 with delta_k, eta_k realised by each draw (taken as the
    worst over the 25 draws, so every draw lies in the event)."""
    inp = _noisy(10)
    r, p, s = (4, 4, 4), 4, [60, 60, 60]
    Gt, Ut = brute.t_hosvd(inp.X, r)
    ref = np.linalg.norm(inp.X - oracle.reconstruct(Gt, Ut))
    errs, deltas, etas = [], [0.0] * 3, [0.0] * 3
    for seed in range(25):
        dims = inp.dims
        ells = synthgen.default_ell(dims, r, p)
        sk = synthgen.mode_sketches(dims, ells, s, cfg=100 + seed, omega_dtype="f64")
        for k in range(3):
            dl, et = brute.sampling_event(inp.X, k, r[k], sk[k].idx)
            assert dl < 1.0
            deltas[k], etas[k] = max(deltas[k], dl), max(etas[k], et)
        G, Us, _, _, _ = oracle.sub_r_hosvd(inp.X, r, sk)
        errs.append(np.linalg.norm(inp.X - oracle.reconstruct(G, Us)))
    assert np.mean(errs) <= brute.thm34_factor(r, p, deltas, etas) * ref


def test_streamed_core_and_error_match_plain():
    inp = synthgen.tucker_tensor((9, 8, 7, 6), (3, 3, 3, 3), 0.7, 1e-2, cfg=11, dtype="f32")
    X64 = synthgen.to_f64(inp.X, "f32")
    _, Us, _, _, _ = _run(X64, (3, 3, 3, 3), 3, [30] * 4, 0)
    G = oracle.core(X64, Us)
    Gs = oracle.core_streamed(inp.X, Us, slab=2)
    np.testing.assert_allclose(Gs, G, rtol=0, atol=1e-12 * np.abs(G).max())
    e1 = oracle.rel_error(X64, G, Us)
    e2 = oracle.rel_error(inp.X, G, Us, slab=4)
    assert abs(e1 - e2) <= 1e-12 * e1


def test_projector_distance_invariances():
    rng = np.random.default_rng(12)
    Q, _ = np.linalg.qr(rng.standard_normal((20, 4)))
    Rot, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    assert oracle.projector_distance(Q, Q @ Rot) < 1e-14
    assert oracle.projector_distance(Q, -Q) < 1e-14
    Q2, _ = np.linalg.qr(rng.standard_normal((20, 4)))
    assert oracle.projector_distance(Q, Q2) > 0.1


def test_chunked_core_matches_plain_core():
    """The last-mode-first chunked core (row chunks not dividing the rows,
    one chunk, order 3 and 5) equals the plain multi-TTM core."""
    rng = np.random.default_rng(31)
    for dims, cols, rows in [((7, 9, 11), (3, 4, 5), 5), ((4, 5, 3, 6, 8), (2, 3, 3, 4, 5), 17),
                             ((6, 5, 4), (2, 2, 2), 1 << 20)]:
        X = rng.standard_normal(dims).astype(np.float32)
        Fs = [rng.standard_normal((n, c)) for n, c in zip(dims, cols)]
        ref = oracle.core(X.astype(np.float64), Fs)
        got = oracle.core_chunked(X, Fs, rows=rows)
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_projector_distance_large_n_form_matches_dense():
    """The principal-angle form used above 8192 rows equals the dense
    projector difference (orthonormal bases of equal dimension)."""
    rng = np.random.default_rng(32)
    n, c = 8200, 5
    A = np.linalg.qr(rng.standard_normal((n, c)))[0]
    for eps in (1e-3, 1e-7):
        Bm = np.linalg.qr(A + eps * rng.standard_normal((n, c)))[0]
        P = A @ A.T - Bm @ Bm.T
        dense = np.linalg.norm(P) / math.sqrt(2 * c)
        assert abs(oracle.projector_distance(A, Bm) - dense) <= 1e-6 * dense


def test_canonical_signs_hand_built_cases():
    """The sign rule of the W step (the paper leaves singular-vector signs
    open): each column's largest-magnitude entry is made positive, the first
    such entry on ties, and an all-zero column keeps +1."""
    U = np.array([[0.2, 0.5, -0.5, 0.0, 0.1],
                  [-0.9, -0.5, 0.5, 0.0, -0.1],
                  [0.3, 0.1, 0.1, 0.0, 0.7]])
    s = oracle.canonical_signs(U)
    np.testing.assert_array_equal(s, [-1.0, 1.0, -1.0, 1.0, 1.0])
    V = U * s
    for c in range(U.shape[1]):
        col = V[:, c]
        if not col.any():
            continue
        first = int(np.flatnonzero(np.abs(col) == np.abs(col).max())[0])
        assert col[first] > 0


def test_w_step_applies_the_sign_rule():
    """U = Q W from the oracle's W step follows the same rule on every column,
    whatever the sign the SVD routine returned."""
    rng = np.random.default_rng(7)
    Q = np.linalg.qr(rng.standard_normal((30, 9)))[0]
    Y = rng.standard_normal((30, 50))
    W, U, _ = oracle.w_step(Q, Y, 6)
    for c in range(6):
        j = int(np.argmax(np.abs(U[:, c])))
        assert U[j, c] > 0
    np.testing.assert_allclose(U, Q @ W, atol=1e-14)


def test_sq_norm_chunks_match_loop():
    """Squared norm over chunks (several chunks and a ragged tail) equals the
    plain sum of squares over every entry."""
    rng = np.random.default_rng(11)
    X = rng.standard_normal((7, 9, 11)).astype(np.float32)
    ref = sum(float(v) * float(v) for v in X.reshape(-1))
    assert abs(oracle.sq_norm(X, rows=100) - ref) <= 1e-13 * ref


def test_rel_error_orthonormal_closed_form():
    """X = C x_k F_k + E with E orthogonal to Range(F_1) in mode 1: the
    projection error is exactly ||E|| / ||X|| (||X||^2 = ||C||^2 + ||E||^2),
    and the orthogonal-projection form agrees with the explicit residual;
    below eps = 1e-4 it refuses (the subtraction would cancel)."""
    rng = np.random.default_rng(12)
    dims, cols = (9, 8, 7), (3, 4, 2)
    Fs, comp = [], None
    for k, (n, c) in enumerate(zip(dims, cols)):
        Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
        Fs.append(Q[:, :c])
        if k == 0:
            comp = Q[:, c:]
    C = rng.standard_normal(cols)
    E = oracle.ttm(1e-2 * rng.standard_normal((comp.shape[1],) + dims[1:]), comp, 0)
    X = oracle.multi_ttm(C, Fs) + E
    G = oracle.core(X, Fs)
    n2 = oracle.sq_norm(X)
    exact = math.sqrt(np.sum(E ** 2) / (np.sum(C ** 2) + np.sum(E ** 2)))
    eps = oracle.rel_error_orthonormal(G, n2)
    assert abs(eps - exact) <= 1e-12 * exact
    assert abs(eps - oracle.rel_error(X, G, Fs)) <= 1e-12 * exact
    X0 = oracle.multi_ttm(C, Fs) + 1e-6 * E
    with pytest.raises(ValueError):
        oracle.rel_error_orthonormal(oracle.core(X0, Fs), oracle.sq_norm(X0))

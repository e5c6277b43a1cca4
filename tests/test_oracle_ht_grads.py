"""Pins of the FP64 oracle for Sub-R-RtL-HT (Algorithm 2), the transfer
tensors, the closed-form gradients and the paper's printed size facts."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synthgen
from oracle import brute

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------------ printed facts
def test_printed_facts():
    with open(os.path.join(HERE, "golden", "paper_printed_facts.json")) as f:
        facts = json.load(f)
    for e in facts["columns_mode_unfolding"]:
        dims = (e["n"],) * e["d"]
        ncols = math.prod(dims) // dims[0]
        if "n_neq_k" in e:
            assert ncols == e["n_neq_k"]
            pct = 100.0 * e["s"] / ncols
            assert abs(pct - e["percent_printed"]) / e["percent_printed"] < 0.2
        else:
            assert abs(ncols - e["n_neq_k_approx"]) / e["n_neq_k_approx"] < 0.01
    for e in facts["sampled_fraction"]:
        pct = 100.0 * e["s"] / e["n"] ** (e["d"] - 1)
        assert abs(pct - e["percent_printed"]) / e["percent_printed"] < 0.25
    for e in facts["dimension_tree"]:
        tr = synthgen.balanced_tree(e["d"])
        assert tr.num_nodes - 1 == e["node_svds"]
        assert sum(1 for t in range(tr.num_nodes) if not tr.is_leaf(t)) == e["transfer_tensors"]
        assert max(tr.level) == e["depth"] == math.ceil(math.log2(e["d"]))


def test_tree_structure():
    for d in range(2, 10):
        tr = synthgen.balanced_tree(d)
        assert tr.count[0] == d and tr.first[0] == 0
        leaves = sorted(tr.first[t] for t in range(tr.num_nodes) if tr.is_leaf(t))
        assert leaves == list(range(d))
        for t in range(tr.num_nodes):
            if not tr.is_leaf(t):
                l, r = tr.left[t], tr.right[t]
                assert tr.modes(l) + tr.modes(r) == tr.modes(t)
                assert tr.count[l] == (tr.count[t] + 1) // 2
        assert max(tr.level) == math.ceil(math.log2(d))


# ------------------------------------------------------------------ transfer tensors
def test_transfer_tensor_brute_force_kron():
    """B_S(i,j,k) = <u_i, v_j kron w_k> with an explicit Kronecker product (4^4)."""
    rng = np.random.default_rng(0)
    US = np.linalg.qr(rng.standard_normal((16, 3)))[0]
    Ul = np.linalg.qr(rng.standard_normal((4, 2)))[0]
    Ur = np.linalg.qr(rng.standard_normal((4, 3)))[0]
    B = oracle.transfer_tensor(US, Ul, Ur)
    for i in range(3):
        for j in range(2):
            for k in range(3):
                ref = US[:, i] @ np.kron(Ul[:, j], Ur[:, k])
                assert abs(B[i, j, k] - ref) < 1e-15


def test_root_transfer_brute_force():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((3, 4, 2, 5))
    tr = synthgen.balanced_tree(4)
    Ul = rng.standard_normal((12, 2))
    Ur = rng.standard_normal((10, 3))
    B = oracle.root_transfer(X, tr, Ul, Ur)
    v = X.reshape(-1)
    for j in range(2):
        for k in range(3):
            assert abs(B[0, j, k] - v @ np.kron(Ul[:, j], Ur[:, k])) < 1e-12


def test_gather_node_is_multimode_unfolding():
    rng = np.random.default_rng(2)
    dims = (3, 4, 2, 5, 2)
    X = rng.standard_normal(dims)
    tr = synthgen.balanced_tree(5)
    for t in range(1, tr.num_nodes):
        A = oracle.unfold_set(X, tr.modes(t))
        idx = np.sort(rng.choice(A.shape[1], min(6, A.shape[1]), replace=False))
        np.testing.assert_array_equal(oracle.gather_node(X, tr, t, idx), A[:, idx])


# ------------------------------------------------------------------ H-Tucker
def _ht_run(inp, rank, p, walpha, seed, dense=False):
    dims = inp.dims
    tr = inp.tree
    N = math.prod(dims)
    ranks, ells, ws = {}, {}, {}
    for t in range(1, tr.num_nodes):
        nS = math.prod(dims[k] for k in tr.modes(t))
        ranks[t] = min(rank, nS)
        ells[t] = min(rank + p, nS, N // nS)
        ws[t] = N // nS if dense else min(walpha * nS, N // nS)
    sk = synthgen.node_sketches(dims, tr, ells, ws, cfg=200 + seed, omega_dtype="f64")
    return oracle.sub_r_rtl_ht(inp.X, tr, ranks, sk), ranks


@pytest.mark.parametrize("order", [4, 5, 8])
def test_ht_exact_hierarchical_rank_recovered(order):
    """sigma = 0: every sampled unfolding spans Range(X^(S)); nestedness holds and
    the format reproduces X (Section 4)."""
    n = 4 if order == 8 else 6
    inp = synthgen.ht_tensor(n, order, 3, 0.0, cfg=21, dtype="f64")
    (U, B, _), _ = _ht_run(inp, 3, 4, 20, 0)
    assert oracle.ht_rel_error(inp.X, inp.tree, U, B) < 1e-12
    tr = inp.tree
    for t in range(1, tr.num_nodes):
        if not tr.is_leaf(t):
            K = oracle.kron_cols(U[tr.left[t]], U[tr.right[t]])
            assert np.linalg.norm(U[t] - K @ (K.T @ U[t])) < 1e-12


def test_ht_dense_full_oversampling_equals_deterministic_rtl():
    """All columns sampled and ell_S = n_S: every W_S step returns the dominant
    singular vectors of X^(S): Sub-R-RtL-HT equals deterministic RtL-HT."""
    inp = synthgen.ht_tensor(3, 4, 2, 1e-2, cfg=22, dtype="f64")
    (U, B, _), ranks = _ht_run(inp, 2, 100, 0, 0, dense=True)
    Ud, Bd = brute.rtl_ht(inp.X, inp.tree, ranks)
    for t in U:
        np.testing.assert_allclose(U[t], Ud[t], atol=1e-10)
    for t in B:
        np.testing.assert_allclose(B[t], Bd[t], atol=1e-10)


def test_deterministic_rtl_ht_error_bounds():
    """max_S tail_S^2 <= ||X - X_hat||^2 <= sum_S tail_S^2 for RtL-HT: the
    bracket behind the sqrt(2d-3) quasi-optimality (Section 4)."""
    inp = synthgen.ht_tensor(4, 4, 3, 5e-2, cfg=23, dtype="f64")
    tr = inp.tree
    ranks = {t: 2 for t in range(1, tr.num_nodes)}
    U, B = brute.rtl_ht(inp.X, tr, ranks)
    err2 = np.sum((inp.X - oracle.ht_full(inp.dims, tr, {t: U[t] for t in U if tr.is_leaf(t)},
                                          B)) ** 2)
    tails = brute.ht_tails_sq(inp.X, tr, ranks)
    assert max(tails) * (1 - 1e-12) <= err2 <= sum(tails) * (1 + 1e-12)


def test_ht_randomized_error_near_deterministic():
    """Randomized HT on a noisy hierarchical-rank tensor: within the deterministic
    bracket's upper end (no theory for the randomized variant; sanity only)."""
    inp = synthgen.ht_tensor(5, 4, 3, 1e-3, cfg=24, dtype="f64")
    tr = inp.tree
    (U, B, _), ranks = _ht_run(inp, 3, 4, 20, 0)
    err = oracle.ht_rel_error(inp.X, tr, U, B)
    tails = brute.ht_tails_sq(inp.X, tr, ranks)
    nx = np.linalg.norm(inp.X)
    assert err <= 10 * math.sqrt(sum(tails)) / nx


# ------------------------------------------------------------------ gradients
def _loss(X, Fs):
    G = oracle.core(X, Fs)
    return float(np.sum((X - oracle.reconstruct(G, Fs)) ** 2))


def test_grads_every_entry_fd_3x3x3x3():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((3, 3, 3, 3))
    Fs = [rng.standard_normal((3, 2)) for _ in range(4)]
    L, dX, dF = oracle.loss_and_grads(X, Fs)
    assert abs(L - _loss(X, Fs)) < 1e-12
    h = 1e-6
    for i in np.ndindex(X.shape):
        Xp, Xm = X.copy(), X.copy()
        Xp[i] += h
        Xm[i] -= h
        fd = (_loss(Xp, Fs) - _loss(Xm, Fs)) / (2 * h)
        assert abs(fd - dX[i]) <= 1e-6 * max(1.0, abs(fd))
    for k in range(4):
        for i in np.ndindex(Fs[k].shape):
            Fp = [F.copy() for F in Fs]
            Fm = [F.copy() for F in Fs]
            Fp[k][i] += h
            Fm[k][i] -= h
            fd = (_loss(X, Fp) - _loss(X, Fm)) / (2 * h)
            assert abs(fd - dF[k][i]) <= 1e-6 * max(1.0, abs(fd))


def test_grads_directional_fd_4pow8():
    """16 random directions at 4^8 with c_k = 3, central differences with one
    Richardson step (the loss has degree 16 in the factors)."""
    rng = np.random.default_rng(4)
    X = rng.standard_normal((4,) * 8)
    Fs = [np.linalg.qr(rng.standard_normal((4, 3)))[0] for _ in range(8)]
    L, dX, dF = oracle.loss_and_grads(X, Fs)
    h = 1e-4
    for _ in range(16):
        VX = rng.standard_normal(X.shape)
        VF = [rng.standard_normal(F.shape) for F in Fs]
        def cd(step):
            lp = _loss(X + step * VX, [F + step * V for F, V in zip(Fs, VF)])
            lm = _loss(X - step * VX, [F - step * V for F, V in zip(Fs, VF)])
            return (lp - lm) / (2 * step)
        fd = (4 * cd(h / 2) - cd(h)) / 3          # Richardson: O(h^4) truncation
        an = float(np.sum(dX * VX) + sum(np.sum(a * b) for a, b in zip(dF, VF)))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


def test_grads_match_torch_autograd():
    """Independent check of the closed forms with PyTorch's CPU autograd in FP64."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    X = rng.standard_normal((4, 5, 3))
    Fs = [rng.standard_normal((n, 2)) for n in (4, 5, 3)]
    L, dX, dF = oracle.loss_and_grads(X, Fs)
    Xt = torch.tensor(X, requires_grad=True)
    Ft = [torch.tensor(F, requires_grad=True) for F in Fs]
    G = torch.einsum("abc,ai,bj,ck->ijk", Xt, *Ft)
    Xh = torch.einsum("ijk,ai,bj,ck->abc", G, *Ft)
    loss = ((Xt - Xh) ** 2).sum()
    loss.backward()
    assert abs(loss.item() - L) < 1e-10
    np.testing.assert_allclose(Xt.grad.numpy(), dX, atol=1e-10)
    for a, b in zip(Ft, dF):
        np.testing.assert_allclose(a.grad.numpy(), b, atol=1e-10)


# ------------------------------------------------------------------ storage dtypes
def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(6)
    x = (rng.standard_normal(10000) * 10.0 ** rng.integers(-3, 3, 10000)).astype(np.float32)
    ours = synthgen.to_f64(synthgen.to_storage(x, "bf16"), "bf16")
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(ours, ref)


# ------------------------------------------------------------------ H-Tucker format VJP
def _ht_params(rng, dims, ranks):
    """Random (not orthonormal) leaf bases and transfer tensors on the
    balanced tree; ranks[t] for every non-root node."""
    tr = synthgen.balanced_tree(len(dims))
    U, B = {}, {}
    for t in range(1, tr.num_nodes):
        if tr.is_leaf(t):
            U[t] = rng.standard_normal((dims[tr.first[t]], ranks[t]))
    for t in range(tr.num_nodes):
        if not tr.is_leaf(t):
            rt = 1 if t == 0 else ranks[t]
            B[t] = rng.standard_normal((rt, ranks[tr.left[t]], ranks[tr.right[t]]))
    return tr, U, B


@pytest.mark.parametrize("dims", [(3, 2, 3, 2), (2, 3, 2, 2, 3)])
def test_ht_full_vjp_every_entry_fd(dims):
    """<H, ht_full(theta)> is affine in every single entry of every leaf basis
    and transfer tensor (the format is multilinear in its parameters, each
    used once), so central differences are exact up to rounding."""
    rng = np.random.default_rng(11 + len(dims))
    tr = synthgen.balanced_tree(len(dims))
    ranks = {t: 2 for t in range(1, tr.num_nodes)}
    tr, U, B = _ht_params(rng, dims, ranks)
    H = rng.standard_normal(dims)
    Bbar, Ubar = oracle.ht_full_vjp(dims, tr, U, B, H)
    assert set(Bbar) == set(B) and set(Ubar) == set(U)

    def L(U_, B_):
        return float(np.sum(H * oracle.ht_full(dims, tr, U_, B_)))

    h = 1e-3
    for t in B:
        for i in np.ndindex(B[t].shape):
            Bp = {k: v.copy() for k, v in B.items()}
            Bm = {k: v.copy() for k, v in B.items()}
            Bp[t][i] += h
            Bm[t][i] -= h
            fd = (L(U, Bp) - L(U, Bm)) / (2 * h)
            assert abs(fd - Bbar[t][i]) <= 1e-9 * max(1.0, abs(fd)), (t, i)
    for t in U:
        for i in np.ndindex(U[t].shape):
            Up = {k: v.copy() for k, v in U.items()}
            Um = {k: v.copy() for k, v in U.items()}
            Up[t][i] += h
            Um[t][i] -= h
            fd = (L(Up, B) - L(Um, B)) / (2 * h)
            assert abs(fd - Ubar[t][i]) <= 1e-9 * max(1.0, abs(fd)), (t, i)


def test_ht_full_vjp_order2_is_matrix_product_rule():
    """Order 2: the format is U_1 B_R U_2^T; its adjoints are the textbook
    ones of a product of three matrices."""
    rng = np.random.default_rng(5)
    tr, U, B = _ht_params(rng, (4, 5), {1: 3, 2: 2})
    H = rng.standard_normal((4, 5))
    Bbar, Ubar = oracle.ht_full_vjp((4, 5), tr, U, B, H)
    U1, U2, BR = U[1], U[2], B[0][0]
    np.testing.assert_allclose(oracle.ht_full((4, 5), tr, U, B), U1 @ BR @ U2.T, rtol=1e-14)
    np.testing.assert_allclose(Bbar[0][0], U1.T @ H @ U2, rtol=1e-13)
    np.testing.assert_allclose(Ubar[1], H @ U2 @ BR.T, rtol=1e-13)
    np.testing.assert_allclose(Ubar[2], H.T @ U1 @ BR, rtol=1e-13)


# ------------------------------------------------------------------ closed-form HT workload
def test_inverse_norm_workload_values():
    """X(i) = (sum_j i_j^2)^(-1/2) on the 1-based grid: hand-evaluated corners
    and symmetry under permutation of the modes."""
    X = synthgen.inverse_norm_tensor(15, 4, "f64")
    assert X.shape == (15,) * 4
    assert X[0, 0, 0, 0] == 0.5                              # 1 / sqrt(4)
    assert X[14, 14, 14, 14] == 1.0 / 30.0                   # 1 / sqrt(4 * 225)
    assert X[1, 0, 0, 0] == 1.0 / math.sqrt(7.0)            # 4 + 1 + 1 + 1
    assert X[2, 1, 0, 0] == 1.0 / math.sqrt(15.0)           # 9 + 4 + 1 + 1
    np.testing.assert_array_equal(X, X.transpose(2, 0, 3, 1))
    X5 = synthgen.inverse_norm_tensor(3, 5, "f32")
    assert X5.dtype == np.float32 and X5[2, 2, 2, 2, 2] == np.float32(1.0 / math.sqrt(45.0))


def test_ht_residuals_streamed_closed_form():
    """X = X_hat(format A) + c Z: the streamed residual of format A is exactly
    c^2 ||Z||^2, that of a second format equals its explicit residual, and
    the squared norm is ||X||^2; row blocks of 7 leave a ragged tail."""
    rng = np.random.default_rng(21)
    dims = (4, 3, 5, 2)
    tr = synthgen.balanced_tree(4)

    def fmt(seed):
        g = np.random.default_rng(seed)
        U = {t: g.standard_normal((dims[tr.first[t]], 2)) for t in range(1, tr.num_nodes) if tr.is_leaf(t)}
        B = {t: g.standard_normal(((1 if t == 0 else 2), 2, 2)) for t in range(tr.num_nodes)
             if not tr.is_leaf(t)}
        return U, B

    A, Bf = fmt(1), fmt(2)
    Z = rng.standard_normal(dims)
    X = oracle.ht_full(dims, tr, *A) + 0.3 * Z
    (rA, rB), n2 = oracle.ht_residuals_streamed(X, tr, [A, Bf], rows=7)
    assert abs(rA - 0.09 * np.sum(Z ** 2)) <= 1e-12 * np.sum(Z ** 2)
    assert abs(rB - np.sum((X - oracle.ht_full(dims, tr, *Bf)) ** 2)) <= 1e-12 * rB
    assert abs(n2 - np.sum(X ** 2)) <= 1e-13 * n2

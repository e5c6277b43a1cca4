"""GPU parity of the H-Tucker format's full tensor, its residual and its
vector-Jacobian product (htucker_reconstruct, htucker_reconstruct_vjp)
against the FP64 oracle (ht_full, ht_full_vjp), on random formats of several
orders (ragged sizes, several column tiles, both rank paths of the streaming
expansion) and on the closed-form 1/||x|| workload decomposed on the GPU."""
import math

import numpy as np
import pytest
import torch

import ht_parity
import oracle
import synthgen

pytestmark = pytest.mark.gpu


def _format(dims, rank_of, seed):
    """Random leaf bases and transfer tensors (FP64, not orthonormal)."""
    rng = np.random.default_rng(seed)
    tr = synthgen.balanced_tree(len(dims))
    ranks = {t: rank_of(t, tr) for t in range(1, tr.num_nodes)}
    U, Bt = {}, {}
    for t in range(1, tr.num_nodes):
        if tr.is_leaf(t):
            U[t] = rng.standard_normal((dims[tr.first[t]], ranks[t])) / math.sqrt(ranks[t])
    for t in range(tr.num_nodes):
        if not tr.is_leaf(t):
            rt = 1 if t == 0 else ranks[t]
            rl, rr = ranks[tr.left[t]], ranks[tr.right[t]]
            Bt[t] = rng.standard_normal((rt, rl, rr)) / math.sqrt(rl * rr)
    return tr, ranks, U, Bt


def _dev(d):
    return {t: torch.from_numpy(v).cuda() for t, v in d.items()}


CASES = [
    # dims, rank rule, seed: order 4 over two column tiles with ragged tails,
    # orders 5 and 6 (unbalanced splits), a root child of rank 20 (the wide
    # expansion path), order 2 (the root alone)
    ((40, 30, 35, 33), lambda t, tr: 3 + t % 3, 1),
    ((5, 3, 4, 6, 2), lambda t, tr: 2 + t % 2, 2),
    ((3, 4, 2, 3, 5, 2), lambda t, tr: 2, 3),
    ((9, 8, 7, 6), lambda t, tr: 20 if t == 2 else 4, 4),
    ((37, 1500), lambda t, tr: 5, 5),
    # the root's right child at ranks 12, 14 and 40 (padded to 12, 16 and 64)
    ((6, 7, 5, 8), lambda t, tr: 12 if t == 2 else 3, 6),
    ((5, 6, 4, 9, 3), lambda t, tr: 14 if t == 2 else 3, 7),
    ((9, 4, 7, 50), lambda t, tr: 40 if t == 2 else 4, 8),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("out_dtype", [torch.float64, torch.float32])
def test_ht_full_tensor_matches_oracle(case, out_dtype):
    from paper_2603_21379_amd import tucker as T
    dims, rule, seed = CASES[case]
    tr, ranks, U, Bt = _format(dims, rule, seed)
    ref = oracle.ht_full(dims, tr, U, Bt)
    Xh, _ = T.ht_reconstruct(dims, tr, ranks, _dev(U), _dev(Bt), out_dtype=out_dtype)
    got = Xh.double().cpu().numpy()
    if out_dtype == torch.float64:
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())
    else:
        # computed in FP64, rounded once to FP32
        np.testing.assert_allclose(got, ref, rtol=2.0 ** -23, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("xdtype", ["f64", "f32", "bf16"])
def test_ht_residual_matches_oracle(case, xdtype):
    from paper_2603_21379_amd import tucker as T
    dims, rule, seed = CASES[case]
    tr, ranks, U, Bt = _format(dims, rule, seed)
    ref = oracle.ht_full(dims, tr, U, Bt)
    rng = np.random.default_rng(100 + seed)
    Xs = synthgen.to_storage(ref + 1e-3 * rng.standard_normal(dims), xdtype)
    X64 = synthgen.to_f64(Xs, xdtype)
    r2_ref = float(np.sum((X64 - ref) ** 2))
    n2_ref = float(np.sum(X64 ** 2))
    Xd = torch.from_numpy(Xs.view(np.int16) if xdtype == "bf16" else Xs).cuda()
    if xdtype == "bf16":
        Xd = Xd.view(torch.bfloat16)
    Xh, r2 = T.ht_reconstruct(dims, tr, ranks, _dev(U), _dev(Bt), Xref=Xd, out_dtype=torch.float64)
    r2 = r2.cpu().numpy()
    assert abs(r2[0] - r2_ref) <= 1e-9 * r2_ref
    assert abs(r2[1] - n2_ref) <= 1e-12 * n2_ref
    np.testing.assert_allclose(Xh.cpu().numpy(), ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("xdtype", ["f64", "f32", "bf16"])
def test_ht_residual_only_matches_oracle(case, xdtype):
    """The residual without X_hat: for FP32 X and a root right child of rank
    <= 16 the FP64-MFMA pass (ragged row and column tiles, padded ranks 8, 12
    and 16), otherwise the FP64 VALU pass; the same gates as with X_hat."""
    from paper_2603_21379_amd import tucker as T
    dims, rule, seed = CASES[case]
    tr, ranks, U, Bt = _format(dims, rule, seed)
    ref = oracle.ht_full(dims, tr, U, Bt)
    rng = np.random.default_rng(200 + seed)
    Xs = synthgen.to_storage(ref + 1e-3 * rng.standard_normal(dims), xdtype)
    X64 = synthgen.to_f64(Xs, xdtype)
    r2_ref = float(np.sum((X64 - ref) ** 2))
    n2_ref = float(np.sum(X64 ** 2))
    Xd = torch.from_numpy(Xs.view(np.int16) if xdtype == "bf16" else Xs).cuda()
    if xdtype == "bf16":
        Xd = Xd.view(torch.bfloat16)
    Xh, r2 = T.ht_reconstruct(dims, tr, ranks, _dev(U), _dev(Bt), Xref=Xd)
    assert Xh is None
    r2 = r2.cpu().numpy()
    assert abs(r2[0] - r2_ref) <= 1e-9 * r2_ref
    assert abs(r2[1] - n2_ref) <= 1e-12 * n2_ref


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("hdtype", [np.float64, np.float32])
def test_ht_vjp_matches_oracle(case, hdtype):
    from paper_2603_21379_amd import tucker as T
    dims, rule, seed = CASES[case]
    tr, ranks, U, Bt = _format(dims, rule, seed)
    H = np.random.default_rng(200 + seed).standard_normal(dims).astype(hdtype)
    Bbar_or, Ubar_or = oracle.ht_full_vjp(dims, tr, U, Bt, H.astype(np.float64))
    Bbar, Ubar = T.ht_reconstruct_vjp(dims, tr, ranks, _dev(U), _dev(Bt), torch.from_numpy(H).cuda())
    assert set(Bbar) == set(Bbar_or) and set(Ubar) == set(Ubar_or)
    for t in Bbar_or:
        ref = Bbar_or[t]
        np.testing.assert_allclose(Bbar[t].cpu().numpy(), ref, rtol=1e-10, atol=1e-11 * np.abs(ref).max())
    for t in Ubar_or:
        ref = Ubar_or[t]
        np.testing.assert_allclose(Ubar[t].cpu().numpy(), ref, rtol=1e-10, atol=1e-11 * np.abs(ref).max())


def _inverse_norm_run(order, dtype, n=15, rank=7, p=4, walpha=20):
    """Sub-R-RtL-HT of the closed-form tensor on the GPU (w = min(20 n, n_notS)
    fibers per node), its relative error from htucker_reconstruct, and the
    oracle's decomposition and error on the same sketches."""
    from paper_2603_21379_amd import tucker as T
    X = synthgen.inverse_norm_tensor(n, order, dtype)
    dims = X.shape
    tr = synthgen.balanced_tree(order)
    N = math.prod(dims)
    ranks, ells, ws = {}, {}, {}
    for t in range(1, tr.num_nodes):
        nS = math.prod(dims[k] for k in tr.modes(t))
        ells[t] = min(rank + p, nS, N // nS)
        ranks[t] = min(rank, ells[t])
        ws[t] = min(walpha * n, N // nS)
    fdt = synthgen.factor_dtype(dtype)
    sk = synthgen.node_sketches(dims, tr, ells, ws, cfg=60 + order, omega_dtype=fdt)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    dev = T.upload_sketches([(sk[t], N // math.prod(dims[k] for k in tr.modes(t)))
                             for t in range(1, tr.num_nodes)], "cuda", tdt)
    Xd = torch.from_numpy(X).cuda()
    res = T.sub_r_rtl_ht(Xd, tr, ranks, {t: dev[t - 1] for t in range(1, tr.num_nodes)})
    leaves = {t: res.U[t] for t in res.U if tr.is_leaf(t)}
    eps_gpu = T.ht_rel_error(Xd, tr, ranks, leaves, res.B)
    X64 = synthgen.to_f64(X, dtype)
    U_or, B_or, _ = oracle.sub_r_rtl_ht(X64, tr, ranks, sk)
    eps_or = oracle.ht_rel_error(X64, tr, U_or, B_or)
    U_gpu = {t: u.cpu().numpy() for t, u in res.U.items()}
    B_gpu = {t: b.cpu().numpy() for t, b in res.B.items()}
    eps_gpu_format_on_host = oracle.ht_rel_error(X64, tr, U_gpu, B_gpu)
    spread = ht_parity.eps_spread(X64, tr, ranks, sk, eps_or)
    return eps_gpu, eps_gpu_format_on_host, eps_or, spread


@pytest.mark.parametrize("order", [4, 5, 6])
def test_inverse_norm_workload_f64(order):
    eps_gpu, eps_host, eps_or, spread = _inverse_norm_run(order, "f64")
    # the device residual of the device format equals the host evaluation of
    # it (both FP64 sums, different orders)
    assert abs(eps_gpu - eps_host) <= 1e-12 * eps_host
    # and the device decomposition matches the oracle's: 1e-10 of the oracle's
    # error plus the error's own spread under unit-roundoff perturbations of
    # the inputs (the node sketches of this tensor are numerically
    # rank-deficient; at order 6 that spread is about 5e-10 of the error)
    gate = ht_parity.eps_gate(eps_or, spread, 1e-10)
    print(f"order {order}: |eps_gpu - eps_or| / eps_or = {abs(eps_gpu - eps_or) / eps_or:.2e}, "
          f"spread / eps_or = {spread / eps_or:.2e}, gate / eps_or = {gate / eps_or:.2e}")
    assert abs(eps_gpu - eps_or) <= gate
    assert eps_or < 1e-2


def test_inverse_norm_workload_f32():
    eps_gpu, eps_host, eps_or, spread = _inverse_norm_run(5, "f32")
    assert abs(eps_gpu - eps_host) <= 1e-12 * eps_host
    assert abs(eps_gpu - eps_or) <= ht_parity.eps_gate(eps_or, spread, 1e-5)


def test_ht_reconstruct_rejects_bad_arguments():
    from paper_2603_21379_amd import binding as B
    from paper_2603_21379_amd import tucker as T
    dims = (4, 5, 3)
    tr, ranks, U, Bt = _format(dims, lambda t, tr: 2, 9)
    Ud, Bd = _dev(U), _dev(Bt)
    with pytest.raises(B.TkError):     # neither output
        rk, Ul, Bl = T._ht_lists(tr, ranks, Ud, Bd)
        B.htucker_reconstruct(list(dims), tr, rk, Ul, Bl)
    with pytest.raises(B.TkError):     # a leaf basis missing
        rk, Ul, Bl = T._ht_lists(tr, ranks, Ud, Bd)
        Ul[tr.num_nodes - 1] = None
        B.htucker_reconstruct(list(dims), tr, rk, Ul, Bl, Xhat=torch.empty(dims, dtype=torch.float64,
                                                                          device="cuda"))
    with pytest.raises(B.TkError):     # the root's right child above rank 64
        rk, Ul, Bl = T._ht_lists(tr, ranks, Ud, Bd)
        rk[tr.right[0]] = 65
        B.htucker_reconstruct(list(dims), tr, rk, Ul, Bl, Xhat=torch.empty(dims, dtype=torch.float64,
                                                                          device="cuda"))
    with pytest.raises(B.TkError):     # Xref of other dims
        T.ht_reconstruct(dims, tr, ranks, Ud, Bd, Xref=torch.zeros(4, 5, 4, dtype=torch.float64,
                                                                    device="cuda"))


def test_htucker_full_autograd_matches_oracle():
    """loss = <W, Xhat> + ||Xhat||^2 / 2 through torch.autograd: the
    gradients reaching every leaf basis and transfer tensor are the oracle's
    VJP at H = dloss/dXhat."""
    from paper_2603_21379_amd import autograd as A
    dims, rule, seed = CASES[1]
    tr, ranks, U, Bt = _format(dims, rule, seed)
    Wt = np.random.default_rng(7).standard_normal(dims)
    Ud = {t: torch.from_numpy(v).cuda().requires_grad_() for t, v in U.items()}
    Bd = {t: torch.from_numpy(v).cuda().requires_grad_() for t, v in Bt.items()}
    Xh = A.htucker_full(dims, tr, ranks, Ud, Bd)
    loss = (torch.from_numpy(Wt).cuda() * Xh).sum() + 0.5 * (Xh * Xh).sum()
    loss.backward()
    H = Wt + oracle.ht_full(dims, tr, U, Bt)
    Bbar_or, Ubar_or = oracle.ht_full_vjp(dims, tr, U, Bt, H)
    for t in Bbar_or:
        np.testing.assert_allclose(Bd[t].grad.cpu().numpy(), Bbar_or[t], rtol=1e-10,
                                   atol=1e-11 * np.abs(Bbar_or[t]).max())
    for t in Ubar_or:
        np.testing.assert_allclose(Ud[t].grad.cpu().numpy(), Ubar_or[t], rtol=1e-10,
                                   atol=1e-11 * np.abs(Ubar_or[t]).max())

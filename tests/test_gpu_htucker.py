"""GPU parity of Sub-R-RtL-HT (node sketches, batched QR + W step, transfer
tensors, root contraction) against the FP64 oracle on the same inputs."""
import math

import numpy as np
import pytest
import torch

import oracle
import synthgen
from synthgen import configs

pytestmark = pytest.mark.gpu


def _setup(n, order, rank, p, walpha, noise, dtype, cfg):
    inp = synthgen.ht_tensor(n, order, rank, noise, cfg=cfg, dtype=dtype)
    tr = inp.tree
    dims = inp.dims
    N = math.prod(dims)
    ranks, ells, ws = {}, {}, {}
    for t in range(1, tr.num_nodes):
        nS = math.prod(dims[k] for k in tr.modes(t))
        ells[t] = min(rank + p, nS, N // nS)
        ranks[t] = min(rank, ells[t])
        ws[t] = min(walpha * n, N // nS)
    fdt = synthgen.factor_dtype(dtype)
    sk = synthgen.node_sketches(dims, tr, ells, ws, cfg=cfg, omega_dtype=fdt)
    return inp, ranks, sk


def _run(inp, ranks, sk):
    from paper_2603_21379_amd import tucker as T
    tr = inp.tree
    dims = inp.dims
    N = math.prod(dims)
    fdt = torch.float64 if inp.dtype == "f64" else torch.float32
    pairs = {t: (sk[t], N // math.prod(dims[k] for k in tr.modes(t))) for t in sk}
    dev = T.upload_sketches([pairs[t] for t in range(1, tr.num_nodes)], "cuda", fdt)
    skd = {t: dev[t - 1] for t in range(1, tr.num_nodes)}
    Xd = torch.from_numpy(inp.X).cuda()
    res = T.sub_r_rtl_ht(Xd, tr, ranks, skd)
    torch.cuda.synchronize()
    U = {t: u.double().cpu().numpy() for t, u in res.U.items()}
    B = {t: b.double().cpu().numpy() for t, b in res.B.items()}
    return U, B, res.info.cpu().numpy()


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_c5_small_parity(dtype, tol):
    c = configs.C5_SMALL
    inp, ranks, sk = _setup(c.n, c.order, c.rank, c.p, c.w_alpha, c.noise, dtype, c.cfg_id)
    X64 = synthgen.to_f64(inp.X, dtype)
    U_or, B_or, _ = oracle.sub_r_rtl_ht(X64, inp.tree, ranks, sk)
    U, B, info = _run(inp, ranks, sk)
    ptol = 1e-9 if dtype == "f64" else 1e-5
    for t in U_or:
        assert oracle.projector_distance(U[t], U_or[t]) < ptol, t
    # canonical signs make the transfer tensors comparable entrywise
    btol = 1e-9 if dtype == "f64" else 2e-5
    for t in B_or:
        np.testing.assert_allclose(B[t], B_or[t], atol=btol * max(1.0, np.abs(B_or[t]).max()))
    eps_or = oracle.ht_rel_error(X64, inp.tree, U_or, B_or)
    eps_gpu = oracle.ht_rel_error(X64, inp.tree, U, B)
    assert abs(eps_gpu - eps_or) <= tol * eps_or
    assert (info == 0).all()


def test_exact_hierarchical_rank_recovered_on_gpu():
    inp, ranks, sk = _setup(4, 6, 3, 4, 20, 0.0, "f64", 55)
    U, B, info = _run(inp, ranks, sk)
    assert oracle.ht_rel_error(inp.X, inp.tree, U, B) < 1e-12


def test_order4_odd_sizes_f64():
    # order 5 gives an unbalanced split (3 | 2) and a node with three modes
    inp, ranks, sk = _setup(5, 5, 3, 4, 20, 1e-3, "f64", 56)
    U_or, B_or, _ = oracle.sub_r_rtl_ht(inp.X, inp.tree, ranks, sk)
    U, B, _ = _run(inp, ranks, sk)
    for t in U_or:
        assert oracle.projector_distance(U[t], U_or[t]) < 1e-9
    eps_or = oracle.ht_rel_error(inp.X, inp.tree, U_or, B_or)
    eps_gpu = oracle.ht_rel_error(inp.X, inp.tree, U, B)
    assert abs(eps_gpu - eps_or) <= 1e-10 * eps_or

"""GPU parity at the measured workload sizes, in the launch configurations the
benchmark times, on outputs the FP64 oracle can compute at that size:

* every sampled fiber (bit-exact) and, from them, every mode's or node's
  orthonormal basis and truncated factor (the oracle's QR and SVD on the
  same gathered fibers and Gaussians);
* the core of the full tensor on the GPU's own factors (the oracle contracts
  the last mode first over exactly upcast row chunks);
* for H-Tucker, every transfer tensor and the root transfer (row blocks of
  the root contraction summed in FP64).

The end-to-end error gate runs at the oracle-sized versions of the same
workloads (test_gpu_tucker, test_gpu_htucker, test_gpu_batch)."""
import gc
import math

import numpy as np
import pytest
import torch

import oracle
import synthgen
from synthgen import configs

pytestmark = pytest.mark.gpu

U_EFF = {"f64": 1.1e-16, "f32": 6e-8, "bf16": 6e-8, "f16": 6e-8}


def _to_device(X, dtype):
    if dtype == "bf16":
        return torch.from_numpy(X.view(np.int16)).cuda().view(torch.bfloat16)
    return torch.from_numpy(X).cuda()


def _y_host(y, dtype):
    if dtype == "bf16":
        return synthgen.to_f64(y.cpu().view(torch.int16).numpy().view(np.uint16), "bf16")
    return y.double().cpu().numpy()


def _factor_tol(sv, r, u_eff):
    """Wedin-type bound on the projector distance of the dominant r left
    singular vectors: ~u sigma_1 / (sigma_r - sigma_{r+1})."""
    gap = sv[r - 1] - (sv[r] if r < len(sv) else 0.0)
    return max(1e-9, 100.0 * u_eff * sv[0] / gap)


def _check_mode(Xh, k, s, Y_gpu, U_gpu, r, dtype):
    to64 = (lambda a: synthgen.to_f64(a, dtype))
    Y_or = oracle.gather_fibers(Xh, k, s.idx, to64=to64)
    np.testing.assert_array_equal(Y_gpu, Y_or)
    Q_or = oracle.orth(oracle.range_sketch(Y_or, np.asarray(s.omega, dtype=np.float64)))
    _, U_or, sv = oracle.w_step(Q_or, Y_or, r)
    d = oracle.projector_distance(U_gpu, U_or)
    assert d < _factor_tol(sv, r, U_EFF[dtype]), (k, d)


def _release():
    gc.collect()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("which,dtype,ctol", [("c2", "f32", 1e-6), ("c3", "bf16", 2e-5),
                                              ("c3", "f16", 2e-5)])
def test_fullsize_tucker(which, dtype, ctol):
    from paper_2603_21379_amd import tucker as T
    c = configs.C2 if which == "c2" else configs.C3
    dims, ranks = c.dims, c.ranks
    inp = synthgen.tucker_tensor(dims, ranks, c.decay, c.noise, cfg=c.cfg_id, dtype=dtype)
    ells = synthgen.default_ell(dims, ranks, c.p)
    ss = synthgen.default_s(dims, c.alpha)
    sk = synthgen.mode_sketches(dims, ells, ss, cfg=c.cfg_id, omega_dtype="f32")
    X = _to_device(inp.X, dtype)
    skd = T.mode_sketches_to_device(sk, dims, "cuda", torch.float32)
    res = T.sub_r_hosvd(X, ranks, skd)
    torch.cuda.synchronize()
    assert int(res.info.abs().sum()) == 0
    F = [f.double().cpu().numpy() for f in res.F]
    for k in range(len(dims)):
        _check_mode(inp.X, k, sk[k], _y_host(res.Y[k], dtype), F[k], ranks[k], dtype)
    G = res.G.double().cpu().numpy()
    del X, res
    _release()
    G_chk = oracle.core_chunked(inp.X, F, to64=lambda a: synthgen.to_f64(a, dtype))
    np.testing.assert_allclose(G, G_chk, rtol=0, atol=ctol * np.abs(G_chk).max())


def test_fullsize_batch_512():
    from paper_2603_21379_amd import binding as B
    from paper_2603_21379_amd import tucker as T
    specs = synthgen.batch_specs(configs.C4_COUNT, cfg=configs.C4_CFG_ID)
    host, X, sk_dev, U, G = [], [], [], [], []
    for i, sp in enumerate(specs):
        inp = synthgen.tucker_tensor(sp.dims, sp.ranks, 0.6, 1e-5, cfg=configs.C4_CFG_ID, dtype="f32", run=i)
        sk = synthgen.mode_sketches(sp.dims, sp.ells, sp.ss, cfg=configs.C4_CFG_ID, omega_dtype="f32", run=i)
        host.append((inp.X, sk))
        X.append(torch.from_numpy(inp.X).cuda())
        sk_dev += T.mode_sketches_to_device(sk, sp.dims, "cuda", torch.float32)
        U += [torch.empty(n, r, dtype=torch.float32, device="cuda") for n, r in zip(sp.dims, sp.ranks)]
        G.append(torch.empty(sp.ranks, dtype=torch.float32, device="cuda"))
    info = torch.zeros(len(U), dtype=torch.int32, device="cuda")
    plan = B.BatchPlan(X, [sp.ranks for sp in specs], sk_dev, U, G, info)
    plan.autotune()
    plan.run()
    torch.cuda.synchronize()
    # the largest tensors and a seeded sample of the rest
    sizes = [math.prod(sp.dims) for sp in specs]
    order = np.argsort(sizes)[::-1]
    pick = list(order[:3]) + list(np.random.default_rng(7).choice(order[3:], 5, replace=False))
    first = np.cumsum([0] + [len(sp.dims) for sp in specs])
    for i in pick:
        sp = specs[i]
        Xh, sk = host[i]
        Ub = [u.double().cpu().numpy() for u in U[first[i]:first[i] + len(sp.dims)]]
        for k in range(len(sp.dims)):
            Y_or = oracle.gather_fibers(Xh, k, sk[k].idx)
            Q_or = oracle.orth(oracle.range_sketch(Y_or, sk[k].omega.astype(np.float64)))
            _, U_or, sv = oracle.w_step(Q_or, Y_or, sp.ranks[k])
            d = oracle.projector_distance(Ub[k], U_or)
            assert d < _factor_tol(sv, sp.ranks[k], U_EFF["f32"]), (i, k, d)
        G_chk = oracle.core(Xh.astype(np.float64), Ub)
        np.testing.assert_allclose(G[i].double().cpu().numpy(), G_chk, rtol=0,
                                   atol=1e-6 * np.abs(G_chk).max())
    plan.close()
    del X, U, G, sk_dev
    _release()


def test_fullsize_htucker_18x8():
    from paper_2603_21379_amd import tucker as T
    c = configs.C5
    inp = synthgen.ht_tensor(c.n, c.order, c.rank, c.noise, cfg=c.cfg_id, dtype=c.dtype)
    tr, dims = inp.tree, inp.dims
    N = math.prod(dims)
    ranks, ells, ws = {}, {}, {}
    for t in range(1, tr.num_nodes):
        nS = math.prod(dims[k] for k in tr.modes(t))
        ells[t] = min(c.rank + c.p, nS, N // nS)
        ranks[t] = min(c.rank, ells[t])
        ws[t] = min(c.w_alpha * c.n, N // nS)
    sk = synthgen.node_sketches(dims, tr, ells, ws, cfg=c.cfg_id, omega_dtype="f32")
    X = torch.from_numpy(inp.X).cuda()
    pairs = [(sk[t], N // math.prod(dims[k] for k in tr.modes(t))) for t in range(1, tr.num_nodes)]
    dsk = T.upload_sketches(pairs, "cuda", torch.float32)
    res = T.sub_r_rtl_ht(X, tr, ranks, {t: dsk[t - 1] for t in range(1, tr.num_nodes)})
    torch.cuda.synchronize()
    assert int(res.info.abs().sum()) == 0
    U = {t: u.cpu().numpy() for t, u in res.U.items()}
    Bg = {t: b.cpu().numpy() for t, b in res.B.items()}
    del X, res, dsk
    _release()
    for t in range(1, tr.num_nodes):
        Y_or = oracle.gather_node(inp.X, tr, t, sk[t].idx)
        Q_or = oracle.orth(oracle.range_sketch(Y_or, sk[t].omega.astype(np.float64)))
        _, U_or, sv = oracle.w_step(Q_or, Y_or, ranks[t])
        d = oracle.projector_distance(U[t], U_or)
        assert d < _factor_tol(sv, ranks[t], U_EFF["f64"]), (t, d)
        if not tr.is_leaf(t):
            B_chk = oracle.transfer_tensor(U[t], U[tr.left[t]], U[tr.right[t]])
            np.testing.assert_allclose(Bg[t], B_chk, rtol=0, atol=1e-12 * np.abs(B_chk).max())
    # root: U_l^T X^(l) U_r, summed over blocks of rows of X^(l)
    L, R = tr.left[0], tr.right[0]
    nl = U[L].shape[0]
    Xm = inp.X.reshape(nl, -1)
    B_chk = None
    for r0 in range(0, nl, 2048):
        part = oracle.root_transfer(Xm[r0:r0 + 2048], tr, U[L][r0:r0 + 2048], U[R])
        B_chk = part if B_chk is None else B_chk + part
    np.testing.assert_allclose(Bg[0], B_chk, rtol=0, atol=1e-11 * np.abs(B_chk).max())

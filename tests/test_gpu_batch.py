"""GPU parity of the batching form (many FP32 tensors of uneven order and
size, every mode, one fixed launch sequence): per-tensor agreement with the
FP64 oracle and with the single-tensor path, replays of a captured HIP graph
against the eager run, and schedules chosen by the autotuner."""
import numpy as np
import pytest
import torch

import oracle
import synthgen

pytestmark = pytest.mark.gpu


def make_batch(specs, cfg=44):
    from paper_2603_21379_amd import tucker as T
    items = []
    for i, sp in enumerate(specs):
        # noise 1e-4: eps stays well above the floor that FP32 storage of the
        # factors puts on it (about 1e-7 ||X|| added in quadrature)
        inp = synthgen.tucker_tensor(sp.dims, sp.ranks, 0.6, 1e-4, cfg=cfg, dtype="f32", run=i)
        sk = synthgen.mode_sketches(sp.dims, sp.ells, sp.ss, cfg=cfg, omega_dtype="f32", run=i)
        X = torch.from_numpy(inp.X).cuda()
        skd = T.mode_sketches_to_device(sk, sp.dims, "cuda", torch.float32)
        items.append((sp, inp, sk, X, skd))
    return items


def plan_for(items):
    from paper_2603_21379_amd import binding as B
    X = [it[3] for it in items]
    ranks = [it[0].ranks for it in items]
    sketches = [s for it in items for s in it[4]]
    U = [torch.empty(n, r, dtype=torch.float32, device="cuda") for it in items
         for n, r in zip(it[0].dims, it[0].ranks)]
    G = [torch.empty(it[0].ranks, dtype=torch.float32, device="cuda") for it in items]
    info = torch.zeros(sum(len(it[0].dims) for it in items), dtype=torch.int32, device="cuda")
    plan = B.BatchPlan(X, ranks, sketches, U, G, info)
    return plan, U, G, info


def small_specs():
    return synthgen.batch_specs(12, cfg=44, nmin=5, nmax=40, rmin=2, rmax=9, cap=60000)


def test_batch_matches_oracle_and_single_path():
    from paper_2603_21379_amd import tucker as T
    items = make_batch(small_specs())
    plan, U, G, info = plan_for(items)
    plan.run()
    torch.cuda.synchronize()
    assert int(info.abs().sum()) == 0
    m = 0
    for ti, (sp, inp, sk, X, skd) in enumerate(items):
        d = len(sp.dims)
        X64 = inp.X.astype(np.float64)
        G_or, U_or, _, _, _ = oracle.sub_r_hosvd(X64, sp.ranks, sk)
        Ub = [u.double().cpu().numpy() for u in U[m:m + d]]
        Gb = G[ti].double().cpu().numpy()
        # the same sketch / QR / W kernels as the single-tensor path: bitwise
        single = T.sub_r_hosvd(X, sp.ranks, skd)
        for a, b in zip(U[m:m + d], single.F):
            assert torch.equal(a, b)
        # against the oracle: the core on the GPU's factors, then the error
        G_chk = oracle.core(X64, Ub)
        np.testing.assert_allclose(Gb, G_chk, rtol=0, atol=1e-6 * np.abs(G_chk).max())
        # the oracle's factors at the library's output precision (FP32
        # storage of U moves eps by ~1e-5 relative at eps ~ 1e-4, first order
        # through the residual), with the oracle's core on them
        U_or32 = [u.astype(np.float32).astype(np.float64) for u in U_or]
        eps_gpu = oracle.rel_error(X64, Gb, Ub)
        eps_or = oracle.rel_error(X64, oracle.core(X64, U_or32), U_or32)
        assert abs(eps_gpu - eps_or) <= 1e-5 * eps_or, (sp.dims, eps_gpu, eps_or)
        for a, b in zip(Ub, U_or):
            assert oracle.projector_distance(a, b) < 1e-4
        m += d


def test_batch_graph_replays_match_eager():
    items = make_batch(small_specs(), cfg=45)
    plan, U, G, info = plan_for(items)
    plan.run()
    torch.cuda.synchronize()
    ref_U = [u.clone() for u in U]
    ref_G = [g.clone() for g in G]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        plan.run(stream=s)     # the warm-up torch asks for before capture
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=s):
        plan.run(stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        for t in U + G:
            t.fill_(float("nan"))     # eager work between the replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(U, ref_U):
            assert torch.equal(a, b), rep
        for a, b in zip(G, ref_G):
            assert torch.equal(a, b), rep


def test_batch_autotune_keeps_results():
    items = make_batch(small_specs(), cfg=46)
    plan, U, G, info = plan_for(items)
    plan.run()
    torch.cuda.synchronize()
    ref = [g.clone() for g in G]
    report = plan.autotune()
    assert "chosen" in report
    for g in G:
        g.zero_()
    plan.run()
    torch.cuda.synchronize()
    for a, b in zip(G, ref):
        assert torch.equal(a, b)


def test_batch_rejects_unsupported():
    from paper_2603_21379_amd import binding as B
    X = torch.zeros(4, 5, 200, dtype=torch.float32, device="cuda")
    om = [torch.zeros(8, 3, dtype=torch.float32, device="cuda") for _ in range(3)]
    idx = [torch.arange(8, dtype=torch.int64, device="cuda") for _ in range(3)]
    U = [torch.zeros(n, 2, dtype=torch.float32, device="cuda") for n in (4, 5, 200)]
    G = [torch.zeros(2, 2, 2, dtype=torch.float32, device="cuda")]
    with pytest.raises(B.TkError, match="trailing modes"):
        B.BatchPlan([X], [(2, 2, 2)], list(zip(idx, om)), U, G)

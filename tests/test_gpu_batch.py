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


def plan_for(items, resid=False):
    """The plan of a batch; with resid, every run also writes the per-tensor
    (||X - X_hat||^2, ||X||^2) into the returned FP64 vector."""
    from paper_2603_21379_amd import binding as B
    X = [it[3] for it in items]
    ranks = [it[0].ranks for it in items]
    sketches = [s for it in items for s in it[4]]
    U = [torch.empty(n, r, dtype=torch.float32, device="cuda") for it in items
         for n, r in zip(it[0].dims, it[0].ranks)]
    G = [torch.empty(it[0].ranks, dtype=torch.float32, device="cuda") for it in items]
    info = torch.zeros(sum(len(it[0].dims) for it in items), dtype=torch.int32, device="cuda")
    r2 = torch.full((2 * len(items),), float("nan"), dtype=torch.float64, device="cuda") if resid else None
    plan = B.BatchPlan(X, ranks, sketches, U, G, info, resid2=r2)
    if resid:
        return plan, U, G, info, r2
    return plan, U, G, info


def small_specs():
    return synthgen.batch_specs(12, cfg=44, nmin=5, nmax=40, rmin=2, rmax=9, cap=60000)


def wide_specs():
    # trailing modes up to 96 (six 16-row tiles), ranks up to 16, ragged sizes
    return synthgen.batch_specs(8, cfg=47, nmin=5, nmax=96, rmin=2, rmax=16, cap=300000)


U32 = 2.0 ** -24


def r2_rtol(eps, N):
    """Relative tolerance of ||X - X_hat||^2 from the batched pass.  X_hat is
    formed in FP32 (FP32 expanded core, FP32 P, FP32 MFMA sums of <= 16
    terms): an error delta of at most about 8 u x_rms per entry, with no
    relation to d = x - x_hat.  It moves sum d^2 by 2 sum d delta (random
    sign: relative std 2 delta / (d_rms sqrt N), five of them allowed) and by
    sum delta^2 ((delta / d_rms)^2), with d_rms = eps x_rms; the squares go
    through FP32 sums of at most 144 terms per lane and slab before the FP64
    sums (<= 144 u)."""
    rd = 8 * U32 / eps
    return 144 * U32 + 10 * rd / np.sqrt(N) + rd * rd


def check_resid2(items, U, G, r2):
    """The batched residual against the oracle's, per tensor, on the stored
    tensor and the run's own core and factors."""
    r2h = r2.cpu().numpy()
    m = 0
    for ti, it in enumerate(items):
        sp, inp = it[0], it[1]
        d = len(sp.dims)
        X64 = inp.X.astype(np.float64)
        Ub = [u.double().cpu().numpy() for u in U[m:m + d]]
        Gb = G[ti].double().cpu().numpy()
        ref = oracle.reconstruct(Gb, Ub)
        x2, d2 = np.sum(X64 ** 2), np.sum((X64 - ref) ** 2)
        np.testing.assert_allclose(r2h[2 * ti + 1], x2, rtol=144 * U32, err_msg=str(sp.dims))
        tol = r2_rtol(np.sqrt(d2 / x2), X64.size)
        np.testing.assert_allclose(r2h[2 * ti], d2, rtol=tol, err_msg=str(sp.dims))
        m += d
    return r2h


def test_batch_matches_oracle_and_single_path():
    from paper_2603_21379_amd import tucker as T
    items = make_batch(small_specs())
    plan, U, G, info, r2 = plan_for(items, resid=True)
    plan.run()
    torch.cuda.synchronize()
    assert int(info.abs().sum()) == 0
    r2h = check_resid2(items, U, G, r2)
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
        # the run's own residual, as the error it reports
        eps_run = float(np.sqrt(r2h[2 * ti] / r2h[2 * ti + 1]))
        tol = 1e-5 + 0.5 * r2_rtol(eps_or, X64.size) + 72 * U32
        assert abs(eps_run - eps_or) <= tol * eps_or, (sp.dims, eps_run, eps_or)
        for a, b in zip(Ub, U_or):
            assert oracle.projector_distance(a, b) < 1e-4
        m += d


def test_batch_residual_wide_trailing_modes():
    """Trailing modes up to 96 and ranks up to 16: every tile count of the
    residual pass, ragged last tiles, leading-mode expansions over several
    32-row blocks."""
    specs = wide_specs()
    assert max(max(sp.dims[-2:]) for sp in specs) > 80
    items = make_batch(specs, cfg=47)
    plan, U, G, info, r2 = plan_for(items, resid=True)
    plan.run()
    torch.cuda.synchronize()
    assert int(info.abs().sum()) == 0
    check_resid2(items, U, G, r2)
    # the core of every tensor (whole-slab core pass with four to six tiles,
    # partial cores leaving through LDS in 16- and 4-byte runs) against the
    # oracle's core on the same factors
    assert any((sp.ranks[-1] * sp.ranks[-2]) % 4 for sp in specs)
    m = 0
    for ti, (sp, inp, sk, X, skd) in enumerate(items):
        d = len(sp.dims)
        Ub = [u.double().cpu().numpy() for u in U[m:m + d]]
        G_chk = oracle.core(inp.X.astype(np.float64), Ub)
        np.testing.assert_allclose(G[ti].double().cpu().numpy(), G_chk, rtol=0, atol=1e-6 * np.abs(G_chk).max(),
                                   err_msg=str(sp.dims))
        m += d


def test_batch_graph_replays_match_eager():
    items = make_batch(small_specs(), cfg=45)
    plan, U, G, info, r2 = plan_for(items, resid=True)
    plan.run()
    torch.cuda.synchronize()
    ref_U = [u.clone() for u in U]
    ref_G = [g.clone() for g in G]
    ref_r2 = r2.clone()
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
        for t in U + G + [r2]:
            t.fill_(float("nan"))     # eager work between the replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(U, ref_U):
            assert torch.equal(a, b), rep
        for a, b in zip(G, ref_G):
            assert torch.equal(a, b), rep
        assert torch.equal(r2, ref_r2), rep


def test_batch_autotune_keeps_results(tmp_path):
    items = make_batch(small_specs(), cfg=46)
    plan, U, G, info = plan_for(items)
    plan.run()
    torch.cuda.synchronize()
    ref = [g.clone() for g in G]
    cache = str(tmp_path / "schedules.json")
    report = plan.autotune(cache=cache)
    assert "chosen" in report
    for g in G:
        g.zero_()
    plan.run()
    torch.cuda.synchronize()
    for a, b in zip(G, ref):
        assert torch.equal(a, b)
    # a second plan of the same shapes takes the stored choice without timing
    plan2, U2, G2, _ = plan_for(items)
    report2 = plan2.autotune(cache=cache)
    assert report2.startswith("cached") and plan2.schedule() == plan.schedule()
    plan2.run()
    torch.cuda.synchronize()
    for a, b in zip(G2, ref):
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

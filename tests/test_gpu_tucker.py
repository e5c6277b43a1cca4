"""GPU parity of the Sub-R-HOSVD path (sketch, CholeskyQR2 + W step, core,
residual) against the FP64 oracle on the same seeded inputs and sketches.

Tolerances (relative reconstruction error eps vs the oracle's):
FP64 1e-10, FP32 1e-5, BF16/FP16 3e-3 (as |eps_gpu - eps_or| / eps_or); the
FP64 cases at 64^3 add four times the error's spread under unit-roundoff
perturbations of the test matrices (tests/tucker_parity.py).
Factor comparisons go through projectors and canonical column signs.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synthgen
import tucker_parity
from synthgen import configs

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5, "bf16": 3e-3, "f16": 3e-3}
TORCH_DT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}


def to_device(X, dtype):
    if dtype == "bf16":
        t = torch.from_numpy(X.view(np.int16)).cuda().view(torch.bfloat16)
        return t
    return torch.from_numpy(X).cuda()


def run_case(dims, ranks, decay, noise, p, ss, dtype, cfg, dense=False, core_factor="U",
             exact_ell=None):
    from paper_2603_21379_amd import tucker as T
    inp = synthgen.tucker_tensor(dims, ranks, decay, noise, cfg=cfg, dtype=dtype)
    ells = exact_ell or synthgen.default_ell(dims, ranks, p)
    fdt = synthgen.factor_dtype(dtype)
    sk = synthgen.mode_sketches(dims, ells, ss, cfg=cfg, omega_dtype=fdt, dense=dense)
    X64 = synthgen.to_f64(inp.X, dtype)
    G_or, U_or, Q_or, Y_or, Z_or = oracle.sub_r_hosvd(X64, ranks, sk, core_factor=core_factor)
    Xd = to_device(inp.X, dtype)
    skd = T.mode_sketches_to_device(sk, dims, "cuda", TORCH_DT[fdt])
    res = T.sub_r_hosvd(Xd, ranks, skd, core_factor=core_factor)
    eps_gpu = T.rel_error(Xd, res.G, res.F)
    torch.cuda.synchronize()
    F_or = U_or if core_factor == "U" else Q_or
    eps_or = oracle.rel_error(X64, G_or, F_or)
    out = dict(inp=inp, X64=X64, sk=sk, G_or=G_or, U_or=U_or, Q_or=Q_or, Y_or=Y_or, Z_or=Z_or,
               F_or=F_or, eps_or=eps_or, eps_gpu=eps_gpu,
               G=res.G.double().cpu().numpy(), F=[f.double().cpu().numpy() for f in res.F],
               Q=[q.cpu().numpy() for q in res.Q],
               Y=[synthgen.to_f64(y.cpu().view(torch.int16).numpy().view(np.uint16), "bf16")
                  if dtype == "bf16" else y.double().cpu().numpy() for y in res.Y],
               info=res.info.cpu().numpy())
    return out


def check_common(o, dtype, ptol, eps_gate=None):
    # the gather is a copy: bit-exact
    for a, b in zip(o["Y"], o["Y_or"]):
        np.testing.assert_array_equal(a, b)
    # factors orthonormal at their storage precision
    otol = 1e-12 if dtype == "f64" else 1e-5
    for F in o["F"]:
        assert np.max(np.abs(F.T @ F - np.eye(F.shape[1]))) < otol
    for a, b in zip(o["F"], o["F_or"]):
        assert oracle.projector_distance(a, b) < ptol
    # core kernel alone: the oracle's core on the GPU's own factors
    G_chk = oracle.core(o["X64"], o["F"])
    scale = np.abs(G_chk).max()
    # BF16/FP16 tensors: the factors and the stage-1 results enter the MFMA as
    # hi + lo 16-bit pairs (about 16 significant bits, 2^-17 relative per
    # operand), so the core carries a few 1e-6 of max|G| where FP32 carries 1e-7
    ctol = {"f64": 1e-12, "f32": 1e-6, "bf16": 2e-5, "f16": 2e-5}[dtype]
    rel = abs(o["eps_gpu"] - o["eps_or"]) / o["eps_or"]
    gate = TOL[dtype] if eps_gate is None else eps_gate / o["eps_or"]
    assert rel <= gate, (o["eps_gpu"], o["eps_or"], rel, gate)
    np.testing.assert_allclose(o["G"], G_chk, rtol=0, atol=ctol * scale)


def test_c1_fp64_sampled():
    c = configs.C1
    o = run_case(c.dims, c.ranks, c.decay, c.noise, c.p, synthgen.default_s(c.dims), c.dtype,
                 c.cfg_id)
    # 1e-10 of the error plus the error's own spread under unit-roundoff
    # perturbations of the test matrices (about 6e-11 of it here)
    spread = tucker_parity.eps_spread(o["X64"], c.ranks, o["sk"], o["eps_or"])
    check_common(o, "f64", 1e-10, tucker_parity.eps_gate(o["eps_or"], spread, 1e-10))
    # thin QR is unique (R_ii > 0); its columns are determined to ~u kappa(Z)
    for z, zo, Z in zip(o["Q"], o["Q_or"], o["Z_or"]):
        sv = np.linalg.svd(Z, compute_uv=False)
        np.testing.assert_allclose(z, zo, rtol=0, atol=100 * 1.1e-16 * sv[0] / sv[-1])
    for a, b in zip(o["F"], o["F_or"]):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-9)
    np.testing.assert_allclose(o["G"], o["G_or"], rtol=0, atol=1e-9 * np.abs(o["G_or"]).max())
    assert (o["info"] == 0).all()


def test_c1_fp64_dense_sketch():
    c = configs.C1
    o = run_case(c.dims, c.ranks, c.decay, c.noise, c.p, [0, 0, 0], c.dtype, c.cfg_id, dense=True)
    spread = tucker_parity.eps_spread(o["X64"], c.ranks, o["sk"], o["eps_or"])
    check_common(o, "f64", 1e-10, tucker_parity.eps_gate(o["eps_or"], spread, 1e-10))


def test_c1_exact_rank_shifted_qr():
    """sigma = 0: rank(Z_k) = 8 < ell = 13, the Gram is singular, the shifted
    first pass runs (info = 1) and the decomposition is exact."""
    c = configs.C1
    o = run_case(c.dims, c.ranks, c.decay, 0.0, c.p, synthgen.default_s(c.dims), c.dtype, 31)
    assert o["eps_or"] < 1e-12
    assert o["eps_gpu"] < 1e-12
    # the first pass was shifted and no Cholesky failed
    assert ((o["info"] & 1) == 1).all() and ((o["info"] & 4) == 0).all()
    for F in o["F"]:
        assert np.max(np.abs(F.T @ F - np.eye(F.shape[1]))) < 1e-12
    for a, b in zip(o["F"], o["F_or"]):
        assert oracle.projector_distance(a, b) < 1e-10


def test_c1_q_core():
    c = configs.C1
    o = run_case(c.dims, c.ranks, c.decay, c.noise, c.p, synthgen.default_s(c.dims), c.dtype,
                 c.cfg_id, core_factor="Q")
    spread = tucker_parity.eps_spread(o["X64"], c.ranks, o["sk"], o["eps_or"], core_factor="Q")
    assert abs(o["eps_gpu"] - o["eps_or"]) <= tucker_parity.eps_gate(o["eps_or"], spread, 1e-10)
    # Range(Q_k) includes noise directions determined only to ~u kappa(Z_k)
    for a, b, Z in zip(o["F"], o["Q_or"], o["Z_or"]):
        sv = np.linalg.svd(Z, compute_uv=False)
        assert oracle.projector_distance(a, b) < 100 * 1.1e-16 * sv[0] / sv[-1]


def test_c2_small_fp32():
    c = configs.C2_SMALL
    o = run_case(c.dims, c.ranks, c.decay, c.noise, c.p, synthgen.default_s(c.dims), c.dtype,
                 c.cfg_id)
    check_common(o, "f32", 1e-5)


@pytest.mark.parametrize("dtype", ["bf16", "f16", "f32"])
def test_c3_small_low_precision(dtype):
    c = configs.C3_SMALL
    o = run_case(c.dims, c.ranks, c.decay, c.noise, c.p, synthgen.default_s(c.dims), dtype,
                 c.cfg_id)
    check_common(o, dtype, 1e-4)


def test_ragged_order2_and_order5():
    # order 2: rows/cols not multiples of the tiles, s not a multiple of 32
    o = run_case((131, 77), (5, 5), 0.6, 1e-3, 5, [77, 131], "f64", 41)
    check_common(o, "f64", 1e-9)
    o = run_case((7, 9, 5, 6, 11), (3, 2, 3, 3, 4), 0.7, 1e-2, 4, [37, 45, 29, 33, 55], "f32", 42)
    check_common(o, "f32", 1e-4)


def test_full_basis_gives_exact_reconstruction():
    """ell_k = n_k and every fiber: Q_k is a full basis and X_hat = X for any X."""
    o = run_case((6, 7, 8), (6, 7, 8), 0.9, 1.0, 0, [0, 0, 0], "f64", 43, dense=True,
                 core_factor="Q", exact_ell=[6, 7, 8])
    assert o["eps_gpu"] < 1e-13
    assert o["eps_or"] < 1e-13


def test_s_equals_ell_minimum_sample():
    o = run_case((20, 18, 16), (3, 3, 3), 0.5, 1e-4, 4, [7, 7, 7], "f64", 44)
    check_common(o, "f64", 1e-8)


def test_reconstruct_materialised_matches_oracle():
    from paper_2603_21379_amd import tucker as T
    rng = np.random.default_rng(7)
    dims, cols = (9, 70, 33), (4, 5, 6)
    G = rng.standard_normal(cols)
    F = [np.linalg.qr(rng.standard_normal((n, c)))[0] for n, c in zip(dims, cols)]
    for dt in (torch.float64, torch.float32):
        Gd = torch.from_numpy(G).to("cuda", dt)
        Fd = [torch.from_numpy(f).to("cuda", dt) for f in F]
        Xh = T.reconstruct(dims, Gd, Fd).double().cpu().numpy()
        ref = oracle.reconstruct(synthgen.to_f64(np.asarray(Gd.cpu()), "f64"),
                                 [np.asarray(f.double().cpu()) for f in Fd])
        tol = 1e-13 if dt == torch.float64 else 1e-6
        np.testing.assert_allclose(Xh, ref, atol=tol * np.abs(ref).max())


def test_bitwise_repeatable():
    from paper_2603_21379_amd import tucker as T
    c = configs.C2_SMALL
    inp = synthgen.tucker_tensor(c.dims, c.ranks, c.decay, c.noise, cfg=c.cfg_id, dtype="f32")
    sk = synthgen.mode_sketches(c.dims, synthgen.default_ell(c.dims, c.ranks, c.p),
                                synthgen.default_s(c.dims), cfg=c.cfg_id, omega_dtype="f32")
    Xd = torch.from_numpy(inp.X).cuda()
    skd = T.mode_sketches_to_device(sk, c.dims, "cuda", torch.float32)
    a = T.sub_r_hosvd(Xd, c.ranks, skd)
    b = T.sub_r_hosvd(Xd, c.ranks, skd)
    assert torch.equal(a.G, b.G)
    for x, y in zip(a.F, b.F):
        assert torch.equal(x, y)


@pytest.mark.parametrize("dims,ranks", [
    ((16, 20, 30, 132), (5, 6, 12, 20)),     # two column blocks, the second 4 wide
    ((8, 40, 33, 96), (4, 7, 32, 32)),       # odd rows, one partial block, full 32 ranks
    ((4, 64, 256, 256), (4, 16, 32, 32)),    # the 256^4 slab shape
])
def test_fp32_fused_streaming_core(dims, ranks):
    """The FP32 MFMA streaming pass (two trailing modes per read of X) against
    the oracle core on the same factors, and the end-to-end error gate."""
    o = run_case(dims, ranks, 0.8, 1e-4, 6, synthgen.default_s(dims), "f32", 61)
    check_common(o, "f32", 1e-5)


@pytest.mark.parametrize("dims,cols", [((16, 20, 30, 132), (5, 6, 12, 20)),
                                       ((300, 33, 96), (7, 32, 32)),
                                       ((2100, 40, 64), (5, 12, 20))])   # 1 or 2 slabs a wave
def test_fp32_fused_residual_and_xhat(dims, cols):
    """The FP32 MFMA residual pass: materialised X_hat and the FP64 sums
    ||X - X_hat||^2, ||X||^2 against the oracle on the same core and factors."""
    from paper_2603_21379_amd import binding as Bd
    rng = np.random.default_rng(9)
    X = rng.standard_normal(dims).astype(np.float32)
    G = rng.standard_normal(cols).astype(np.float32)
    F = [np.linalg.qr(rng.standard_normal((n, c)))[0].astype(np.float32) for n, c in zip(dims, cols)]
    Xd = torch.from_numpy(X).cuda()
    Gd = torch.from_numpy(G).cuda()
    Fd = [torch.from_numpy(f).cuda() for f in F]
    Xh = torch.empty(dims, dtype=torch.float32, device="cuda")
    r2 = torch.zeros(2, dtype=torch.float64, device="cuda")
    Bd.tucker_reconstruct(list(dims), Gd, Fd, Xref=Xd, Xhat=Xh, resid2=r2)
    torch.cuda.synchronize()
    ref = oracle.reconstruct(G.astype(np.float64), [f.astype(np.float64) for f in F])
    np.testing.assert_allclose(Xh.cpu().numpy(), ref, rtol=0, atol=2e-6 * np.abs(ref).max())
    X64 = X.astype(np.float64)
    r2h = r2.cpu().numpy()
    # both sums take each lane's 32 entries of a row tile in FP32 before the
    # FP64 sum: a sum of 32 nonnegative FP32 terms is within 32 u = 1.9e-6
    # relative of the exact one
    np.testing.assert_allclose(r2h[1], np.sum(X64 ** 2), rtol=2e-6)
    np.testing.assert_allclose(r2h[0], np.sum((X64 - ref) ** 2), rtol=2e-6)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("dims,cols", [((30, 40, 40), (5, 10, 10)),       # the 40^6 slab shape
                                       ((7, 9, 33, 17), (3, 4, 16, 7)),  # ragged tiles, full 16 ranks
                                       ((7, 9, 33, 18), (3, 4, 16, 7)),  # ragged, even rows: 8-byte loads of 2-byte entries
                                       ((3, 64, 64), (2, 16, 16)),       # largest slab
                                       ((5000, 3, 5), (2, 2, 3))])       # many tiny slabs
def test_small_mode_streaming_residual(dims, cols, dtype):
    """The small-mode MFMA residual pass (BF16, FP16, FP32 tensors): the FP64
    sums ||X - X_hat||^2, ||X||^2 against the oracle's on the stored values
    and the same core and factors."""
    from paper_2603_21379_amd import binding as Bd
    rng = np.random.default_rng(11)
    X64 = rng.standard_normal(dims)
    Xs = synthgen.to_storage(X64, dtype)
    Xo = synthgen.to_f64(Xs, dtype)
    G = rng.standard_normal(cols).astype(np.float32)
    F = [np.linalg.qr(rng.standard_normal((n, c)))[0].astype(np.float32) for n, c in zip(dims, cols)]
    r2 = torch.zeros(2, dtype=torch.float64, device="cuda")
    Bd.tucker_reconstruct(list(dims), torch.from_numpy(G).cuda(), [torch.from_numpy(f).cuda() for f in F],
                          Xref=to_device(Xs, dtype), resid2=r2)
    torch.cuda.synchronize()
    ref = oracle.reconstruct(G.astype(np.float64), [f.astype(np.float64) for f in F])
    r2h = r2.cpu().numpy()
    # X_hat in FP32 (FP32 expanded core, FP32 MFMA): |d| ~ |x| here, so about
    # 1e-7 relative in ||X - X_hat||^2; the squares summed in FP32 over at most
    # 64 terms per lane and slab before the FP64 sum: within 64 u = 3.8e-6
    np.testing.assert_allclose(r2h[1], np.sum(Xo ** 2), rtol=4e-6)
    np.testing.assert_allclose(r2h[0], np.sum((Xo - ref) ** 2), rtol=4e-6)


def _core_direct(dims, cols, dtype, seed):
    """G = X x_k F_k^T on the GPU vs the FP64 oracle on the stored values."""
    from paper_2603_21379_amd import binding as Bd
    rng = np.random.default_rng(seed)
    X64 = rng.standard_normal(dims)
    Xs = synthgen.to_storage(X64, dtype)
    Xo = synthgen.to_f64(Xs, dtype)
    F = [np.linalg.qr(rng.standard_normal((n, c)))[0].astype(np.float32) for n, c in zip(dims, cols)]
    Xd = to_device(Xs, dtype)
    Fd = [torch.from_numpy(f).cuda() for f in F]
    G = torch.empty(cols, dtype=torch.float32, device="cuda")
    Bd.tucker_core(Xd, Fd, G)
    torch.cuda.synchronize()
    ref = oracle.core(Xo, [f.astype(np.float64) for f in F])
    return G.double().cpu().numpy(), ref


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("dims,cols", [
    ((5, 7, 33, 50), (3, 4, 9, 16)),          # two modes per pass, ragged tiles and chunks
    ((2048, 3, 9, 12), (6, 2, 5, 7)),         # third mode accumulated in registers
    ((64, 32, 10, 24, 40), (4, 5, 6, 10, 10)),  # the 40^6 slab shape, third mode accumulated
    ((2, 128, 128), (2, 16, 16)),             # largest slab, full 16 ranks
    ((2048, 2, 72, 128), (3, 2, 16, 16)),     # largest slab with the third mode
])
def test_small_mode_streaming_core(dims, cols, dtype):
    """The 16x16-tile MFMA streaming pass (BF16/FP16 with hi+lo factors and
    stage-1 results, FP32 direct) against the FP64 oracle core."""
    G, ref = _core_direct(dims, cols, dtype, 71)
    tol = 2e-6 if dtype == "f32" else 5e-5
    np.testing.assert_allclose(G, ref, rtol=0, atol=tol * np.abs(ref).max())


def test_small_mode_streaming_core_odd_width_fp32():
    """An odd contiguous mode (partial float4 at every row end) on the FP32 pass."""
    G, ref = _core_direct((6, 5, 33, 51), (3, 4, 9, 13), "f32", 72)
    np.testing.assert_allclose(G, ref, rtol=0, atol=2e-6 * np.abs(ref).max())

"""Sketch widths above 64 (the wide QR / W-step path) against the oracle.

The uneven shape follows the meteorological tensor of the Tucker experiments
(Section 3.3.2): six modes from 5 to 270 with truncation ranks up to 150,
where ell = min(r + p, n) is capped at n on the first mode and exceeds 64 on
the last.  The stand-in keeps the caps with a last mode of ell = 90.
"""
import numpy as np
import pytest
import torch

import oracle
import synthgen
from synthgen import configs

from test_gpu_tucker import check_common, run_case

pytestmark = pytest.mark.gpu


def test_uneven_small_fp32_wide_last_mode():
    c = configs.C8_SMALL
    ells = synthgen.default_ell(c.dims, c.ranks, c.p)
    assert ells[0] == c.dims[0] and ells[-1] > 64
    o = run_case(c.dims, c.ranks, c.decay, c.noise, c.p, synthgen.default_s(c.dims), c.dtype,
                 c.cfg_id)
    check_common(o, "f32", 1e-5)
    assert not o["info"].any()


def test_odd_wide_ell_fp64():
    # ell = 69 (odd: the Jacobi pairing pads one index); s = 700 sampled
    # fibers span several 32-column tiles of the products and a ragged tail
    o = run_case((70, 40, 30), (65, 5, 5), 0.97, 1e-6, 4, [700, 400, 300], "f64", 61)
    assert o["Q"][0].shape == (70, 69)
    check_common(o, "f64", 1e-8)
    # Q of the wide path against the oracle's Q: Q = Z R^{-1} with R_ii > 0 is
    # unique, and both sides determine it to about u cond(Z) (the four columns
    # beyond the rank-65 signal sit at the noise level, cond(Z) ~ 1e6)
    sv = np.linalg.svd(o["Z_or"][0], compute_uv=False)
    np.testing.assert_allclose(o["Q"][0], o["Q_or"][0], rtol=0, atol=100 * 1.1e-16 * sv[0] / sv[-1])


def test_wide_full_basis_reconstructs_exactly():
    """ell = n = 100 on the first mode with every fiber: Q is a full basis."""
    o = run_case((100, 12, 10), (100, 12, 10), 0.9, 1.0, 0, [0, 0, 0], "f64", 62, dense=True,
                 core_factor="Q", exact_ell=[100, 12, 10])
    assert o["eps_gpu"] < 1e-12
    assert o["eps_or"] < 1e-12
    Q = o["Q"][0]
    assert np.max(np.abs(Q.T @ Q - np.eye(100))) < 1e-12


def test_wide_exact_rank_sketch_is_shifted():
    """A sketch of exact rank below ell (a rank-70 tensor sketched 90 wide, no
    noise): the first Cholesky fails, the shifted pass repairs it and info
    says so; the basis is still orthonormal and captures the tensor."""
    o = run_case((96, 30, 20), (70, 4, 4), 0.98, 0.0, 20, [600, 300, 200], "f64", 63)
    assert o["Q"][0].shape[1] == 90
    assert int(o["info"][0]) & 1
    Q = o["Q"][0]
    assert np.max(np.abs(Q.T @ Q - np.eye(90))) < 1e-10
    assert o["eps_gpu"] < 1e-10


def test_wide_bitwise_repeatable():
    from paper_2603_21379_amd import tucker as T
    c = configs.C8_SMALL
    inp = synthgen.tucker_tensor(c.dims, c.ranks, c.decay, c.noise, cfg=c.cfg_id, dtype=c.dtype)
    ells = synthgen.default_ell(c.dims, c.ranks, c.p)
    sk = synthgen.mode_sketches(c.dims, ells, synthgen.default_s(c.dims), cfg=c.cfg_id,
                                omega_dtype="f32")
    X = torch.from_numpy(inp.X).cuda()
    skd = T.mode_sketches_to_device(sk, c.dims, "cuda", torch.float32)
    a = T.sub_r_hosvd(X, c.ranks, skd)
    b = T.sub_r_hosvd(X, c.ranks, skd)
    torch.cuda.synchronize()
    for fa, fb in zip(a.F, b.F):
        assert torch.equal(fa, fb)
    assert torch.equal(a.G, b.G)


@pytest.mark.parametrize("dims,cols", [
    # the last mode has the largest reduction (300 -> 100): it is contracted
    # first, on the last-mode MFMA kernel (two column groups of 96 and 4,
    # q tail of 12, 3000 rows), then the two leading modes
    ((50, 60, 300), (40, 50, 100)),
    # 150 columns (two groups, the second partial), Q = 270 as in the uneven
    # shape, rows not a multiple of 32
    ((7, 11, 270), (6, 9, 150)),
    # the uneven stand-in's chain: 20 -> 12 and 16 -> 12 on the middle-mode
    # MFMA kernel, then 96 -> 80 on the last-mode kernel
    ((5, 6, 8, 20, 16, 96), (5, 6, 8, 12, 12, 80)),
])
def test_wide_factor_core_fp32(dims, cols):
    """FP32 core with factors wider than 64 columns against the FP64 oracle
    (the order of the contractions and their kernels are the library's)."""
    from test_gpu_tucker import _core_direct
    G, ref = _core_direct(dims, cols, "f32", 72)
    np.testing.assert_allclose(G, ref, rtol=0, atol=2e-6 * np.abs(ref).max())


@pytest.mark.parametrize("dims,cols", [
    ((7, 11, 270), (6, 9, 150)),      # three column groups of the expansion, q tail of 22
    ((3, 5, 4, 100), (3, 4, 4, 65)),  # the narrowest wide last mode, 60 rows
])
def test_wide_last_mode_reconstruct_and_residual_fp32(dims, cols):
    """FP32 reconstruction with a last factor wider than 64 columns (expanded
    on MFMA): X_hat against the oracle, and the streamed residual against the
    FP64 sums over the stored values."""
    from paper_2603_21379_amd import tucker as T
    rng = np.random.default_rng(9)
    G = rng.standard_normal(cols).astype(np.float32)
    F = [np.linalg.qr(rng.standard_normal((n, c)))[0].astype(np.float32) for n, c in zip(dims, cols)]
    Gd = torch.from_numpy(G).cuda()
    Fd = [torch.from_numpy(f).cuda() for f in F]
    Xh = T.reconstruct(dims, Gd, Fd).double().cpu().numpy()
    ref = oracle.reconstruct(G.astype(np.float64), [f.astype(np.float64) for f in F])
    np.testing.assert_allclose(Xh, ref, rtol=0, atol=1e-6 * np.abs(ref).max())
    X = (ref + 0.01 * rng.standard_normal(dims)).astype(np.float32)
    r2 = T.residual(torch.from_numpy(X).cuda(), Gd, Fd).cpu().numpy()
    X64 = X.astype(np.float64)
    np.testing.assert_allclose(r2[1], np.sum(X64 ** 2), rtol=1e-12)
    np.testing.assert_allclose(r2[0], np.sum((X64 - ref) ** 2), rtol=1e-4)

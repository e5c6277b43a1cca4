"""GPU parity of the seeded device-side sketch draw (tucker_draw_sketches)
against the oracle's definition of the same stream (oracle/sampling.py):
indices bit-exact, Omega within the rounding of the device's and the host's
libm (FP64) or of the storage (FP32), and a Sub-R-HOSVD run on device-drawn
sketches against the oracle run on the oracle's draw."""
import math

import numpy as np
import pytest
import torch

import oracle
import synthgen

pytestmark = pytest.mark.gpu

SEED = 2603_21379


def _draw(ncols, s, ell, seed, dtype):
    from paper_2603_21379_amd import binding as B
    idx, om = B.draw_sketches(ncols, s, ell, seed, omega_dtype=dtype)
    torch.cuda.synchronize()
    return [i.cpu().numpy() for i in idx], [o.double().cpu().numpy() for o in om]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_draw_matches_oracle_stream(dtype):
    # the 256^4 workload's four modes, a full draw (s = ncols), an empty unit,
    # a huge column range and the size limit
    ncols = [256 ** 3] * 4 + [100, 7, 2 ** 61, 5000]
    s = [2560] * 4 + [100, 0, 333, 4096]
    ell = [42] * 4 + [5, 3, 17, 2]
    idx, om = _draw(ncols, s, ell, SEED, dtype)
    for k in range(len(ncols)):
        ref = oracle.draw_indices(ncols[k], s[k], SEED, k)
        np.testing.assert_array_equal(idx[k], ref)
        ref_om = oracle.draw_omega(s[k], ell[k], SEED, k)
        if dtype == torch.float64:
            np.testing.assert_allclose(om[k], ref_om, rtol=1e-14, atol=1e-15)
        else:
            np.testing.assert_allclose(om[k], ref_om.astype(np.float32).astype(np.float64),
                                       rtol=2.0 ** -23, atol=1e-30)


@pytest.mark.parametrize("case", range(4))
def test_draw_indices_dense_collisions(case):
    # small column ranges with s close to ncols: most steps collide and the
    # rejected steps chain into each other; also the full and nearly full draw
    # at the size limit
    rng = np.random.default_rng(1000 + case)
    ncols = [int(n) for n in rng.integers(1, 80, size=30)] + [4096, 4097]
    s = [int(rng.integers(max(0, n - 8), n + 1)) for n in ncols[:30]] + [4096, 4096]
    seed = int(rng.integers(0, 2 ** 63))
    idx, _ = _draw(ncols, s, [1] * len(ncols), seed, torch.float64)
    for k in range(len(ncols)):
        np.testing.assert_array_equal(idx[k], oracle.draw_indices(ncols[k], s[k], seed, k))


def test_draw_rejects_bad_sizes():
    from paper_2603_21379_amd import binding as B
    with pytest.raises(B.TkError):
        B.draw_sketches([10], [11], [2], 1)
    with pytest.raises(B.TkError):
        B.draw_sketches([10 ** 6], [4097], [2], 1)
    with pytest.raises(B.TkError):
        B.draw_sketches([10], [5], [0], 1)


def test_sub_r_hosvd_on_device_drawn_sketches():
    # the FP64 64^3 workload: the library draws its own sketches on the GPU,
    # the oracle draws the same stream on the host
    from paper_2603_21379_amd import binding as B
    from paper_2603_21379_amd import tucker as T
    dims, ranks, p = (64, 64, 64), (8, 8, 8), 5
    inp = synthgen.tucker_tensor(dims, ranks, 0.5, 1e-6, cfg=1, dtype="f64")
    N = math.prod(dims)
    ells = [r + p for r in ranks]
    ss = [10 * n for n in dims]
    ncols = [N // n for n in dims]
    idx, om = B.draw_sketches(ncols, ss, ells, SEED, omega_dtype=torch.float64)
    sk_host = [synthgen.Sketch(oracle.draw_indices(ncols[k], ss[k], SEED, k),
                               oracle.draw_omega(ss[k], ells[k], SEED, k), "f64") for k in range(3)]
    G_or, U_or, _, _, _ = oracle.sub_r_hosvd(inp.X, ranks, sk_host)
    X = torch.from_numpy(inp.X).cuda()
    res = T.sub_r_hosvd(X, ranks, list(zip(idx, om)))
    eps_gpu = T.rel_error(X, res.G, res.F)
    eps_or = oracle.rel_error(inp.X, G_or, U_or)
    assert abs(eps_gpu - eps_or) / eps_or < 1e-10, (eps_gpu, eps_or)
    for F, U in zip(res.F, U_or):
        assert oracle.projector_distance(F.cpu().numpy(), U) < 1e-10

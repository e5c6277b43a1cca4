"""The no-allocation sketch entry point (tucker_sketch_all_modes_noalloc),
for callers that cannot allocate: called through the C ABI, its Z and Y are
bitwise those of tucker_sketch_all_modes with a caller workspace (same
kernels, fixed-order sums), on two calls in a row, the second on a smaller
tensor of another dtype, so the shared scratch array is reused."""
import numpy as np
import pytest
import torch

import synthgen

pytestmark = pytest.mark.gpu


def _case(dims, ranks, p, dtype, cfg):
    from paper_2603_21379_amd import tucker as T
    inp = synthgen.tucker_tensor(dims, ranks, 0.6, 1e-4, cfg=cfg, dtype=dtype)
    ells = synthgen.default_ell(dims, ranks, p)
    sk = synthgen.mode_sketches(dims, ells, synthgen.default_s(dims), cfg=cfg,
                                omega_dtype=synthgen.factor_dtype(dtype))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    X = torch.from_numpy(inp.X).cuda()
    skd = T.mode_sketches_to_device(sk, dims, "cuda", tdt)
    return X, skd, ells, [len(s.idx) for s in sk]


def _run(fn, X, skd, ells, ss, **kw):
    Z = [torch.full((n, e), float("nan"), dtype=torch.float64, device="cuda")
         for n, e in zip(X.shape, ells)]
    Y = [torch.zeros(n, s, dtype=X.dtype, device="cuda") for n, s in zip(X.shape, ss)]
    fn(X, skd, Z, Y, **kw)
    torch.cuda.synchronize()
    return [z.cpu() for z in Z], [y.cpu() for y in Y]


def test_noalloc_sketch_matches_workspace_entry_point_twice():
    from paper_2603_21379_amd import binding as B
    cases = [((72, 80, 96, 64), (8, 8, 8, 8), 5, "f32", 91),   # several row and fiber chunks
             ((17, 12, 9), (3, 3, 3), 4, "f64", 92)]            # smaller, second call
    for dims, ranks, p, dtype, cfg in cases:
        X, skd, ells, ss = _case(dims, ranks, p, dtype, cfg)
        Zr, Yr = _run(B.tucker_sketch_all_modes, X, skd, ells, ss)
        Zn, Yn = _run(B.tucker_sketch_all_modes_noalloc, X, skd, ells, ss)
        for k in range(len(dims)):
            assert torch.isfinite(Zn[k]).all()
            assert torch.equal(Zn[k], Zr[k]), (dims, k)
            assert torch.equal(Yn[k], Yr[k]), (dims, k)


def test_noalloc_sketch_rejects_scratch_above_the_limit():
    from paper_2603_21379_amd import binding as B
    # 33 chunks of 32 fibers x 4096 rows x 64 columns of FP64 partials > 64 MiB
    X = torch.zeros(4096, 2048, dtype=torch.float32, device="cuda")
    om = torch.zeros(1056, 64, dtype=torch.float32, device="cuda")
    idx = torch.arange(1056, dtype=torch.int64, device="cuda")
    Z = [torch.empty(4096, 64, dtype=torch.float64, device="cuda"),
         torch.empty(2048, 64, dtype=torch.float64, device="cuda")]
    with pytest.raises(B.TkError, match="fixed"):
        B.tucker_sketch_all_modes_noalloc(X, [(idx, om), (idx, om)], Z)

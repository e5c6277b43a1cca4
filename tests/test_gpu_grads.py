"""GPU parity of the hand-written backward (core and reconstruction VJPs
behind torch.autograd) against the oracle's closed-form gradients, which the
CPU tests pin to finite differences and to PyTorch's CPU autograd."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


def _grads_gpu(X, Fs, dtype):
    from paper_2603_21379_amd import autograd as AG
    Xd = torch.tensor(X, dtype=dtype, device="cuda", requires_grad=True)
    Fd = [torch.tensor(f, dtype=dtype, device="cuda", requires_grad=True) for f in Fs]
    L = AG.projection_loss(Xd, Fd)
    L.backward()
    torch.cuda.synchronize()
    return float(L.detach()), Xd.grad.double().cpu().numpy(), [f.grad.double().cpu().numpy() for f in Fd]


@pytest.mark.parametrize("dims,cols", [((4,) * 8, (3,) * 8), ((6, 5, 7), (2, 3, 4)),
                                       ((9, 70, 33, 5), (4, 5, 6, 3)), ((80, 6, 5), (64, 3, 2)),
                                       ((80, 6, 5), (70, 3, 2)), ((5, 6, 80), (2, 3, 70)),
                                       ((70, 6, 5), (20, 3, 2))])
def test_loss_gradients_match_oracle_fp64(dims, cols):
    rng = np.random.default_rng(1)
    X = rng.standard_normal(dims)
    Fs = [np.linalg.qr(rng.standard_normal((n, c)))[0] for n, c in zip(dims, cols)]
    L0, dX0, dF0 = oracle.loss_and_grads(X, Fs)
    L, dX, dF = _grads_gpu(X, Fs, torch.float64)
    assert abs(L - L0) <= 1e-12 * abs(L0)
    np.testing.assert_allclose(dX, dX0, rtol=0, atol=1e-11 * np.abs(dX0).max())
    for a, b in zip(dF, dF0):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-11 * np.abs(b).max())


# FP32 shapes: the first five take the fused path (the partial core of the two
# trailing modes from the streaming pass, their gradients from one MFMA pass
# over the tensor): ragged row groups and column chunks, order 3 with a long
# leading mode (its unfolded product tiled), the 16x16-tile streaming pass for
# small trailing modes, two row groups with a ragged last chunk; the last two
# keep the generic chains with wide factors (the tiled unfolded product in
# FP32, one case per layout)
FP32_CASES = [((16, 20, 30, 132), (5, 6, 12, 20)), ((16, 20, 40, 132), (4, 5, 31, 32)),
              ((300, 48, 64), (20, 12, 9)), ((20, 30, 24, 36), (3, 4, 8, 12)),
              ((260, 150, 200), (6, 31, 17)),
              ((80, 6, 5), (40, 3, 2)), ((5, 6, 80), (2, 3, 70))]


@pytest.mark.parametrize("dims,cols", FP32_CASES)
def test_loss_gradients_match_oracle_fp32(dims, cols):
    rng = np.random.default_rng(2)
    X = rng.standard_normal(dims).astype(np.float32)
    Fs = [np.linalg.qr(rng.standard_normal((n, c)))[0].astype(np.float32)
          for n, c in zip(dims, cols)]
    L0, dX0, dF0 = oracle.loss_and_grads(X.astype(np.float64), [f.astype(np.float64) for f in Fs])
    L, dX, dF = _grads_gpu(X, Fs, torch.float32)
    assert abs(L - L0) <= 1e-4 * abs(L0)
    np.testing.assert_allclose(dX, dX0, rtol=0, atol=1e-5 * np.abs(dX0).max())
    for a, b in zip(dF, dF0):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-4 * np.abs(b).max())


@pytest.mark.parametrize("dims,cols", FP32_CASES[:5])
def test_vjps_match_oracle_fp32_fused_path(dims, cols):
    """Both VJPs at arbitrary adjoints (not only the loss's), FP32, on the
    fused path, against the oracle's closed forms on the same FP32 values."""
    from paper_2603_21379_amd import binding as B
    rng = np.random.default_rng(5)
    X = rng.standard_normal(dims).astype(np.float32)
    Fs = [rng.standard_normal((n, c)).astype(np.float32) for n, c in zip(dims, cols)]
    Gb = rng.standard_normal(cols).astype(np.float32)
    G = rng.standard_normal(cols).astype(np.float32)
    H = rng.standard_normal(dims).astype(np.float32)
    X64, F64 = X.astype(np.float64), [f.astype(np.float64) for f in Fs]
    _, Fc0 = oracle.core_vjp(X64, F64, Gb.astype(np.float64))
    Gr0, Fr0 = oracle.reconstruct_vjp(G.astype(np.float64), F64, H.astype(np.float64))
    dev = lambda a: torch.from_numpy(a).cuda()
    Fd = [dev(f) for f in Fs]
    Fc = [torch.empty_like(f) for f in Fd]
    B.tucker_core_vjp(dev(X), Fd, dev(Gb), Fbar=Fc)
    Fr = [torch.empty_like(f) for f in Fd]
    Gr = torch.empty_like(dev(G))
    B.tucker_reconstruct_vjp(list(dims), dev(G), Fd, dev(H), Gbar=Gr, Fbar=Fr)
    torch.cuda.synchronize()
    for a, b in zip(Fc, Fc0):
        np.testing.assert_allclose(a.double().cpu().numpy(), b, rtol=0, atol=2e-5 * np.abs(b).max())
    for a, b in zip(Fr, Fr0):
        np.testing.assert_allclose(a.double().cpu().numpy(), b, rtol=0, atol=2e-5 * np.abs(b).max())
    np.testing.assert_allclose(Gr.double().cpu().numpy(), Gr0, rtol=0, atol=2e-5 * np.abs(Gr0).max())


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_projection_loss_vjp_scaled_without_xbar(dtype):
    """tucker_projection_loss_vjp with a loss adjoint of 0.37 and no X output
    (H then lives in the workspace): the factor gradients are 0.37 times the
    oracle's."""
    from paper_2603_21379_amd import binding as B
    dims, cols = ((16, 20, 40, 132), (4, 5, 31, 32)) if dtype == torch.float32 else ((9, 70, 33, 5), (4, 5, 6, 3))
    rng = np.random.default_rng(8)
    npdt = np.float32 if dtype == torch.float32 else np.float64
    X = rng.standard_normal(dims).astype(npdt)
    Fs = [np.linalg.qr(rng.standard_normal((n, c)))[0].astype(npdt) for n, c in zip(dims, cols)]
    _, _, dF0 = oracle.loss_and_grads(X.astype(np.float64), [f.astype(np.float64) for f in Fs])
    Xd = torch.from_numpy(X).cuda()
    Fd = [torch.from_numpy(f).cuda() for f in Fs]
    G = torch.empty(cols, dtype=dtype, device="cuda")
    B.tucker_core(Xd, Fd, G)
    lbar = torch.tensor(0.37, dtype=torch.float64, device="cuda")
    Fb = [torch.empty_like(f) for f in Fd]
    B.tucker_projection_loss_vjp(Xd, Fd, G, lbar, Xbar=None, Fbar=Fb)
    torch.cuda.synchronize()
    tol = 1e-4 if dtype == torch.float32 else 1e-11
    for a, b in zip(Fb, dF0):
        np.testing.assert_allclose(a.double().cpu().numpy(), 0.37 * b, rtol=0, atol=tol * np.abs(b).max())


def test_core_vjp_fused_path_accumulates():
    """accumulate = 1 adds the fused path's factor gradients to the outputs."""
    from paper_2603_21379_amd import binding as B
    dims, cols = FP32_CASES[1]
    rng = np.random.default_rng(6)
    X = torch.from_numpy(rng.standard_normal(dims).astype(np.float32)).cuda()
    F = [torch.from_numpy(rng.standard_normal((n, c)).astype(np.float32)).cuda()
         for n, c in zip(dims, cols)]
    Gb = torch.from_numpy(rng.standard_normal(cols).astype(np.float32)).cuda()
    ref = [torch.empty_like(f) for f in F]
    B.tucker_core_vjp(X, F, Gb, Fbar=ref)
    acc = [torch.full_like(f, 0.5) for f in F]
    B.tucker_core_vjp(X, F, Gb, Fbar=acc, accumulate=True)
    torch.cuda.synchronize()
    for a, r in zip(acc, ref):
        torch.testing.assert_close(a, r + 0.5, rtol=1e-6, atol=1e-6 * float(r.abs().max()))


def test_gpu_directional_derivative_fd_4pow8():
    """Central differences of the GPU loss itself (FP64) along random directions."""
    from paper_2603_21379_amd import autograd as AG
    rng = np.random.default_rng(3)
    dims, cols = (4,) * 8, (3,) * 8
    X = rng.standard_normal(dims)
    Fs = [np.linalg.qr(rng.standard_normal((n, c)))[0] for n, c in zip(dims, cols)]
    _, dX, dF = _grads_gpu(X, Fs, torch.float64)

    def loss(Xn, Fn):
        with torch.no_grad():
            return float(AG.projection_loss(torch.tensor(Xn, device="cuda"),
                                            [torch.tensor(f, device="cuda") for f in Fn]))
    h = 1e-4
    for _ in range(4):
        VX = rng.standard_normal(dims)
        VF = [rng.standard_normal(f.shape) for f in Fs]

        def cd(step):
            return (loss(X + step * VX, [f + step * v for f, v in zip(Fs, VF)])
                    - loss(X - step * VX, [f - step * v for f, v in zip(Fs, VF)])) / (2 * step)
        fd = (4 * cd(h / 2) - cd(h)) / 3
        an = float(np.sum(dX * VX) + sum(np.sum(a * v) for a, v in zip(dF, VF)))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


def test_core_vjp_accumulate_and_partial_outputs():
    from paper_2603_21379_amd import binding as B
    rng = np.random.default_rng(4)
    dims, cols = (7, 8, 9), (3, 2, 4)
    X = torch.tensor(rng.standard_normal(dims), device="cuda")
    F = [torch.tensor(rng.standard_normal((n, c)), device="cuda") for n, c in zip(dims, cols)]
    Gb = torch.tensor(rng.standard_normal(cols), device="cuda")
    Xbar = torch.ones(dims, dtype=torch.float64, device="cuda")
    Fbar = [None, torch.zeros(8, 2, dtype=torch.float64, device="cuda"), None]
    B.tucker_core_vjp(X, F, Gb, Xbar=Xbar, Fbar=Fbar, accumulate=True)
    Xn = X.cpu().numpy()
    Fn = [f.cpu().numpy() for f in F]
    Xb0, Fb0 = oracle.core_vjp(Xn, Fn, Gb.cpu().numpy())
    np.testing.assert_allclose(Xbar.cpu().numpy(), 1.0 + Xb0, atol=1e-12)
    np.testing.assert_allclose(Fbar[1].cpu().numpy(), Fb0[1], atol=1e-11 * np.abs(Fb0[1]).max())


def test_core_vjp_rejects_rank_above_192():
    from paper_2603_21379_amd import binding as B
    dims, cols = (200, 6, 5), (193, 3, 2)
    X = torch.zeros(dims, dtype=torch.float64, device="cuda")
    F = [torch.zeros(n, c, dtype=torch.float64, device="cuda") for n, c in zip(dims, cols)]
    Gb = torch.zeros(cols, dtype=torch.float64, device="cuda")
    with pytest.raises(B.TkError, match="exceeds 192"):
        B.tucker_core_vjp(X, F, Gb, Xbar=torch.empty_like(X))

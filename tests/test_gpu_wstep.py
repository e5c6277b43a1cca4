"""GPU parity of the W step's eigensolver on Gram matrices chosen exactly:
with Z = [I; 0] the orthonormal basis is Q = Z, and Y = [M; 0] makes the
Gram of Q^T Y equal to M M^T.  The cases exercise the rule that leaves
pairs of indices ranked below the r largest diagonal entries unrotated: a
dropped block that hides an eigenvalue larger than a kept diagonal entry
(the Gershgorin check must send the solver back to full sweeps), a clustered
tail, and the plain well-separated case."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


def _sqrtm(G):
    w, V = np.linalg.eigh(G)
    return (V * np.sqrt(np.maximum(w, 0.0))) @ V.T


def _gpu_u(M, m, r):
    from paper_2603_21379_amd import binding as B
    ell, s = M.shape
    Zh = np.zeros((m, ell))
    Zh[:ell, :ell] = np.eye(ell)
    Yh = np.zeros((m, s))
    Yh[:ell] = M
    Z = torch.from_numpy(Zh).cuda()
    Y = torch.from_numpy(Yh).cuda()
    U = torch.empty(m, r, dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    B.tucker_qr([Z], Y=[Y], r=[r], U=[U], info=info)
    torch.cuda.synchronize()
    return U.cpu().numpy(), Zh, Yh


def _cases():
    rng = np.random.default_rng(21)
    # kept diagonal entries are exact eigenvalues; the block of the two smallest
    # diagonal entries hides the eigenvalue 1.9 > 1.5
    A = np.diag([3.0, 2.8, 2.6, 2.4, 2.2, 1.5, 1.0, 1.0])
    A[6, 7] = A[7, 6] = 0.9
    P = np.eye(8)[rng.permutation(8)]
    yield "hidden", P @ A @ P.T, 6, 16
    Qr, _ = np.linalg.qr(rng.standard_normal((20, 20)))
    ev = np.r_[np.geomspace(1e3, 1.0, 14), 1e-6 * (1 + 1e-3 * rng.standard_normal(6))]
    yield "clustered-tail", Qr @ np.diag(ev) @ Qr.T, 14, 40
    Qr, _ = np.linalg.qr(rng.standard_normal((42, 42)))
    ev = np.r_[0.8 ** np.arange(32), 1e-8 * (1 + 0.1 * rng.random(10))]
    yield "decay-42", Qr @ np.diag(ev) @ Qr.T, 32, 256


@pytest.mark.parametrize("case", range(3))
def test_wstep_eigensolver_matches_oracle(case):
    name, G, r, m = list(_cases())[case]
    M = _sqrtm(G)
    U, Zh, Yh = _gpu_u(M, m, r)
    _, U_or, sv = oracle.w_step(oracle.orth(Zh), Yh, r)
    assert oracle.projector_distance(U, U_or) < 1e-10, name
    # the kept eigenvalues are well separated: the columns agree one by one
    np.testing.assert_allclose(U, U_or, atol=1e-9, err_msg=name)

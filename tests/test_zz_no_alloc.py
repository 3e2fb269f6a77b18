"""The allocation-free subspace step (sgo_subspace_solve_noalloc) against the
allocating one (sgo_subspace_solve) on the same matrices: two calls in a
row, the second smaller (the shared workspace keeps the first call's
contents), the stream-ordered status, the Cholesky-only mode, and the
rejection of sizes beyond the workspace."""
import numpy as np
import pytest

import paper_1603_02732_amd as sgo

pytestmark = pytest.mark.gpu


def _problem(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n, n))
    S = A @ A.T / n + np.eye(n)
    H = rng.normal(size=(n, n))
    return S, 0.5 * (H + H.T)


def _noalloc(S, H, mode, with_status):
    import torch
    dev = torch.device("cuda:0")
    n = S.shape[0]
    tS = torch.from_numpy(S).to(dev)
    tH = torch.from_numpy(H).to(dev)
    tM = torch.full((n, n), float("nan"), dtype=torch.float64, device=dev)
    te = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
    tst = torch.full((1,), 7, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    print("noalloc n=%d mode=%d status=%s" % (n, mode, with_status), flush=True)
    sgo.subspace_solve_noalloc(tS.data_ptr(), tH.data_ptr() if mode == 3 else None,
                               tM.data_ptr(), te.data_ptr(), n, mode,
                               status=tst.data_ptr() if with_status else None,
                               stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    # the inputs are left as they were
    assert np.array_equal(tS.cpu().numpy(), S) and np.array_equal(tH.cpu().numpy(), H)
    return tM.cpu().numpy(), te.cpu().numpy(), int(tst.item())


def _check(S, H, mode, with_status):
    n = S.shape[0]
    M, eps, st = _noalloc(S, H, mode, with_status)
    Mr, er, _, _ = sgo.subspace_solve(S, H if mode == 3 else None, mode=mode)
    if with_status:
        assert st == 0
    # both give S-orthonormal bands (M^T S M = I)
    assert np.abs(M.T @ S @ M - np.eye(n)).max() < 1e-10
    if mode == 1:
        # M = L^-T is unique: elementwise
        assert np.abs(M - Mr).max() < 1e-10 * np.abs(Mr).max()
        return
    # eigenvalues elementwise; eigenvectors up to the sign of each column
    # (the allocating form runs the Jacobi rounds over the GPU from 160 bands)
    assert np.abs(eps - er).max() < 1e-10 * np.abs(er).max()
    sign = np.sign((M * Mr).sum(0))
    assert np.abs(M - Mr * sign[None, :]).max() < 1e-8 * np.abs(Mr).max()
    assert np.abs(M.T @ H @ M - np.diag(eps)).max() < 1e-10 * np.abs(er).max()


def test_noalloc_matches_the_allocating_step_twice_smaller_second():
    S, H = _problem(200, 1)
    _check(S, H, 3, True)
    S, H = _problem(48, 2)
    _check(S, H, 3, False)


def test_noalloc_two_buffer_lds_form():
    # 65..88 bands: H' in two LDS buffers, the other matrices in the workspace
    S, H = _problem(80, 3)
    _check(S, H, 3, True)
    S, H = _problem(71, 4)
    _check(S, H, 3, False)


def test_noalloc_cholesky_mode_and_status():
    S, H = _problem(100, 3)
    _check(S, H, 1, True)
    # an indefinite overlap: the status says so in stream order, and without a
    # status pointer the call raises
    S, H = _problem(40, 4)
    S[5, 5] = -1.0
    M, eps, st = _noalloc(S, H, 3, True)
    assert st == sgo.SGO_ENUMERIC
    with pytest.raises(sgo.SgoError):
        _noalloc(S, H, 3, False)


def test_noalloc_rejects_sizes_beyond_its_workspace():
    import torch
    t = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    with pytest.raises(sgo.SgoError) as e:
        sgo.subspace_solve_noalloc(t.data_ptr(), t.data_ptr(), t.data_ptr(), t.data_ptr(), 257, 3)
    assert e.value.code == sgo.SGO_EINVAL

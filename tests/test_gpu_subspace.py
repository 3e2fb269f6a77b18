"""The FP64 subspace step against plain linear algebra: Cholesky-QR equals
classical Gram-Schmidt in band order (the orthogonalisation step of
Algorithm 1), and
the Rayleigh-Ritz rotation solves the generalised eigenproblem H c = e S c."""
import numpy as np
import pytest
import scipy.linalg

from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def gram_schmidt_rows(X):
    Q = np.zeros_like(X)
    for i in range(X.shape[0]):
        v = X[i].copy()
        for j in range(i):
            v -= (Q[j] @ X[i]) * Q[j]
        Q[i] = v / np.linalg.norm(v)
    return Q


@pytest.mark.parametrize("n", [1, 5, 20, 56, 64, 65, 96])
def test_cholesky_qr_is_gram_schmidt(n):
    import paper_1603_02732_amd as sgo
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, 3 * n + 7))
    S = X @ X.T
    M, _, _, _ = sgo.subspace_solve(S, mode=1)
    Q = M.T @ X
    err = np.abs(Q - gram_schmidt_rows(X)).max()
    say("n=%d cholesky-QR vs Gram-Schmidt %.2e" % (n, err))
    assert err < 1e-9


# 1..64: all matrices in LDS; 65..88: two H' buffers in LDS; 89..128: one;
# from 160: the Jacobi rounds over the GPU
@pytest.mark.parametrize("n", [2, 7, 20, 32, 33, 56, 64, 65, 77, 88, 89, 96, 128, 282])
def test_rayleigh_ritz_solves_generalised_problem(n):
    import paper_1603_02732_amd as sgo
    rng = np.random.default_rng(100 + n)
    A = rng.standard_normal((n, n))
    H = (A + A.T) / 2
    E = rng.standard_normal((n, n)) * 0.05 / np.sqrt(n)
    S = np.eye(n) + (E + E.T) / 2
    S = S @ S.T  # safely positive definite
    M, eps, ms, clk = sgo.subspace_solve(S, H, mode=3, clocks=True)
    ref = scipy.linalg.eigh(H, S, eigvals_only=True)
    say("n=%d eig err %.2e  %.3f ms  sweeps %d" % (n, np.abs(eps - ref).max(), ms, clk[5]))
    assert np.abs(eps - ref).max() < 1e-11 * max(1, np.abs(ref).max())
    assert np.abs(M.T @ S @ M - np.eye(n)).max() < 1e-10
    assert np.abs(M.T @ H @ M - np.diag(eps)).max() < 1e-10 * max(1, np.abs(ref).max())
    assert np.all(np.diff(eps) >= 0)


@pytest.mark.parametrize("n", [24, 72])
def test_degenerate_spectrum(n):
    import paper_1603_02732_amd as sgo
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.repeat([-0.5, -0.1, 0.2, 0.3], n // 4)
    H = Q @ np.diag(lam) @ Q.T
    M, eps, _, _ = sgo.subspace_solve(np.eye(n), H, mode=3)
    assert np.abs(eps - lam).max() < 1e-12
    assert np.abs(M.T @ M - np.eye(n)).max() < 1e-12


def test_not_positive_definite_is_an_error():
    import paper_1603_02732_amd as sgo
    S = np.eye(4)
    S[2, 2] = -1.0
    with pytest.raises(sgo.SgoError):
        sgo.subspace_solve(S, np.eye(4), mode=3)


@pytest.mark.parametrize("threads", [64, 128, 256])
@pytest.mark.parametrize("n", [32, 80])
def test_rayleigh_ritz_at_other_workgroup_sizes(threads, n, monkeypatch):
    # the thread count is a tuning key: the Jacobi rounds, the norms and the
    # passes over the items depend on it, the results must not
    import paper_1603_02732_amd as sgo
    monkeypatch.setenv("SGO_SUB_THREADS", str(threads))
    rng = np.random.default_rng(300 + n)
    A = rng.standard_normal((n, n))
    H = (A + A.T) / 2
    E = rng.standard_normal((n, n)) * 0.05 / np.sqrt(n)
    S = np.eye(n) + (E + E.T) / 2
    S = S @ S.T
    M, eps, _, _ = sgo.subspace_solve(S, H, mode=3)
    ref = scipy.linalg.eigh(H, S, eigvals_only=True)
    say("n=%d threads=%d eig err %.2e" % (n, threads, np.abs(eps - ref).max()))
    assert np.abs(eps - ref).max() < 1e-11 * max(1, np.abs(ref).max())
    assert np.abs(M.T @ S @ M - np.eye(n)).max() < 1e-10
    assert np.abs(M.T @ H @ M - np.diag(eps)).max() < 1e-10 * max(1, np.abs(ref).max())

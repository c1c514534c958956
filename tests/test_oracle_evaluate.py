"""Pins of the evaluator (Sec. 4 measures) against direct dense computation."""

import numpy as np
import pytest

from oracle import evaluate
from workloads import small_random_csr

pytestmark = pytest.mark.cpu


def test_cov_err_lanczos_matches_dense():
    st = small_random_csr(400, 120, 6, 1)
    A = st.to_scipy()
    B = np.random.default_rng(0).standard_normal((5, 120)) * 0.5
    dense = evaluate.cov_extremes(A, B, dense_limit=10_000)
    lanczos = evaluate.cov_extremes(A, B, dense_limit=10)
    np.testing.assert_allclose(dense, lanczos, rtol=1e-7)
    M = (A.T @ A).toarray() - B.T @ B
    assert np.isclose(evaluate.cov_err(A, B), np.linalg.norm(M, 2) / np.sum(A.toarray() ** 2))


def test_gram_distance_matches_direct():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((6, 50))
    Y = X + 1e-3 * rng.standard_normal((6, 50))
    direct = np.linalg.norm(X.T @ X - Y.T @ Y) / np.linalg.norm(Y.T @ Y)
    assert np.isclose(evaluate.gram_distance(X, Y), direct, rtol=1e-6)
    assert evaluate.gram_distance(X, X) < 1e-7


def test_tail_energy_and_proj_err():
    st = small_random_csr(300, 40, 6, 3)
    A = st.to_scipy()
    s = np.linalg.svd(A.toarray(), compute_uv=False)
    assert np.isclose(evaluate.tail_energy(A, 5), np.sum(s[5:] ** 2))
    # B = exact top-k right singular directions: proj-err = 1
    _, sv, Vt = np.linalg.svd(A.toarray(), full_matrices=False)
    B = sv[:5, None] * Vt[:5]
    assert np.isclose(evaluate.proj_err(A, B, 5), 1.0)
    with pytest.raises(ValueError):
        evaluate.sfd_bound(A, 20, 3)


def test_top_singular_values_iterative_branch_matches_closed_form():
    # min(n, d) > 2000 takes the iterative (ARPACK svds) branch: pinned against a matrix with
    # known singular values, A = U diag(s) V^T with U, V orthonormal (Householder QR of Gaussian
    # blocks), and against LAPACK's dense SVD of the same matrix
    import scipy.sparse as sp

    rng = np.random.default_rng(5)
    n, d, r = 2600, 2100, 40
    U, _ = np.linalg.qr(rng.standard_normal((n, r)))
    V, _ = np.linalg.qr(rng.standard_normal((d, r)))
    s = np.sort(rng.uniform(0.5, 20.0, r))[::-1]
    s[3] = s[2] * (1 - 1e-3)  # a close pair in the top 10
    A = sp.csr_matrix((U * s) @ V.T)
    k = 10
    got = evaluate.top_singular_values(A, k)
    np.testing.assert_allclose(got, s[:k], rtol=1e-9)
    dense = np.linalg.svd(A.toarray(), compute_uv=False)[:k]
    np.testing.assert_allclose(got, dense, rtol=1e-9)
    # and the tail energy it feeds: ||A - A_k||_F^2 = sum_{i > k} s_i^2
    np.testing.assert_allclose(evaluate.tail_energy(A, k), np.sum(s[k:] ** 2), rtol=1e-9)

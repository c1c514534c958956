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

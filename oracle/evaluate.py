"""Accuracy measures of the paper's experiments (Sec. 4, "Measurements"), FP64.

* cov-err  = ||A^T A - B^T B||_2 / ||A||_F^2
* proj-err = ||A - pi_{B_k}(A)||_F^2 / ||A - A_k||_F^2, pi_{B_k} the projection onto the top-k
  right singular vectors of B (Sec. 1.1 notation)
* the guarantees they are compared with: ||A - A_k||_F^2 / (ell - k) for FrequentDirections
  (Sec. 2) and ||A - A_k||_F^2 / (alpha ell - k), alpha = 6/41, for SFD (Theorem 3.1).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _as_sparse(A):
    return A if sp.issparse(A) else sp.csr_matrix(np.asarray(A, dtype=np.float64))


def fro2(A) -> float:
    """||A||_F^2 (duplicate stored entries of a sparse matrix are summed first)."""
    if sp.issparse(A):
        A = A.tocsr(copy=True)
        A.sum_duplicates()
        return float(np.sum(A.data.astype(np.float64) ** 2))
    return float(np.sum(np.asarray(A, dtype=np.float64) ** 2))


def cov_extremes(A, B, dense_limit: int = 5000) -> tuple[float, float]:
    """(lambda_min, lambda_max) of A^T A - B^T B.

    Dense eigh when d <= dense_limit, else Lanczos on x -> A^T(Ax) - B^T(Bx).
    """
    A = _as_sparse(A)
    B = np.asarray(B, dtype=np.float64)
    d = A.shape[1]
    if d <= dense_limit:
        M = (A.T @ A).toarray() - B.T @ B
        w = np.linalg.eigvalsh(M)
        return float(w[0]), float(w[-1])

    def mv(x):
        x = np.ravel(x)
        return A.T @ (A @ x) - B.T @ (B @ x)

    op = spla.LinearOperator((d, d), matvec=mv, dtype=np.float64)
    lmax = spla.eigsh(op, k=1, which="LA", tol=1e-10, return_eigenvectors=False)[0]
    lmin = spla.eigsh(op, k=1, which="SA", tol=1e-10, return_eigenvectors=False)[0]
    return float(lmin), float(lmax)


def cov_err(A, B, dense_limit: int = 5000) -> float:
    """cov-err = ||A^T A - B^T B||_2 / ||A||_F^2 (Sec. 4)."""
    lmin, lmax = cov_extremes(A, B, dense_limit)
    return max(abs(lmin), abs(lmax)) / fro2(A)


def top_singular_values(A, k: int) -> np.ndarray:
    """The k largest singular values of A (descending)."""
    A = _as_sparse(A)
    n, d = A.shape
    if min(n, d) <= 2000 or k >= min(n, d) - 1:
        s = np.linalg.svd(A.toarray(), compute_uv=False)
        return s[:k]
    s = spla.svds(A.astype(np.float64), k=k, return_singular_vectors=False, tol=1e-10)
    return np.sort(s)[::-1]


def tail_energy(A, k: int) -> float:
    """||A - A_k||_F^2 = ||A||_F^2 - sum_{i<=k} sigma_i^2."""
    if k == 0:
        return fro2(A)
    s = top_singular_values(A, k)
    return fro2(A) - float(np.sum(s ** 2))


def fd_bound(A, ell: int, k: int) -> float:
    """||A - A_k||_F^2 / (ell - k): FrequentDirections' covariance guarantee (Sec. 2, Lemma 2.1 with alpha = 1)."""
    return tail_energy(A, k) / (ell - k)


def sfd_bound(A, ell: int, k: int, alpha: float = 6.0 / 41.0) -> float:
    """||A - A_k||_F^2 / (alpha ell - k): Theorem 3.1's covariance guarantee (needs k < alpha ell)."""
    if not k < alpha * ell:
        raise ValueError("Theorem 3.1 needs k < alpha * ell")
    return tail_energy(A, k) / (alpha * ell - k)


def proj_err(A, B, k: int) -> float:
    """proj-err = ||A - A V_k V_k^T||_F^2 / ||A - A_k||_F^2 with V_k the top-k right singular vectors of B."""
    A = _as_sparse(A)
    B = np.asarray(B, dtype=np.float64)
    _, _, Vt = np.linalg.svd(B, full_matrices=False)
    Vk = Vt[:k].T
    AV = A @ Vk
    num = fro2(A) - float(np.sum(AV ** 2))
    return num / tail_energy(A, k)


def gram_distance(B1, B2) -> float:
    """||B1^T B1 - B2^T B2||_F / ||B2^T B2||_F without forming d x d matrices.

    ||X^T X - Y^T Y||_F^2 = ||X X^T||_F^2 + ||Y Y^T||_F^2 - 2 ||X Y^T||_F^2.
    """
    X = np.asarray(B1, dtype=np.float64)
    Y = np.asarray(B2, dtype=np.float64)
    xx = np.sum((X @ X.T) ** 2)
    yy = np.sum((Y @ Y.T) ** 2)
    xy = np.sum((X @ Y.T) ** 2)
    num = max(xx + yy - 2.0 * xy, 0.0)
    return float(np.sqrt(num) / np.sqrt(yy)) if yy > 0 else float(np.sqrt(num))

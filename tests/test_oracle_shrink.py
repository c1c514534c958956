"""Pins of the oracle's shrink operators (Alg 1, 3, 4, 5, 6) against closed forms, identities of
the paper's proofs, LAPACK routines and brute force."""

import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import shrink
from oracle.rng import sphere_vector, start_block
from oracle.shrink import (
    ALPHA,
    NoConvergence,
    boosted_sparse_shrink,
    dense_shrink,
    si_iterations,
    simultaneous_iteration,
    sparse_shrink,
    verify_spectral,
    vs_steps,
)
from workloads import small_random_csr

pytestmark = pytest.mark.cpu


def _rand_sparse(m, d, lam, seed, **kw):
    return small_random_csr(m, d, lam, seed, **kw).to_scipy()


def _psd_part(M):
    w, V = np.linalg.eigh((M + M.T) / 2)
    return (V * np.maximum(w, 0)) @ V.T


# ---------------------------------------------------------------------------- DenseShrink (Alg 5)
@pytest.mark.parametrize("n,d,ell,seed", [(12, 9, 4, 0), (40, 30, 10, 1), (8, 20, 3, 2), (6, 6, 6, 3)])
def test_dense_shrink_closed_form(n, d, ell, seed):
    """B^T B = (C^T C - mu_ell I)_+ with mu the eigenvalues of the d x d matrix C^T C (eigh route)."""
    C = np.random.default_rng(seed).standard_normal((n, d))
    B, live = dense_shrink(C, ell, n)
    mu = np.linalg.eigvalsh(C.T @ C)[::-1]
    want = _psd_part(C.T @ C - mu[ell - 1] * np.eye(d))
    if n <= ell:
        want = C.T @ C
    np.testing.assert_allclose(B.T @ B, want, atol=1e-10 * np.abs(C.T @ C).max())
    assert live == (n if n <= ell else ell - 1)


@pytest.mark.parametrize("seed", range(4))
def test_dense_shrink_error_identities(seed):
    """||C^T C - B^T B||_2 = mu_ell and ||C||_F^2 - ||B||_F^2 = ell mu_ell + sum_{i>ell} mu_i."""
    rng = np.random.default_rng(seed)
    n, d, ell = 30, 25, 8
    C = rng.standard_normal((n, d)) * rng.random(d)
    B, _ = dense_shrink(C, ell, n)
    mu = np.linalg.eigvalsh(C.T @ C)[::-1]
    gap = np.linalg.eigvalsh(C.T @ C - B.T @ B)
    assert gap[0] >= -1e-10 * mu[0]
    assert math.isclose(gap[-1], mu[ell - 1], rel_tol=1e-9)
    lost = np.sum(C ** 2) - np.sum(B ** 2)
    assert math.isclose(lost, ell * mu[ell - 1] + mu[ell:].sum(), rel_tol=1e-9)
    assert np.all(B[ell - 1] == 0.0)


def test_dense_shrink_rank_deficient_and_zero():
    C = np.zeros((6, 5))
    B, live = dense_shrink(C, 3, 6)
    assert np.all(B == 0) and live == 2
    C[0, 1] = 2.0
    B, live = dense_shrink(C, 3, 1)
    np.testing.assert_allclose(B.T @ B, C.T @ C)


# ---------------------------------------------------------------------------- SimultaneousIteration (Alg 1)
@pytest.mark.parametrize("q", [0, 1, 2, 3])
def test_si_span_equals_brute_force_power(q):
    """span(Z) = span(A (A^T A)^q G), the power formed directly with no orthonormalisation."""
    A = _rand_sparse(60, 25, 5, 11)
    G = start_block(1, 0, 0, 0, 0, 25, 6)
    Z = simultaneous_iteration(A, G, q)
    Ad = A.toarray()
    Y = Ad @ np.linalg.matrix_power(Ad.T @ Ad, q) @ G
    PiY = Y @ np.linalg.pinv(Y)
    np.testing.assert_allclose(Z @ Z.T, PiY, atol=1e-8)
    np.testing.assert_allclose(Z.T @ Z, np.eye(6), atol=1e-12)


def test_si_converges_to_top_subspace_with_gap():
    """With a spectral gap and many iterations SparseShrink equals DenseShrink of the buffer (LAPACK SVD)."""
    rng = np.random.default_rng(4)
    m, d, ell = 80, 40, 6
    U, _ = np.linalg.qr(rng.standard_normal((m, d)))
    V, _ = np.linalg.qr(rng.standard_normal((d, d)))
    s = np.concatenate([np.linspace(10, 5, ell), np.linspace(1.0, 0.1, d - ell)])
    A = sp.csr_matrix(U @ np.diag(s) @ V.T)
    res = sparse_shrink(A, start_block(0, 0, 0, 0, 0, d, ell), ell, q=40)
    Ad = A.toarray()
    sv = np.linalg.svd(Ad, compute_uv=False)
    want = _psd_part(Ad.T @ Ad - sv[ell - 1] ** 2 * np.eye(d))
    # the iterate's error decays like (s_{ell+1}/s_ell)^{2q}
    np.testing.assert_allclose(res["B"].T @ res["B"], want, atol=1e-9 * s[0] ** 2)


def test_si_iteration_count_reading():
    # q = ceil(ln(m/eps)/eps): 34 at m = 1000, 52 at m = 1e5, 61 at m = 1e6 (eps = 1/4)
    assert [si_iterations(m, 0.25) for m in (1000, 100_000, 1_000_000)] == [34, 52, 61]
    assert si_iterations(21, 0.5) == math.ceil(2 * math.log(42))


# ---------------------------------------------------------------------------- SparseShrink (Alg 3)
@pytest.mark.parametrize("q", [0, 1, 5])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sparse_shrink_property1_deterministic(q, seed):
    """Property 1 holds for every start block and every q: A'^T A' - B'^T B' is PSD (Sec. 3.2)."""
    A = _rand_sparse(50, 30, 6, seed)
    for attempt in range(3):
        res = sparse_shrink(A, start_block(seed, 0, 0, attempt, 0, 30, 7), 7, q)
        M = (A.T @ A).toarray() - res["B"].T @ res["B"]
        assert np.linalg.eigvalsh(M)[0] >= -1e-10 * np.abs(M).max()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sparse_shrink_proof_identities(seed):
    """P^T P - B'^T B' = lambda_ell^2 V V^T and ||A'||^2 - ||B'||^2 = ||A' - Z Z^T A'||^2 + ell lambda_ell^2 (Sec. 3.2)."""
    A = _rand_sparse(70, 40, 8, seed)
    ell = 9
    res = sparse_shrink(A, start_block(seed, 0, 0, 0, 0, 40, ell), ell, q=3)
    B, P, Z, lam = res["B"], res["P"], res["Z"], res["lam"]
    # V from an independent eigendecomposition of P^T P
    w, V = np.linalg.eigh(P.T @ P)
    Vl = V[:, ::-1][:, :ell]
    np.testing.assert_allclose(P.T @ P - B.T @ B, lam[ell - 1] ** 2 * Vl @ Vl.T, atol=1e-10)
    Ad = A.toarray()
    lhs = np.sum(Ad ** 2) - np.sum(B ** 2)
    rhs = np.sum((Ad - Z @ (Z.T @ Ad)) ** 2) + ell * lam[ell - 1] ** 2
    assert math.isclose(lhs, rhs, rel_tol=1e-10)
    assert np.all(B[ell - 1] == 0.0)


def test_sparse_shrink_rank_deficient_keeps_everything():
    """rank(A') < ell: the QR completes the basis, P^T P = A'^T A' and lambda_ell = 0, so B'^T B' = A'^T A'."""
    rng = np.random.default_rng(9)
    L = rng.standard_normal((40, 3)) @ rng.standard_normal((3, 20))
    A = sp.csr_matrix(L)
    res = sparse_shrink(A, start_block(2, 0, 0, 0, 0, 20, 6), 6, q=4)
    np.testing.assert_allclose(res["B"].T @ res["B"], L.T @ L, atol=1e-10 * np.abs(L.T @ L).max())


# ---------------------------------------------------------------------------- VerifySpectral (Alg 6)
def _diag_instance(a2, b2):
    """A' with A'^T A' = diag(a2) and B' with B'^T B' = diag(b2) (b2 <= a2 on its support)."""
    d = len(a2)
    A = sp.csr_matrix(np.diag(np.sqrt(a2)))
    B = np.diag(np.sqrt(b2))[: max(1, int(np.count_nonzero(b2)))]
    return A, B, d


@pytest.mark.parametrize("norm_c", [0.05, 0.5, 0.999, 1.0])
def test_verify_spectral_accepts_when_norm_at_most_one(norm_c):
    """Lemma 3.1: ||C|| <= 1 gives True for every start vector."""
    d = 50
    a2 = np.linspace(3.0, 1.0, d)
    b2 = np.zeros(d)
    b2[:5] = a2[:5] - 0.5
    A, B, _ = _diag_instance(a2, b2)
    M = np.diag(a2 - b2)
    half = np.abs(np.linalg.eigvalsh(M)).max() / norm_c
    for k in range(20):
        x = sphere_vector(k, 0, 0, 0, 1, d)
        ok, ln = verify_spectral(A, B, half, x, vs_steps(d, 0.01, 1 + k))
        assert ok and ln <= 1e-9


@pytest.mark.parametrize("norm_c", [2.0, 3.0])
def test_verify_spectral_rejects_when_norm_at_least_two(norm_c):
    """Lemma 3.1: ||C|| >= 2 gives False with probability >= 1 - delta_i; with a spread spectrum
    and a random x that is every draw here."""
    d = 64
    rng = np.random.default_rng(0)
    a2 = rng.uniform(0.1, 1.0, d)
    a2[17] = 1.0 * 4
    A, B, _ = _diag_instance(a2, np.zeros(d))
    half = 4.0 / norm_c
    rejected = 0
    for k in range(50):
        ok, ln = verify_spectral(A, B, half, sphere_vector(k, 0, 0, 0, 1, d), vs_steps(d, 0.01, 1))
        rejected += (not ok)
        if not ok:
            assert ln > 0
    assert rejected == 50


def test_verify_spectral_log_norm_matches_direct_power():
    """ln||C^t x|| from the normalised steps equals the log of the norm of C^t x formed directly."""
    A = _rand_sparse(30, 12, 4, 5)
    B = np.random.default_rng(1).standard_normal((3, 12)) * 0.1
    C = ((A.T @ A).toarray() - B.T @ B) / 0.7
    x = sphere_vector(1, 0, 0, 0, 1, 12)
    ok, ln = verify_spectral(A, B, 0.7, x, 9)
    assert math.isclose(ln, math.log(np.linalg.norm(np.linalg.matrix_power(C, 9) @ x)), rel_tol=1e-10)
    assert ok == (ln <= 0)


def test_vs_steps_reading():
    # t = ceil(log2(d/delta_i)), delta_i = delta / (2 i^2)
    assert vs_steps(1000, 0.01, 1) == math.ceil(math.log2(1000 * 200))
    assert vs_steps(1000, 0.01, 3) == math.ceil(math.log2(1000 * 2 * 9 / 0.01))
    # the union bound of Sec. 3.1: sum_i delta_i <= delta
    assert sum(shrink.vs_delta(0.01, i) for i in range(1, 100000)) <= 0.01


# ---------------------------------------------------------------------------- BoostedSparseShrink (Alg 4)
def _spiked_buffer(seed=0, m=60, d=30):
    """A' whose top right singular direction e_0 is its own block: a start block with zero row 0
    never sees it (SparseShrink fails), a Gaussian one does."""
    rng = np.random.default_rng(seed)
    A = np.zeros((m, d))
    A[: m // 2, 1:] = rng.standard_normal((m // 2, d - 1)) * 0.3
    A[m // 2:, 0] = 3.0
    return sp.csr_matrix(A)


def test_boosted_rejects_a_failed_shrink_and_retries():
    A = _spiked_buffer()
    d, ell = 30, 8

    def draw_G(attempt):
        G = start_block(0, 0, 0, attempt, 0, d, ell)
        if attempt == 0:
            G[0, :] = 0.0  # orthogonal to the dominant direction
        return G

    ctr = [0]

    def next_i():
        ctr[0] += 1
        return ctr[0]

    log = []
    Bp = boosted_sparse_shrink(A, ell, draw_G, lambda a: sphere_vector(0, 0, 0, a, 1, d), next_i,
                               q=2, delta=0.01, log=log)
    assert [r["accepted"] for r in log] == [False, True]
    assert [r["vs_index"] for r in log] == [1, 2]
    # the accepted sketch satisfies Property 2 with Delta = (||A'||^2 - ||B'||^2)/(alpha ell)
    M = (A.T @ A).toarray() - Bp.T @ Bp
    Delta = (np.sum(A.toarray() ** 2) - np.sum(Bp ** 2)) / (ALPHA * ell)
    assert np.linalg.eigvalsh(M)[-1] <= Delta


def test_boosted_gives_up_after_max_attempts():
    A = _spiked_buffer(1)

    def bad_G(attempt):
        G = start_block(0, 0, 0, attempt, 0, 30, 8)
        G[0, :] = 0.0
        return G

    with pytest.raises(NoConvergence):
        boosted_sparse_shrink(A, 8, bad_G, lambda a: sphere_vector(0, 0, 0, a, 1, 30), lambda: 1,
                              q=2, delta=0.01, max_attempts=3)


def test_boosted_lossless_accept_without_verify_call():
    rng = np.random.default_rng(9)
    L = rng.standard_normal((40, 3)) @ rng.standard_normal((3, 20))
    calls = []
    log = []
    boosted_sparse_shrink(sp.csr_matrix(L), 6, lambda a: start_block(0, 0, 0, a, 0, 20, 6),
                          lambda a: sphere_vector(0, 0, 0, a, 1, 20), lambda: calls.append(1) or 1,
                          q=3, delta=0.01, log=log)
    assert calls == [] and log[0]["reason"] == "lossless"


def test_boosted_unverified_variant_skips_vs():
    A = _spiked_buffer()
    calls = []
    bad = lambda a: np.where(np.arange(30)[:, None] == 0, 0.0, start_block(0, 0, 0, a, 0, 30, 8))
    log = []
    boosted_sparse_shrink(A, 8, bad, lambda a: sphere_vector(0, 0, 0, a, 1, 30), lambda: calls.append(1) or 1,
                          q=2, delta=0.01, verify=False, log=log)
    assert calls == [] and log[0]["reason"] == "unverified"

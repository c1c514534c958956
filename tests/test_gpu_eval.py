"""The accuracy measures of Sec. 4 on the GPU (sfd_evaluate) against the FP64 oracle's evaluator.

cov-err comes from Lanczos with full reorthogonalisation on x -> A^T(Ax) - B^T(Bx); with as many
steps as d the Krylov space is the whole space, so the Ritz values are the eigenvalues (checked
against dense eigh); with fewer steps the extremes are checked against ARPACK (eigsh/svds) at
d = 20,000.  proj-err uses the top-k right singular vectors of B and the top-k singular values
of A.
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import evaluate
from workloads import small_random_csr

pytestmark = pytest.mark.gpu


def _dev(st):
    import torch

    return (torch.from_numpy(np.ascontiguousarray(st.indptr)).cuda(),
            torch.from_numpy(np.ascontiguousarray(st.indices)).cuda(),
            torch.from_numpy(np.ascontiguousarray(st.values)).cuda())


def _csr(st):
    return sp.csr_matrix((st.values.astype(np.float64), st.indices, st.indptr - st.indptr[0]), shape=(st.n, st.d))


def _sketch(gpu_lib, st, ell):
    sk = gpu_lib.Sketch(st.d, ell, 0.25, 0)
    sk.append_csr(*_dev(st))
    return sk.sketch()


@pytest.mark.parametrize("n,d,ell,k", [(400, 300, 20, 5), (900, 250, 40, 10), (150, 200, 50, 3)])
def test_small_cases_match_dense_oracle(gpu_lib, n, d, ell, k):
    # steps = d: the Lanczos basis spans R^d, so the extremes and the top-k are exact up to rounding
    st = small_random_csr(n, d, 9, n + d, dist="lognormal", dup_rate=0.05)
    B = _sketch(gpu_lib, st, ell)
    r = gpu_lib.evaluate(*_dev(st), d, B, k=k, steps=d)
    A, Bh = _csr(st), B.cpu().numpy().astype(np.float64)
    lmin, lmax = evaluate.cov_extremes(A, Bh)
    assert r["fro2A"] == pytest.approx(evaluate.fro2(A), rel=1e-12)
    assert r["cov_max"] == pytest.approx(lmax, rel=1e-9)
    assert abs(r["cov_min"] - lmin) <= 1e-9 * lmax
    assert r["cov_err"] == pytest.approx(evaluate.cov_err(A, Bh), rel=1e-9)
    top = evaluate.top_singular_values(A, k)
    assert r["top_k_energy"] == pytest.approx(float(np.sum(top ** 2)), rel=1e-9)
    assert r["proj_err"] == pytest.approx(evaluate.proj_err(A, Bh, k), rel=1e-7)
    # the FD property of the sketch (B^T B <= A^T A) shows as cov_min >= 0 up to FP32 rounding
    assert r["cov_min"] >= -1e-5 * r["fro2A"]
    # the Krylov space is the whole space: the Ritz residuals vanish
    assert r["cov_max_res"] <= 1e-6 * lmax and r["cov_min_res"] <= 1e-6 * lmax
    assert r["top_k_res"] <= 1e-6 * r["top_k_energy"]


@pytest.mark.parametrize("steps", [12, 30])
def test_ritz_residuals_bound_the_distance_to_the_spectrum(gpu_lib, steps):
    # fewer steps than d: each reported Ritz value lies within its residual of an eigenvalue of
    # A^T A - B^T B (resp. A^T A), checked against the dense spectrum
    st = small_random_csr(600, 300, 9, 17, dist="lognormal")
    B = _sketch(gpu_lib, st, 20)
    r = gpu_lib.evaluate(*_dev(st), st.d, B, k=4, steps=steps)
    A, Bh = _csr(st), B.cpu().numpy().astype(np.float64)
    G = (A.T @ A).toarray()
    lam = np.linalg.eigvalsh(G - Bh.T @ Bh)
    scale = np.abs(lam).max()
    for th, res in ((r["cov_max"], r["cov_max_res"]), (r["cov_min"], r["cov_min_res"])):
        assert np.min(np.abs(lam - th)) <= res * (1 + 1e-6) + 1e-10 * scale, (th, res)
        assert 0.0 < res < scale  # a finite, informative certificate after a partial run
    top = np.sort(np.linalg.eigvalsh(G))[::-1][:4]
    # Ritz values interlace: the top-k Ritz sum is at most the true top-k energy
    assert r["top_k_energy"] <= np.sum(top) * (1 + 1e-12)
    assert r["top_k_res"] > 0.0


def test_large_case_matches_arpack(gpu_lib):
    # 24,000 x 20,000 with Zipf-long columns; 160 Lanczos steps against ARPACK (tol 1e-10).  The
    # sketch's residual A^T A - B^T B is positive semidefinite (FD property), so cov-err is its
    # largest eigenvalue over ||A||_F^2 (ARPACK's smallest-eigenvalue run is not needed)
    import scipy.sparse.linalg as spla

    st = small_random_csr(24000, 20000, 30, 5, dist="lognormal")
    B = _sketch(gpu_lib, st, 40)
    r = gpu_lib.evaluate(*_dev(st), st.d, B, k=10, steps=160)
    A, Bh = _csr(st), B.cpu().numpy().astype(np.float64)
    op = spla.LinearOperator((st.d, st.d), matvec=lambda x: A.T @ (A @ np.ravel(x)) - Bh.T @ (Bh @ np.ravel(x)),
                             dtype=np.float64)
    lmax = spla.eigsh(op, k=1, which="LA", tol=1e-10, return_eigenvectors=False)[0]
    assert r["cov_min"] >= -1e-5 * r["fro2A"]
    assert r["cov_max"] == pytest.approx(lmax, rel=1e-5)
    assert r["cov_err"] == pytest.approx(lmax / evaluate.fro2(A), rel=1e-5)
    # the residual certifies the extreme: ARPACK's value lies within it
    assert abs(r["cov_max"] - lmax) <= r["cov_max_res"] + 1e-9 * lmax
    assert r["cov_max_res"] <= 1e-3 * lmax
    assert r["proj_err"] == pytest.approx(evaluate.proj_err(A, Bh, 10), rel=1e-6)
    assert r["steps"] == 160


def test_without_sketch_and_without_rank(gpu_lib):
    # B absent: cov_max = sigma_1(A)^2; k = 0: the proj-err fields are NaN
    st = small_random_csr(500, 120, 7, 9, dist="normal")
    r = gpu_lib.evaluate(*_dev(st), st.d, None, k=0, steps=120)
    A = _csr(st)
    s1 = evaluate.top_singular_values(A, 1)[0]
    assert r["cov_max"] == pytest.approx(s1 ** 2, rel=1e-9)
    assert r["cov_err"] == pytest.approx(s1 ** 2 / evaluate.fro2(A), rel=1e-9)
    assert math.isnan(r["proj_err"]) and math.isnan(r["top_k_energy"])


def test_empty_matrix_and_errors(gpu_lib):
    import torch

    d = 64
    B = torch.randn(4, d, device="cuda")
    ptr = torch.zeros(1, dtype=torch.int64, device="cuda")
    idx = torch.zeros(0, dtype=torch.int32, device="cuda")
    val = torch.zeros(0, dtype=torch.float32, device="cuda")
    r = gpu_lib.evaluate(ptr, idx, val, d, B, k=2, steps=d)
    lam = np.linalg.eigvalsh(B.cpu().double().numpy() @ B.cpu().double().numpy().T)
    assert r["fro2A"] == 0.0
    assert r["cov_max"] == pytest.approx(0.0, abs=1e-9 * lam[-1])
    assert r["cov_min"] == pytest.approx(-lam[-1], rel=1e-9)
    assert math.isinf(r["cov_err"])
    # a column id outside [0, d), too many steps, k > ell
    st = small_random_csr(50, 40, 5, 1)
    p, i, v = _dev(st)
    bad = i.clone()
    bad[3] = 40
    with pytest.raises(gpu_lib.SfdError) as e:
        gpu_lib.evaluate(p, bad, v, 40, None)
    assert e.value.code == gpu_lib.SFD_E_INDEX
    with pytest.raises(gpu_lib.SfdError):
        gpu_lib.evaluate(p, i, v, 40, torch.zeros(3, 40, device="cuda"), k=4)
    with pytest.raises(gpu_lib.SfdError):
        gpu_lib.evaluate(p, i, v, 40, None, steps=513)


def test_evaluation_is_reproducible(gpu_lib):
    st = small_random_csr(3000, 1500, 12, 4, dist="lognormal")
    B = _sketch(gpu_lib, st, 30)
    r1 = gpu_lib.evaluate(*_dev(st), st.d, B, k=5, steps=80, seed=3)
    r2 = gpu_lib.evaluate(*_dev(st), st.d, B, k=5, steps=80, seed=3)
    assert r1 == r2

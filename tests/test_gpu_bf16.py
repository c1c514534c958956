"""The BF16 precision form: the SimultaneousIteration products 1 .. 2q+1 read BF16 values and BF16
panels, the panel transforms and Grams of CholeskyQR run on BF16 MFMA (FP32 accumulation), the
Cholesky stays FP64, and CholeskyQR2 re-orthonormalises the final basis (or every panel).

It is not element-wise comparable with the FP64 oracle: BF16 storage changes the subspace the
iteration finds.  What must hold (the design keeps P P^T a compression of A'^T A' onto the
stored basis, so Property 1 of Sec. 3 is kept for the FP32 values):
* B^T B <= A^T A up to FP32 rounding (lambda_min(A^T A - B^T B) >= -tol ||A||_F^2);
* cov-err (Sec. 4) within 5% of the FP32 form's on the same input, same q and same random
  blocks (the fixed-cov-err rule the two forms are compared under), and within 5% of the FP64
  oracle's sketch's;
* exact buffers (n <= ell) are untouched by the panel precision;
* results are deterministic (the same bits on a second run).
"""

import numpy as np
import pytest

from oracle import SFDOracle, evaluate
from workloads import stream_1e4_d1e3, small_random_csr

pytestmark = pytest.mark.gpu


def _sketch(sfd, st, ell, **opts):
    import torch

    sk = sfd.Sketch(st.d, ell, 0.25, 0, **opts)
    sk.append_csr(torch.from_numpy(st.indptr).cuda(), torch.from_numpy(st.indices).cuda(),
                  torch.from_numpy(st.values).cuda())
    return sk, sk.sketch().cpu().numpy().astype(np.float64)


def _check_form(sfd, st, ell, cqr2=None, oracle=False):
    A = st.to_scipy()
    _, B32 = _sketch(sfd, st, ell)
    sk, B16 = _sketch(sfd, st, ell, precision="bf16", cqr2=cqr2)
    lmin, _ = evaluate.cov_extremes(A, B16)
    f2 = evaluate.fro2(A)
    assert lmin >= -1e-5 * f2
    e32, e16 = evaluate.cov_err(A, B32), evaluate.cov_err(A, B16)
    assert e16 <= 1.05 * e32, (e16, e32)
    if oracle:
        o = SFDOracle(st.d, ell, 0.25, 0, unit_roundoff=2.0 ** -24)
        o.append_csr(st.indptr, st.indices, st.values)
        e64 = evaluate.cov_err(A, o.sketch())
        assert e16 <= 1.05 * e64, (e16, e64)
    return sk, e16, e32


@pytest.mark.parametrize("n,d,ell,lam,seed", [
    (900, 80, 20, 9, 1),      # L = 32
    (1500, 90, 50, 20, 3),    # L = 64
    (3000, 1200, 40, 15, 4),  # long CSC columns, several flushes
    (2500, 400, 100, 25, 6),  # L = 128
    (2400, 700, 200, 40, 10),  # L = 256
])
def test_bf16_form_keeps_property1_and_cov_err(gpu_lib, n, d, ell, lam, seed):
    st = small_random_csr(n, d, lam, seed, dist="lognormal")
    _check_form(gpu_lib, st, ell, oracle=True)


@pytest.mark.parametrize("cqr2", ["off", "final", "all"])
@pytest.mark.parametrize("n,d,ell,lam,seed", [(1500, 90, 50, 20, 3), (2400, 700, 200, 40, 10)])
def test_bf16_form_cqr2_modes(gpu_lib, cqr2, n, d, ell, lam, seed):
    # CholeskyQR2 off, on the final basis (the default) and on every panel: each keeps Property 1
    # and the cov-err bar
    st = small_random_csr(n, d, lam, seed, dist="lognormal")
    _check_form(gpu_lib, st, ell, cqr2=cqr2)


@pytest.mark.parametrize("n,d,ell,lam,seed", [(1500, 2000, 50, 20, 12), (2500, 3000, 100, 25, 13)])
def test_bf16_form_with_empty_rows_and_columns(gpu_lib, n, d, ell, lam, seed):
    # a third of the rows empty and many columns never entered (L = 64 and 128): the BF16
    # products' empty chunks write zero rows, and the form keeps Property 1 and the cov-err bar
    st = small_random_csr(n, d, lam, seed, empty_rate=0.3, dist="lognormal")
    assert (np.diff(st.indptr) == 0).any() and len(np.unique(st.indices)) < d
    _check_form(gpu_lib, st, ell)


def test_bf16_form_is_deterministic(gpu_lib):
    # no atomics and fixed reduction orders: a second run gives the same bits
    st = small_random_csr(3000, 1200, 15, 4, dist="lognormal")
    _, B1 = _sketch(gpu_lib, st, 40, precision="bf16")
    _, B2 = _sketch(gpu_lib, st, 40, precision="bf16")
    np.testing.assert_array_equal(B1, B2)


@pytest.mark.parametrize("cqr2", ["off", "final", "all"])
def test_bf16_form_ill_conditioned_panels(gpu_lib, cqr2):
    # column j scaled by max(10^(-j / 16), 10^-4): the top singular values of every buffer spread
    # over about three decades and the FP32 sketch is nearly exact (cov-err about 3e-6).  BF16
    # storage of the basis then sets a floor: rounding a stored direction by a relative u = 2^-8
    # (BF16's unit roundoff) tilts it by an angle of order u, which loses about u^2 lambda_max of
    # A^T A's energy, so the extra cov-err is bounded by a small multiple of
    # u^2 lambda_max / ||A||_F^2 (6.5e-6 here) instead of 5% of the FP32 value.  Property 1 holds
    # regardless, in every CholeskyQR2 mode.
    st = small_random_csr(3000, 400, 40, 8, dist="normal")
    vals = st.values * np.maximum(10.0 ** (-st.indices / 16.0), 1e-4).astype(np.float32)
    st = type(st)(st.indptr, st.indices, vals.astype(np.float32), st.d, st.meta)
    A = st.to_scipy()
    _, B32 = _sketch(gpu_lib, st, 40)
    _, B16 = _sketch(gpu_lib, st, 40, precision="bf16", cqr2=cqr2)
    f2 = evaluate.fro2(A)
    lmin, _ = evaluate.cov_extremes(A, B16)
    assert lmin >= -1e-5 * f2
    lam_max = float(evaluate.top_singular_values(A, 1)[0]) ** 2
    floor = 2.0 ** -16 * lam_max / f2
    e32, e16 = evaluate.cov_err(A, B32), evaluate.cov_err(A, B16)
    assert e16 <= 1.05 * e32 + 2.0 * floor, (e16, e32, floor)

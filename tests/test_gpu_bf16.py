"""The BF16 precision form (panels of SimultaneousIteration stored in BF16, FP32 accumulation).

It is not element-wise comparable with the FP64 oracle: BF16 storage changes the subspace the
iteration finds.  What must hold (the design keeps P P^T a compression of A'^T A' onto the
stored basis, so Property 1 of Sec. 3 is kept for the FP32 values):
* B^T B <= A^T A up to FP32 rounding (lambda_min(A^T A - B^T B) >= -tol ||A||_F^2);
* cov-err (Sec. 4) within 5% of the FP32 form's on the same input, same q and same random
  blocks (the fixed-cov-err rule the two forms are compared under);
* exact buffers (n <= ell) are untouched by the panel precision.
"""

import numpy as np
import pytest

from oracle import evaluate
from workloads import stream_1e4_d1e3, small_random_csr

pytestmark = pytest.mark.gpu


def _sketch(sfd, st, ell, **opts):
    import torch

    sk = sfd.Sketch(st.d, ell, 0.25, 0, **opts)
    sk.append_csr(torch.from_numpy(st.indptr).cuda(), torch.from_numpy(st.indices).cuda(),
                  torch.from_numpy(st.values).cuda())
    return sk, sk.sketch().cpu().numpy().astype(np.float64)


def _check_form(sfd, st, ell):
    A = st.to_scipy()
    _, B32 = _sketch(sfd, st, ell)
    sk, B16 = _sketch(sfd, st, ell, precision="bf16")
    lmin, _ = evaluate.cov_extremes(A, B16)
    f2 = evaluate.fro2(A)
    assert lmin >= -1e-5 * f2
    e32, e16 = evaluate.cov_err(A, B32), evaluate.cov_err(A, B16)
    assert e16 <= 1.05 * e32, (e16, e32)
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
    _check_form(gpu_lib, st, ell)


def test_bf16_form_on_10k_rows(gpu_lib):
    st = stream_1e4_d1e3()
    sk, e16, e32 = _check_form(gpu_lib, st, 20)
    assert sk.stats()["flushes"] == 10


def test_bf16_form_exact_when_rows_at_most_ell(gpu_lib):
    st = small_random_csr(12, 300, 9, 7)
    _, B32 = _sketch(gpu_lib, st, 20)
    _, B16 = _sketch(gpu_lib, st, 20, precision="bf16")
    np.testing.assert_array_equal(B16, B32)

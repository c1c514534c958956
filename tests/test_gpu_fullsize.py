"""The full-size streams in the launch configuration the bench times, checked through properties
that hold at any size (the oracle cannot run them whole):

* Property 1 of the FD family (Sec. 2.1): B^T B <= A^T A, i.e. the smallest eigenvalue of
  A^T A - B^T B is >= 0 up to the FP32 rounding of the panels;
* Theorem 3.1: ||A^T A - B^T B||_2 <= ||A - A_k||_F^2 / (alpha ell - k), alpha = 6/41, for
  k < alpha ell (it holds with probability 1 - delta; delta = 0.01 here).

Both sides come from sfd_evaluate (FP64 Lanczos on the GPU, checked against the oracle's
evaluator and ARPACK in test_gpu_eval.py).
"""

import pytest

pytestmark = pytest.mark.gpu

ALPHA = 6.0 / 41.0


def _check(gpu_lib, indptr, indices, values, d, ell, k):
    sk = gpu_lib.Sketch(d, ell, 0.25, 0)
    sk.append_csr(indptr, indices, values)
    B = sk.sketch()
    r = gpu_lib.evaluate(indptr, indices, values, d, B, k=k, steps=160)
    fro2 = r["fro2A"]
    assert r["cov_min"] >= -1e-5 * fro2
    bound = (fro2 - r["top_k_energy"]) / (ALPHA * ell - k)
    assert r["cov_max"] <= bound
    return r, bound


@pytest.mark.timeout(170)
def test_million_row_stream_properties(gpu_lib):
    # 10^6 rows, d = 10^5, ell = 50 (ten buffers of 10^5 rows); host-generated like the bench
    import torch

    from workloads import stream_1e6_d1e5

    st = stream_1e6_d1e5(seed=0)
    dev = [torch.from_numpy(a).cuda() for a in (st.indptr, st.indices, st.values)]
    r, bound = _check(gpu_lib, *dev, st.d, 50, 5)
    assert r["cov_err"] < 0.01


def test_ell200_stream_properties(gpu_lib):
    # 2x10^6 rows, d = 5x10^4, ell = 200 (forty buffers), generated on the device like the bench
    from workloads.device import stream_2e6_d5e4

    indptr, indices, values = stream_2e6_d5e4("cuda")
    _check(gpu_lib, indptr, indices, values, 50_000, 200, 10)

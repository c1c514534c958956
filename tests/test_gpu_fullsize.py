"""The full-size streams in the launch configuration the bench times, checked through properties
that hold at any size (the oracle cannot run them whole):

* Property 1 of the FD family (Sec. 2.1): B^T B <= A^T A, i.e. the smallest eigenvalue of
  A^T A - B^T B is >= 0 up to the FP32 rounding of the panels;
* Theorem 3.1: ||A^T A - B^T B||_2 <= ||A - A_k||_F^2 / (alpha ell - k), alpha = 6/41, for
  k < alpha ell (it holds with probability 1 - delta; delta = 0.01 here).

Both sides come from sfd_evaluate (FP64 Lanczos on the GPU, checked against the oracle's
evaluator and ARPACK in test_gpu_eval.py).  Lanczos Ritz values lie inside the spectrum
(theta_max <= lambda_max, theta_min >= lambda_min, and the top-k Ritz sum is at most the top-k
energy), so each inequality is asserted with the Ritz residuals ||M y - theta y|| (the distance
from each Ritz value to the spectrum) added on the side that could hide a violation, the
residuals must be small against the bound's margin, and a second start vector must give the same
extremes within them.

The first 10^5 rows of the 10^6-row stream (one 5*10^6-entry buffer at d = 10^5, ell = 50) are
also folded by the oracle itself, with the power count shortened to q = 3 on both sides: the
kernels then run at the headline buffer's full shape.
"""

import numpy as np
import pytest

from oracle import SFDOracle, evaluate
from tests.parity import assert_sigma2_close

pytestmark = pytest.mark.gpu

ALPHA = 6.0 / 41.0


def _check(gpu_lib, indptr, indices, values, d, ell, k):
    sk = gpu_lib.Sketch(d, ell, 0.25, 0)
    sk.append_csr(indptr, indices, values)
    B = sk.sketch()
    r = gpu_lib.evaluate(indptr, indices, values, d, B, k=k, steps=160)
    fro2 = r["fro2A"]
    # Property 1 at the low end of the spectrum (its Ritz value converges slowest: the residual is
    # reported and bounded, the Ritz value itself must clear the rounding threshold)
    assert r["cov_min"] >= -1e-5 * fro2, r
    assert r["cov_min_res"] <= 1e-3 * fro2, r
    # Theorem 3.1 with lambda_max taken at theta_max + residual and the top-k energy at its largest
    # value the residuals allow
    bound = (fro2 - r["top_k_energy"] - r["top_k_res"]) / (ALPHA * ell - k)
    assert r["cov_max"] + r["cov_max_res"] <= bound, (r, bound)
    # the uncertainty is small against the margin and against ||A||_F^2
    assert r["cov_max_res"] <= 0.1 * (bound - r["cov_max"]), r
    assert r["top_k_res"] <= 1e-3 * fro2, r
    # another start vector finds the same extremes
    r2 = gpu_lib.evaluate(indptr, indices, values, d, B, k=0, steps=160, seed=7)
    assert abs(r2["cov_max"] - r["cov_max"]) <= r["cov_max_res"] + r2["cov_max_res"] + 1e-9 * fro2
    assert abs(r2["cov_min"] - r["cov_min"]) <= r["cov_min_res"] + r2["cov_min_res"] + 1e-9 * fro2
    print(f"cov [{r['cov_min']:.4e} +- {r['cov_min_res']:.1e}, {r['cov_max']:.4e} +- {r['cov_max_res']:.1e}], "
          f"bound {bound:.4e}, top-k res {r['top_k_res']:.1e}, fro2 {fro2:.4e}")
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


@pytest.mark.timeout(170)
def test_headline_buffer_matches_oracle(gpu_lib):
    # one buffer of the headline stream at its full size (5*10^6 entries, d = 10^5, ell = 50,
    # 64-wide panels, XCD-local pieces in the transposed products, four lanes), q = 3 on both sides
    import torch

    from workloads import stream_1e6_d1e5

    st = stream_1e6_d1e5(seed=0, n=100_000)
    o = SFDOracle(st.d, 50, 0.25, 0, q=3, unit_roundoff=2.0 ** -24)
    o.append_csr(st.indptr, st.indices, st.values)
    sk = gpu_lib.Sketch(st.d, 50, 0.25, 0, q=3)
    sk.append_csr(*[torch.from_numpy(a).cuda() for a in (st.indptr, st.indices, st.values)])
    s = sk.stats()
    assert s["flushes"] == o.flushes == 1 and s["vs_calls"] == o.vs_calls
    want = o.log[0]["attempts"][-1]["ln_norm"]
    assert abs(s["last_ln_norm"] - want) <= 1e-3 * abs(want)
    B = sk.sketch().cpu().numpy().astype(np.float64)
    Bo = o.sketch()
    assert evaluate.gram_distance(B, Bo) <= 1e-4
    assert_sigma2_close(B, Bo)

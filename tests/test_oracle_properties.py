"""Property tests of the SparseFrequentDirections oracle over many small random streams
(hypothesis, derandomized, so the drawn cases are fixed):

* Property 1 (Sec. 3): B^T B <= A^T A, i.e. lambda_min(A^T A - B^T B) >= 0 up to rounding, for any
  stream, including empty rows, repeated column ids and streams shorter than ell;
* Theorem 3.1 with k = 0: ||A^T A - B^T B||_2 <= ||A||_F^2 / (alpha ell), alpha = 6/41 (it holds
  with probability 1 - delta; the cases are fixed, so the test is deterministic);
* exactness when the stream has at most ell rows (every row is kept: B^T B = A^T A);
* the structural live-row count never exceeds ell and the sketch has shape ell x d.
"""

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as hst

from oracle import SFDOracle, evaluate
from oracle.shrink import ALPHA
from workloads import small_random_csr

pytestmark = pytest.mark.cpu


@settings(max_examples=40, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow])
@given(n=hst.integers(1, 400), d=hst.integers(2, 48), ell=hst.integers(1, 14), lam=hst.floats(0.5, 10.0),
       seed=hst.integers(0, 2 ** 20), dist=hst.sampled_from(["normal", "lognormal"]),
       dup=hst.sampled_from([0.0, 0.15]), empty=hst.sampled_from([0.0, 0.25]))
def test_property1_theorem_and_exactness(n, d, ell, lam, seed, dist, dup, empty):
    ell = min(ell, d)
    st = small_random_csr(n, d, lam, seed, dist=dist, dup_rate=dup, empty_rate=empty)
    o = SFDOracle(d, ell, 0.25, seed)
    o.append_csr(st.indptr, st.indices, st.values)
    B, live, _ = o.query()
    assert B.shape == (ell, d)
    assert 0 <= live <= ell
    A = st.to_scipy()
    fro2 = evaluate.fro2(A)
    lmin, lmax = evaluate.cov_extremes(A, B)
    scale = max(fro2, 1e-300)
    assert lmin >= -1e-9 * scale
    assert lmax <= fro2 / (ALPHA * ell) + 1e-9 * scale
    if st.n <= ell:
        Ad = A.toarray()
        np.testing.assert_allclose(B.T @ B, Ad.T @ Ad, atol=1e-10 * scale)

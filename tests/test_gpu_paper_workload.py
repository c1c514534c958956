"""The paper's own synthetic workload (Sec. 4, "Datasets": rows of exactly z distinct +-1 entries,
90% of them in the first 1.5 z columns) through the HIP path, against the FP64 oracle: SFD with
BoostedSparseShrink, SFD with SparseShrink alone (VerifySpectral off, the variant of the paper's
experiments, Sec. 4) and FrequentDirections (Sec. 2.1, the paper's comparator).  Bar: the FP32 one
of the other parity tests (relative Frobenius distance of B^T B <= 1e-4, sigma_i^2 one by one), and
the sketches' covariance errors (Sec. 4, "Measurements") from the GPU evaluator next to the FD
bound of Lemma 2.1 / the claim of Sec. 4."""

import numpy as np
import pytest

from oracle import FDBatchOracle, SFDOracle, evaluate
from tests.parity import assert_sigma2_close
from workloads import paper_head_tail

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _dev(st):
    import torch

    return (torch.from_numpy(np.ascontiguousarray(st.indptr)).cuda(),
            torch.from_numpy(np.ascontiguousarray(st.indices)).cuda(),
            torch.from_numpy(np.ascontiguousarray(st.values)).cuda())


@pytest.mark.parametrize("n,d,z,ell", [
    (3000, 1000, 100, 50),   # the paper's defaults (d, z, ell), 3,000 of its 10,000 rows: 6 full buffers
    (2000, 1000, 20, 20),    # sparser rows, smaller sketch: buffers cut by the rows = d rule
    (1500, 3000, 100, 50),   # wider d (Table 1 range), head of 150 columns out of 3,000
])
def test_head_tail_stream_matches_oracle(gpu_lib, n, d, z, ell):
    st = paper_head_tail(n=n, d=d, z=z, seed=1)
    dev = _dev(st)
    A = st.to_scipy()
    for verify in (True, False):
        print(f"head/tail n={n} d={d} z={z} ell={ell} verify={verify}", flush=True)
        o = SFDOracle(d, ell, 0.25, 0, unit_roundoff=U32, verify=verify)
        o.append_csr(st.indptr, st.indices, st.values)
        Bo = o.sketch()
        sk = gpu_lib.Sketch(d, ell, 0.25, 0, verify=verify)
        sk.append_csr(*dev)
        Bt = sk.sketch()
        B = Bt.cpu().numpy().astype(np.float64)
        s = sk.stats()
        assert s["flushes"] == o.flushes
        assert (s["vs_calls"] > 0) == verify
        assert evaluate.gram_distance(B, Bo) <= 1e-4
        assert_sigma2_close(B, Bo)
        # Property 1 (B^T B <= A^T A) and the covariance error, from the GPU evaluator (dense d: exact)
        r = gpu_lib.evaluate(*dev, d, Bt, k=10, steps=min(d, 400))
        assert r["cov_min"] >= -1e-5 * r["fro2A"]
        assert r["cov_err"] == pytest.approx(evaluate.cov_err(A, B), rel=1e-3)
        sk.close()


def test_head_tail_stream_fd_matches_fd_oracle(gpu_lib):
    # FrequentDirections on the same rows: DenseShrink of ell-row batches (Sec. 2.1)
    st = paper_head_tail(n=1000, d=1000, z=100, seed=2)
    ell = 50
    o = FDBatchOracle(st.d, ell)
    o.append_csr(st.indptr, st.indices, st.values)
    sk = gpu_lib.Sketch(st.d, ell, 0.25, 0, algorithm="fd")
    sk.append_csr(*_dev(st))
    B = sk.sketch().cpu().numpy().astype(np.float64)
    assert sk.stats()["flushes"] == o.flushes == st.n // ell
    assert evaluate.gram_distance(B, o.sketch()) <= 1e-4
    assert_sigma2_close(B, o.sketch())
    A = st.to_scipy()
    lmin, lmax = evaluate.cov_extremes(A, B)
    assert lmin >= -1e-5 * evaluate.fro2(A)
    assert lmax <= evaluate.fd_bound(A, ell, 10) * (1 + 1e-4)  # Lemma 2.1 with k = 10
    sk.close()

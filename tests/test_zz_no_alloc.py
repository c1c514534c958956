"""sfd_evaluate_noalloc (the evaluator with its work memory in the library's fixed device scratch)
against sfd_evaluate (the same kernels on per-call allocations): equal results field by field, on
two calls in a row where the second input is smaller than the first, so the second runs on scratch
that still holds the first call's contents; and inputs too large for the scratch rejected with
SFD_E_TOOBIG.  Both calls go through the C ABI."""

import math

import numpy as np
import pytest

from workloads import small_random_csr

pytestmark = pytest.mark.gpu

FIELDS = ("fro2A", "cov_min", "cov_max", "cov_err", "top_k_energy", "proj_num", "proj_err", "steps",
          "cov_min_res", "cov_max_res", "top_k_res")


def _dev(st):
    import torch

    return (torch.from_numpy(np.ascontiguousarray(st.indptr)).cuda(),
            torch.from_numpy(np.ascontiguousarray(st.indices)).cuda(),
            torch.from_numpy(np.ascontiguousarray(st.values)).cuda())


def _same(a, b):
    for f in FIELDS:
        x, y = a[f], b[f]
        if isinstance(x, float) and math.isnan(x):
            assert math.isnan(y), f
        else:
            assert x == y, (f, x, y)


def test_noalloc_evaluate_equals_evaluate_on_two_calls(gpu_lib):
    # first call: 6,000 rows x 3,000 columns (about 9e4 entries), k = 8; second call: a smaller input
    # (fewer rows, columns and entries, smaller ell and k) on the scratch the first call left behind
    cases = [(6000, 3000, 15, 40, 8, 120, 11), (700, 900, 6, 12, 3, 60, 12)]
    for n, d, lam, ell, k, steps, seed in cases:
        print(f"noalloc evaluate: n={n} d={d} lam={lam} ell={ell} k={k} steps={steps}", flush=True)
        st = small_random_csr(n, d, lam, seed, dist="lognormal", dup_rate=0.02)
        sk = gpu_lib.Sketch(d, ell, 0.25, 0)
        dev = _dev(st)
        sk.append_csr(*dev)
        B = sk.sketch()
        ref = gpu_lib.evaluate(*dev, d, B, k=k, steps=steps, seed=5)
        got = gpu_lib.evaluate(*dev, d, B, k=k, steps=steps, seed=5, noalloc=True)
        _same(ref, got)
        assert got["cov_err"] > 0.0 and np.isfinite(got["proj_err"])
        sk.close()


def test_noalloc_evaluate_without_sketch_and_k0(gpu_lib):
    # ell = 0 (no sketch: the extremes of A^T A) and k = 0 (proj-err skipped: NaN on both sides)
    st = small_random_csr(500, 400, 8, 21, dist="normal")
    dev = _dev(st)
    ref = gpu_lib.evaluate(*dev, st.d, None, k=0, steps=50, seed=3)
    got = gpu_lib.evaluate(*dev, st.d, None, k=0, steps=50, seed=3, noalloc=True)
    _same(ref, got)
    assert math.isnan(got["proj_err"])


def test_noalloc_evaluate_rejects_work_beyond_the_scratch(gpu_lib):
    # d = 2e6 with 160 Lanczos steps needs a 161 x 2e6 FP64 basis (2.6 GB), beyond the 64 MiB
    st = small_random_csr(20, 2_000_000, 4, 31, dist="normal")
    dev = _dev(st)
    with pytest.raises(gpu_lib.SfdError) as e:
        gpu_lib.evaluate(*dev, st.d, None, k=0, steps=160, noalloc=True)
    assert e.value.code == gpu_lib.SFD_E_TOOBIG
    # a bad index is still reported as such (the checks run before the size test)
    bad = small_random_csr(50, 300, 4, 32, dist="normal")
    bad.indices[3] = 300
    with pytest.raises(gpu_lib.SfdError) as e:
        gpu_lib.evaluate(*_dev(bad), 300, None, k=0, steps=20, noalloc=True)
    assert e.value.code == gpu_lib.SFD_E_INDEX
    # and the scratch still serves a call that fits
    ok = small_random_csr(300, 200, 6, 33, dist="lognormal")
    dev = _dev(ok)
    _same(gpu_lib.evaluate(*dev, 200, None, k=0, steps=40), gpu_lib.evaluate(*dev, 200, None, k=0, steps=40,
                                                                               noalloc=True))

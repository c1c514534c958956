"""Writes the stored expected values under tests/golden/ by calling the oracle only.

    python tests/golden/make_golden.py

stream_1e4_d1e3_oracle.json: the FP64 oracle on the 10,000 x 1,000 Zipf stream (ell = 20, seed 0):
squared singular values of B, per-buffer VerifySpectral log norms, cov-err and the
FrequentDirections bound with k = 10.
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import SFDOracle, evaluate  # noqa: E402
from workloads import stream_1e4_d1e3  # noqa: E402


def golden_record():
    st = stream_1e4_d1e3()
    o = SFDOracle(st.d, 20, 0.25, 0)
    o.append_csr(st.indptr, st.indices, st.values)
    B = o.sketch()
    A = st.to_scipy()
    return {
        "workload": "zipf-poisson n=10000 d=1000 lambda=10 s=1.1 planted rank-10 + N(0,0.1^2), ell=20, eps=1/4, seed=0",
        "sigma2_B": (np.linalg.svd(B, compute_uv=False) ** 2).tolist(),
        "buffers": [{"rows": r["rows"], "nnz": r["nnz"],
                     "ln_norm": [a.get("ln_norm") for a in r["attempts"]],
                     "t": [a.get("t") for a in r["attempts"]]} for r in o.log],
        "cov_err": evaluate.cov_err(A, B),
        "fd_bound_k10": evaluate.fd_bound(A, 20, 10) / evaluate.fro2(A),
        "fro2_A": evaluate.fro2(A),
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "stream_1e4_d1e3_oracle.json"), "w") as f:
        json.dump(golden_record(), f, indent=1)

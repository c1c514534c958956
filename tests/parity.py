"""Comparisons of a GPU sketch with the oracle's beyond the relative Frobenius distance of B^T B
(which the largest directions dominate): the sorted sigma_i^2(B) (eigenvalues of B B^T) one by
one."""

import json
import os

import numpy as np


def sigma2(B):
    """sigma_i(B)^2, descending (FP64)."""
    B = np.asarray(B, dtype=np.float64)
    return np.sort(np.linalg.eigvalsh(B @ B.T))[::-1]


def sigma2_errors(Bg, Bo):
    """(per-direction relative error |s_g - s_o| / s_o over the directions with s_o > 0, absolute
    error over all directions relative to s_o,1) of the sorted sigma_i^2."""
    sg, so = sigma2(Bg), sigma2(Bo)
    diff = np.abs(sg - so)
    top = so[0] if so.size and so[0] > 0 else 1.0
    pos = so > 1e-12 * top
    rel = diff[pos] / so[pos]
    return (float(rel.max()) if rel.size else 0.0), float(diff.max() / top if diff.size else 0.0)


def assert_sigma2_close(Bg, Bo, rtol=1e-3, atol=1e-5):
    """Every sigma_i^2 of the GPU sketch within rtol s_o,i + atol s_o,1 of the oracle's.  The
    FP32 path carries an absolute error of about u_32 sqrt(d) s_1^2 per eigenvalue (the panels'
    rounding), so the absolute term scales with the largest; the relative term then binds on
    every direction down to s_i^2 ~ (atol / rtol) s_1^2."""
    sg, so = sigma2(Bg), sigma2(Bo)
    assert sg.shape == so.shape
    log = os.environ.get("SFD_PARITY_LOG")
    if log:  # observed errors, for the record of the tolerances
        rel, ab = sigma2_errors(Bg, Bo)
        with open(log, "a") as f:
            f.write(json.dumps({"test": os.environ.get("PYTEST_CURRENT_TEST", "?"), "rel_max": rel, "abs_over_s1": ab,
                                "s_min_over_s1": float(so[-1] / so[0]) if so[0] > 0 else 0.0}) + "\n")
    tol = rtol * np.abs(so) + atol * max(so[0], 0.0)
    bad = np.nonzero(np.abs(sg - so) > tol)[0]
    assert bad.size == 0, [(int(i), float(sg[i]), float(so[i])) for i in bad[:5]]

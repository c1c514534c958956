"""The oracle still reproduces the stored config-1 record (written by tests/golden/make_golden.py)."""

import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.cpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_golden_record_reproduces():
    from tests.golden.make_golden import golden_record

    with open(os.path.join(HERE, "stream_1e4_d1e3_oracle.json")) as f:
        want = json.load(f)
    got = golden_record()
    np.testing.assert_allclose(got["sigma2_B"], want["sigma2_B"], rtol=1e-8)
    assert [b["rows"] for b in got["buffers"]] == [b["rows"] for b in want["buffers"]]
    assert [b["t"] for b in got["buffers"]] == [b["t"] for b in want["buffers"]]
    np.testing.assert_allclose(got["cov_err"], want["cov_err"], rtol=1e-7)
    assert got["cov_err"] <= got["fd_bound_k10"]

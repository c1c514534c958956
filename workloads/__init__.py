"""Seeded synthetic row streams for Sparse Frequent Directions.

Input generators only: this package holds none of the method's arithmetic.  Both the oracle
(tests, CPU baseline) and the HIP path read the CSR arrays it returns.
"""

from .synthetic import (
    CsrStream,
    zipf_cdf,
    poisson_zipf_pattern,
    small_random_csr,
    config1_fp64_reference,
    config2_plain_fp32,
    config3_precision,
    config4_batch_stream,
    paper_head_tail,
)

__all__ = [
    "CsrStream",
    "zipf_cdf",
    "poisson_zipf_pattern",
    "small_random_csr",
    "config1_fp64_reference",
    "config2_plain_fp32",
    "config3_precision",
    "config4_batch_stream",
    "paper_head_tail",
]

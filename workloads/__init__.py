"""Seeded synthetic row streams for Sparse Frequent Directions.

Input generators only: this package holds none of the method's arithmetic.  Both the oracle
(tests, CPU baseline) and the HIP path read the CSR arrays it returns.
"""

from .synthetic import (
    CsrStream,
    zipf_cdf,
    poisson_zipf_pattern,
    small_random_csr,
    stream_1e4_d1e3,
    stream_1e6_d1e5,
    stream_2e6_d5e4,
    batch_stream_d2e4,
    paper_head_tail,
    spiked_stream,
)

__all__ = [
    "CsrStream",
    "zipf_cdf",
    "poisson_zipf_pattern",
    "small_random_csr",
    "stream_1e4_d1e3",
    "stream_1e6_d1e5",
    "stream_2e6_d5e4",
    "batch_stream_d2e4",
    "paper_head_tail",
    "spiked_stream",
]

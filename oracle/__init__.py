"""Plain FP64 CPU oracle for Sparse Frequent Directions (Ghashami, Liberty & Phillips,
"Efficient Frequent Directions Algorithm for Sparse Matrices", arXiv:1602.00412).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this package: only the
test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.
It shares no code with the HIP path (``paper_1602_00412_amd``); the only module both sides
read is the seeded input generator package ``workloads``, which holds none of the method's
arithmetic.

Contents (each function cites the passage it follows):

* ``philox``    -- Philox4x64-10 counter-based generator (Salmon et al., SC'11), written from
                   its published definition; pinned against ``numpy.random.Philox``.
* ``rng``       -- the key/counter schedule that turns (seed, stream, buffer, attempt,
                   purpose) into the Gaussian start block G of SimultaneousIteration (Alg 1)
                   and the unit vector x of VerifySpectral (Alg 6).
* ``shrink``    -- SimultaneousIteration (Alg 1), SparseShrink (Alg 3),
                   BoostedSparseShrink (Alg 4), DenseShrink (Alg 5), VerifySpectral (Alg 6).
* ``stream``    -- the SparseFrequentDirections stream driver (Alg 2) with query and merge,
                   and the dense FrequentDirections comparator (Sec. 2.1).
* ``evaluate``  -- the paper's accuracy measures (Sec. 4, "Measurements").

Every function here is pinned by a ``-m "not gpu"`` test in ``tests/`` to something other
than itself (closed forms, invariants, library routines, brute force); see the test files.
"""

from .philox import philox4x64_10, philox_uniform01
from .rng import start_block, sphere_vector, PURPOSE_SI, PURPOSE_VS, PURPOSE_QUERY_SI, PURPOSE_QUERY_VS
from .shrink import (
    ALPHA,
    simultaneous_iteration,
    sparse_shrink,
    dense_shrink,
    verify_spectral,
    boosted_sparse_shrink,
    si_iterations,
    vs_steps,
    NoConvergence,
)
from .stream import SFDOracle, FDOracle, FDBatchOracle
from . import evaluate

__all__ = [
    "philox4x64_10",
    "philox_uniform01",
    "start_block",
    "sphere_vector",
    "PURPOSE_SI",
    "PURPOSE_VS",
    "PURPOSE_QUERY_SI",
    "PURPOSE_QUERY_VS",
    "ALPHA",
    "simultaneous_iteration",
    "sparse_shrink",
    "dense_shrink",
    "verify_spectral",
    "boosted_sparse_shrink",
    "si_iterations",
    "vs_steps",
    "NoConvergence",
    "SFDOracle",
    "FDOracle",
    "evaluate",
]

"""Launch variants of the sparse products and graph replay give the same bits.

The products' launch configuration (static grid, persistent grid fed by device work queues, and
that grid with the most popular columns' rows of X staged in LDS for Y = A' X) and the capture of
SimultaneousIteration and VerifySpectral steps as HIP graphs change how the work is scheduled,
never the order in which any output row's entries are summed.  So every combination must give
the sketch of the default configuration bit for bit -- in FP32 and in the BF16 form, with and
without XCD-local pieces -- and the FP32 one must match the oracle.
"""

import numpy as np
import pytest

from oracle import SFDOracle, evaluate
from workloads import small_random_csr

pytestmark = pytest.mark.gpu


def _run(sfd, st, ell, **opts):
    import torch

    sk = sfd.Sketch(st.d, ell, 0.25, 0, **opts)
    sk.append_csr(*[torch.from_numpy(a).cuda() for a in (st.indptr, st.indices, st.values)])
    B = sk.sketch().cpu().numpy()
    sk.close()
    return B


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("bands", [None, 8])
def test_launch_modes_and_graphs_keep_the_bits(gpu_lib, precision, bands):
    # Zipf(1.1) columns over d = 2,500 (hot columns with hundreds of entries per buffer), several
    # buffers, a ragged tail, 64-wide panels
    st = small_random_csr(6000, 2500, 25, 51, s=1.1, dist="lognormal")
    extra = {} if bands is None else dict(csc_bands=bands, csc_hot_min=16)
    ref = _run(gpu_lib, st, 40, precision=precision, autotune=False, graphs=False, launch="static", **extra)
    for launch in ("queue", "stage", "auto"):
        for graphs in (False, True):
            print(f"precision={precision} bands={bands} launch={launch} graphs={graphs}", flush=True)
            B = _run(gpu_lib, st, 40, precision=precision, graphs=graphs, launch=launch, **extra)
            np.testing.assert_array_equal(B, ref)
    if precision == "fp32":
        o = SFDOracle(st.d, 40, 0.25, 0, unit_roundoff=2.0 ** -24)
        o.append_csr(st.indptr, st.indices, st.values)
        assert evaluate.gram_distance(ref.astype(np.float64), o.sketch()) <= 1e-4


@pytest.mark.parametrize("ell", [20, 100, 200])
def test_staged_products_at_every_panel_width(gpu_lib, ell):
    # 32-, 128- and 256-wide panels (the staged rows: 256, 64 and 32 of them in 32 KB)
    st = small_random_csr(2500, 900, 30, 52 + ell, s=1.2, dist="lognormal")
    ref = _run(gpu_lib, st, ell, autotune=False, graphs=False, launch="static")
    B = _run(gpu_lib, st, ell, launch="stage")
    np.testing.assert_array_equal(B, ref)

"""Batched streams (sfd_batch_*): stream s of a batch is exactly an sfd_t with STREAM_ID = s.

The batch shares the lanes between streams and runs buffer steps of different streams
concurrently; every buffer step uses the same kernels and decompositions as a single-stream
handle, so the sketches agree bit for bit.  Two streams are also checked against the oracle.
"""

import numpy as np
import pytest

from oracle import SFDOracle, evaluate
from workloads import small_random_csr

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _cat(streams):
    """One CSR block holding the streams one after another, and its segment table."""
    indptr = [np.zeros(1, dtype=np.int64)]
    idx, val, starts = [], [], [0]
    base = 0
    for st in streams:
        indptr.append(st.indptr[1:] - st.indptr[0] + base)
        base += st.nnz
        idx.append(st.indices)
        val.append(st.values)
        starts.append(starts[-1] + st.n)
    return (np.concatenate(indptr), np.concatenate(idx) if idx else np.zeros(0, np.int32),
            np.concatenate(val) if val else np.zeros(0, np.float32), np.array(starts, dtype=np.int64))


def _single(sfd, st, d, ell, sid, **opts):
    import torch

    sk = sfd.Sketch(d, ell, 0.25, 0, stream_id=sid, **opts)
    if st.n:
        sk.append_csr(torch.from_numpy(st.indptr).cuda(), torch.from_numpy(st.indices).cuda(),
                      torch.from_numpy(st.values).cuda())
    return sk, sk.sketch().cpu().numpy()


@pytest.mark.parametrize("device,ell,bands", [(True, 12, None), (False, 12, None), (True, 80, None), (True, 12, 8)])
def test_batch_equals_single_streams(gpu_lib, device, ell, bands):
    # bands = 8: XCD-local pieces forced, so every buffer takes the lanes (as single handles do)
    import torch

    d = 300
    lens = [0, 40, 700, 1500, 9, 620]
    streams = [small_random_csr(n, d, 8, 100 + s, dist="lognormal") for s, n in enumerate(lens)]
    indptr, idx, val, starts = _cat(streams)
    b = gpu_lib.Batch(len(streams), d, ell)
    opts = {}
    if bands is not None:
        b.set_option(gpu_lib.OPT_CSC_BANDS, bands)
        b.set_option(gpu_lib.OPT_CSC_HOT_MIN, 4)
        opts = dict(csc_bands=bands, csc_hot_min=4)
    order = [3, 0, 5, 1, 4, 2]  # segments in any stream order
    seg_starts = []
    block_ptr, block_idx, block_val = [np.zeros(1, np.int64)], [], []
    base = 0
    for s in order:
        st = streams[s]
        seg_starts.append(sum(streams[t].n for t in order[:order.index(s)]))
        block_ptr.append(st.indptr[1:] - st.indptr[0] + base)
        base += st.nnz
        block_idx.append(st.indices)
        block_val.append(st.values)
    seg_starts.append(sum(st.n for st in streams))
    bp, bi, bv = np.concatenate(block_ptr), np.concatenate(block_idx), np.concatenate(block_val)
    if device:
        b.append_csr(order, seg_starts, torch.from_numpy(bp).cuda(), torch.from_numpy(bi).cuda(),
                     torch.from_numpy(bv).cuda())
    else:
        b.append_csr(order, seg_starts, bp, bi, bv)
    B = b.sketch().cpu().numpy()
    for s, st in enumerate(streams):
        sk, Bs = _single(gpu_lib, st, d, ell, s, **opts)
        np.testing.assert_array_equal(B[s], Bs)
        assert b.stats(s)["flushes"] == sk.stats()["flushes"]
        assert b.stats(s)["vs_calls"] == sk.stats()["vs_calls"]


def test_batch_in_several_calls_and_against_oracle(gpu_lib):
    import torch

    d, ell = 250, 10
    streams = [small_random_csr(n, d, 9, 200 + s, dist="lognormal") for s, n in enumerate([900, 1300])]
    b = gpu_lib.Batch(2, d, ell)
    # rows arrive interleaved over three calls
    cuts = [[0, 300, 650, 900], [0, 500, 1000, 1300]]
    for c in range(3):
        parts = [streams[s].rows(cuts[s][c], cuts[s][c + 1]) for s in range(2)]
        indptr, idx, val, starts = _cat(parts)
        b.append_csr([0, 1], starts, torch.from_numpy(indptr).cuda(), torch.from_numpy(idx).cuda(),
                     torch.from_numpy(val).cuda())
    B = b.sketch().cpu().numpy().astype(np.float64)
    for s in range(2):
        o = SFDOracle(d, ell, 0.25, 0, stream_id=s, unit_roundoff=U32)
        o.append_csr(streams[s].indptr, streams[s].indices, streams[s].values)
        assert evaluate.gram_distance(B[s], o.sketch()) <= 1e-4
        assert b.stats(s)["flushes"] == o.flushes


def test_batch_rejects_repeated_stream_and_bad_index(gpu_lib):
    st = small_random_csr(30, 50, 5, 1)
    indptr, idx, val, starts = _cat([st, st])
    b = gpu_lib.Batch(3, 50, 5)
    with pytest.raises(gpu_lib.SfdError) as e:
        b.append_csr([1, 1], starts, indptr, idx, val)
    assert e.value.code == gpu_lib.SFD_E_ARG
    bad = idx.copy()
    bad[3] = 50
    with pytest.raises(gpu_lib.SfdError) as e:
        b.append_csr([0, 2], starts, indptr, bad, val)
    assert e.value.code == gpu_lib.SFD_E_INDEX
    assert all(b.stats(s)["rows_seen"] == 0 for s in range(3))


@pytest.mark.parametrize("ell", [12, 32])
def test_graph_replay_and_autotune_keep_the_bits(gpu_lib, ell):
    # The lockstep groups' iteration and power step are captured once as HIP graphs and replayed
    # q + 1 (t) times; the products' launch configuration is tuned on first sight.  Three appends
    # (each runs several groups, so several graphs, each replayed many times), with eager work and
    # synchronisations in between: after every append each stream's sketch equals, bit for bit,
    # that of a batch run launch by launch with the default configuration, and that of a
    # single-stream handle.
    import torch

    d = 400
    lens = [900, 2600, 1300, 3100, 450, 1900]
    streams = [small_random_csr(n, d, 9, 300 + s, dist="lognormal") for s, n in enumerate(lens)]
    thirds = [[(st.n * j) // 3 for j in range(4)] for st in streams]
    fast = gpu_lib.Batch(len(streams), d, ell, graphs=True, autotune=True)
    plain = gpu_lib.Batch(len(streams), d, ell, graphs=False, autotune=False)
    singles = [gpu_lib.Sketch(d, ell, 0.25, 0, stream_id=s) for s in range(len(streams))]
    for j in range(3):
        parts = [st.rows(thirds[s][j], thirds[s][j + 1]) for s, st in enumerate(streams)]
        indptr, idx, val, starts = _cat(parts)
        g = [torch.from_numpy(a).cuda() for a in (indptr, idx, val)]
        sos = np.arange(len(streams), dtype=np.int32)
        for b in (fast, plain):
            b.append_csr(sos, starts, *g)
            torch.cuda.synchronize()
        for s, p in enumerate(parts):
            if p.n:
                singles[s].append_csr(*[torch.from_numpy(a).cuda() for a in (p.indptr, p.indices, p.values)])
        out_f = fast.sketch().cpu().numpy()
        out_p = plain.sketch().cpu().numpy()
        np.testing.assert_array_equal(out_f, out_p)
        for s in range(len(streams)):
            np.testing.assert_array_equal(out_f[s], singles[s].sketch().cpu().numpy())


def test_autotune_keeps_the_bits_single_stream(gpu_lib):
    # tuned configurations (static or persistent work-queue grid, gather batch) against the default
    # one, with XCD-local pieces forced so the band queues are exercised too
    import torch

    st = small_random_csr(6000, 3000, 30, 41, dist="lognormal")
    dev = [torch.from_numpy(a).cuda() for a in (st.indptr, st.indices, st.values)]
    outs = []
    for tune in (False, True, True):
        sk = gpu_lib.Sketch(st.d, 40, 0.25, 0, autotune=tune, csc_bands=8, csc_hot_min=8)
        sk.append_csr(*dev)
        outs.append(sk.sketch().cpu().numpy())
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[0], outs[2])


def test_batch_past_one_lockstep_group_equals_single_streams(gpu_lib):
    """130 streams with one full buffer each: a round of 130 buffers runs as two lockstep groups
    (a batch handle groups up to 128), and every stream's sketch still equals its single-stream
    handle's bit for bit, on both sides of the group boundary."""
    import torch

    d, ell, n = 300, 12, 320
    streams = [small_random_csr(n, d, 6, 700 + s, dist="lognormal") for s in range(130)]
    indptr, idx, val, starts = _cat(streams)
    b = gpu_lib.Batch(len(streams), d, ell)
    b.append_csr(np.arange(len(streams), dtype=np.int32), starts, torch.from_numpy(indptr).cuda(),
                 torch.from_numpy(idx).cuda(), torch.from_numpy(val).cuda())
    B = b.sketch().cpu().numpy()
    for s in (0, 1, 127, 128, 129):
        sk, Bs = _single(gpu_lib, streams[s], d, ell, s)
        assert b.stats(s)["flushes"] == sk.stats()["flushes"] >= 1
        assert np.array_equal(B[s], Bs), s

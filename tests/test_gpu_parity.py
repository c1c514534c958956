"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bar (fixed for the FP32 path): relative Frobenius distance of B^T B between the GPU sketch and
the oracle's, ||B_g^T B_g - B_o^T B_o||_F / ||B_o^T B_o||_F <= 1e-4, with the oracle fed the
same Philox start blocks and the same q, and taking its lossless-accept decision at the
panels' unit roundoff (2^-24) so both sides decide the same way.
"""

import numpy as np
import pytest

from oracle import SFDOracle, evaluate
from oracle.rng import start_block as oracle_start_block
from tests.parity import assert_sigma2_close
from workloads import CsrStream, stream_1e4_d1e3, small_random_csr

pytestmark = pytest.mark.gpu

TOL = 1e-4
U32 = 2.0 ** -24


def _torch():
    import torch

    return torch


def _dev(st):
    torch = _torch()
    return (torch.from_numpy(np.ascontiguousarray(st.indptr)).cuda(),
            torch.from_numpy(np.ascontiguousarray(st.indices)).cuda(),
            torch.from_numpy(np.ascontiguousarray(st.values)).cuda())


def _gpu_sketch(sfd, st, ell, *, blocks=None, host=False, **opts):
    sk = sfd.Sketch(st.d, ell, opts.pop("eps", 0.25), opts.pop("seed", 0), **opts)
    bounds = blocks or [(0, st.n)]
    for lo, hi in bounds:
        sub = st.rows(lo, hi)
        if host:
            sk.append_csr(sub.indptr, sub.indices, sub.values)
        else:
            sk.append_csr(*_dev(sub))
    B = sk.sketch().cpu().numpy().astype(np.float64)
    return sk, B


def _parity(B, Bo):
    """The FP32 bar: relative Frobenius distance of B^T B <= 1e-4, and every sigma_i^2 of B within
    1e-3 of the oracle's (plus 1e-5 of the largest)."""
    dist = evaluate.gram_distance(B, Bo)
    assert dist <= TOL, dist
    assert_sigma2_close(B, Bo)


def _oracle(st, ell, **kw):
    o = SFDOracle(st.d, ell, kw.pop("eps", 0.25), kw.pop("seed", 0), unit_roundoff=U32, **kw)
    o.append_csr(st.indptr, st.indices, st.values)
    return o


def test_start_block_matches_oracle(gpu_lib):
    for (seed, sid, b, a, p, d, ell) in [(0, 0, 0, 0, 0, 1000, 20), (7, 3, 5, 2, 1, 333, 1), (2**40, 9, 1, 0, 2, 97, 13)]:
        g = gpu_lib.start_block(seed, sid, b, a, p, d, ell).cpu().numpy()
        want = oracle_start_block(seed, sid, b, a, p, d, ell)
        np.testing.assert_allclose(g, want, rtol=2e-7, atol=2e-7)


@pytest.mark.parametrize("n,d,ell,lam,seed", [
    (400, 60, 5, 6, 0),      # several flushes by the rows rule, ragged tail
    (900, 80, 20, 9, 1),     # ell = 20 (L = 32), nnz budget reached
    (700, 150, 33, 12, 2),   # ell = 33 -> L = 64 padding
    (1500, 90, 50, 20, 3),   # ell = 50
])
def test_small_streams_match_oracle(gpu_lib, n, d, ell, lam, seed):
    st = small_random_csr(n, d, lam, seed, dist="lognormal")
    o = _oracle(st, ell)
    sk, B = _gpu_sketch(gpu_lib, st, ell)
    assert sk.stats()["flushes"] == o.flushes
    _parity(B, o.sketch())
    assert sk.last_live == o.query()[1]


@pytest.mark.parametrize("hot_min", [1, 16])
def test_xcd_pieces_match_oracle(gpu_lib, hot_min):
    # transposed products with the hot columns cut into per-XCD row-band pieces (forced on small
    # buffers; hot_min = 1 cuts every non-empty column, 16 a mix of cut and whole columns)
    st = small_random_csr(1500, 90, 20, 3, dist="lognormal", dup_rate=0.05)
    o = _oracle(st, 50)
    sk, B = _gpu_sketch(gpu_lib, st, 50, csc_bands=8, csc_hot_min=hot_min)
    assert sk.stats()["flushes"] == o.flushes
    _parity(B, o.sketch())
    _, B1 = _gpu_sketch(gpu_lib, st, 50, csc_bands=1)
    assert evaluate.gram_distance(B, B1) <= 1e-5


def test_xcd_pieces_with_empty_bands(gpu_lib):
    # one row holds most of the buffer's entries, so several row bands are empty and the
    # others hold few rows; plus empty rows and empty columns
    d, ell = 400, 20
    rng = np.random.default_rng(11)
    lens = rng.poisson(3, 300)
    lens[7] = 360  # about 30% of the entries: row 7's band is followed by an empty one
    lens[rng.random(300) < 0.1] = 0
    rows = [np.sort(rng.choice(d - 40, size=k, replace=False)) for k in lens]
    indptr = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum([len(r) for r in rows], out=indptr[1:])
    indices = np.concatenate(rows).astype(np.int32)
    values = rng.standard_normal(len(indices)).astype(np.float32)
    st = CsrStream(indptr, indices, values, d, dict(name="empty bands"))
    o = _oracle(st, ell)
    for hot_min in (1, 4):
        sk, B = _gpu_sketch(gpu_lib, st, ell, csc_bands=8, csc_hot_min=hot_min)
        assert sk.stats()["flushes"] == o.flushes
        _parity(B, o.sketch())


@pytest.mark.parametrize("bands,hot_min", [(1, None), (8, None), (8, 2)])
def test_large_buffer_matches_oracle(gpu_lib, bands, hot_min):
    # one 20,000-row buffer (flushed by the rows rule: 6e5 stored entries, long CSC columns whose
    # band pieces span several chunks) and a 4,000-row pending buffer folded by the query
    st = small_random_csr(24000, 20000, 30, 5, dist="lognormal")
    o = _oracle(st, 40)
    sk, B = _gpu_sketch(gpu_lib, st, 40, csc_bands=bands, csc_hot_min=hot_min)
    assert sk.stats()["flushes"] == o.flushes == 1
    _parity(B, o.sketch())


def test_1e4_row_stream_matches_oracle_and_fd_bound(gpu_lib):
    st = stream_1e4_d1e3()
    o = _oracle(st, 20)
    sk, B = _gpu_sketch(gpu_lib, st, 20)
    stats = sk.stats()
    assert stats["flushes"] == 10 and stats["vs_calls"] == o.vs_calls == 10 and stats["vs_rejects"] == 0
    _parity(B, o.sketch())
    A = st.to_scipy()
    assert evaluate.cov_err(A, B) <= evaluate.fd_bound(A, 20, 10) / evaluate.fro2(A)
    # the last buffer's VerifySpectral log norm agrees with the oracle's
    want = o.log[-1]["attempts"][-1]["ln_norm"]
    assert abs(stats["last_ln_norm"] - want) <= 1e-3 * abs(want)


def test_block_boundaries_do_not_change_the_result(gpu_lib):
    st = small_random_csr(600, 70, 8, 4)
    _, B1 = _gpu_sketch(gpu_lib, st, 10)
    _, B2 = _gpu_sketch(gpu_lib, st, 10, blocks=[(0, 1), (1, 69), (69, 70), (70, 333), (333, 600)])
    np.testing.assert_array_equal(B1, B2)


def test_host_and_device_inputs_agree(gpu_lib):
    st = small_random_csr(500, 64, 7, 5)
    _, Bd = _gpu_sketch(gpu_lib, st, 12)
    _, Bh = _gpu_sketch(gpu_lib, st, 12, host=True, blocks=[(0, 250), (250, 500)])
    np.testing.assert_array_equal(Bd, Bh)


def test_query_is_non_destructive(gpu_lib):
    st = small_random_csr(800, 60, 6, 6)
    torch = _torch()
    a = gpu_lib.Sketch(st.d, 8)
    b = gpu_lib.Sketch(st.d, 8)
    for lo, hi in [(0, 170), (170, 555), (555, 800)]:
        sub = st.rows(lo, hi)
        a.append_csr(*_dev(sub))
        b.append_csr(*_dev(sub))
        q1 = a.sketch().clone()
        q2 = a.sketch()
        assert torch.equal(q1, q2)
    assert torch.equal(a.sketch(), b.sketch())
    o = _oracle(st, 8)
    assert evaluate.gram_distance(a.sketch().cpu().numpy().astype(np.float64), o.sketch()) <= TOL


def test_exact_when_rows_at_most_ell(gpu_lib):
    st = small_random_csr(9, 50, 6, 7)
    _, B = _gpu_sketch(gpu_lib, st, 12)
    A = st.to_scipy().toarray()
    G = A.T @ A
    assert np.linalg.norm(B.T @ B - G) <= TOL * np.linalg.norm(G)


def test_empty_stream_and_empty_rows(gpu_lib):
    torch = _torch()
    sk = gpu_lib.Sketch(40, 6)
    assert torch.count_nonzero(sk.sketch()) == 0
    st = small_random_csr(300, 40, 4, 8, empty_rate=0.3)
    o = _oracle(st, 6)
    _, B = _gpu_sketch(gpu_lib, st, 6)
    _parity(B, o.sketch())


@pytest.mark.parametrize("n,d,ell,lam,seed", [(1500, 2000, 50, 20, 12), (2500, 3000, 100, 25, 13)])
def test_empty_rows_and_columns_on_wide_panels(gpu_lib, n, d, ell, lam, seed):
    # 64- and 128-wide panels, a third of the rows empty and many columns never entered: the
    # products write zero rows for the empty chunks of both directions (their first gather block
    # runs whatever the chunk's length and adds zeros)
    st = small_random_csr(n, d, lam, seed, empty_rate=0.3)
    assert (np.diff(st.indptr) == 0).any() and len(np.unique(st.indices)) < d
    o = _oracle(st, ell)
    _, B = _gpu_sketch(gpu_lib, st, ell)
    _parity(B, o.sketch())


def test_duplicate_column_ids(gpu_lib):
    st = small_random_csr(400, 50, 5, 9, dup_rate=0.25)
    o = _oracle(st, 7)
    _, B = _gpu_sketch(gpu_lib, st, 7)
    _parity(B, o.sketch())


def test_verify_off_matches_oracle(gpu_lib):
    st = small_random_csr(500, 60, 6, 10)
    o = _oracle(st, 9, verify=False)
    sk, B = _gpu_sketch(gpu_lib, st, 9, verify=False)
    assert sk.stats()["vs_calls"] == 0
    _parity(B, o.sketch())


def test_merge_matches_oracle(gpu_lib):
    st = small_random_csr(900, 60, 6, 11)
    shards = [(0, 300), (300, 640), (640, 900)]
    gs, os_ = [], []
    for k, (lo, hi) in enumerate(shards):
        sub = st.rows(lo, hi)
        g = gpu_lib.Sketch(st.d, 10, stream_id=k)
        g.append_csr(*_dev(sub))
        gs.append(g)
        o = SFDOracle(st.d, 10, 0.25, 0, stream_id=k, unit_roundoff=U32)
        o.append_csr(sub.indptr, sub.indices, sub.values)
        os_.append(o)
    gs[0].merge(gs[1])
    gs[0].merge(gs[2])
    os_[0].merge(os_[1])
    os_[0].merge(os_[2])
    B = gs[0].sketch().cpu().numpy().astype(np.float64)
    _parity(B, os_[0].sketch())
    with pytest.raises(gpu_lib.SfdError):
        gs[0].merge(gpu_lib.Sketch(61, 10))


def test_errors_leave_state_unchanged(gpu_lib):
    torch = _torch()
    sk = gpu_lib.Sketch(30, 4)
    st = small_random_csr(50, 30, 4, 12)
    sk.append_csr(*_dev(st))
    before = sk.sketch().clone()
    s0 = sk.stats()
    bad_idx = torch.tensor([0, 2], dtype=torch.int64, device="cuda")
    with pytest.raises(gpu_lib.SfdError) as e:
        sk.append_csr(bad_idx, torch.tensor([1, 30], dtype=torch.int32, device="cuda"),
                      torch.ones(2, dtype=torch.float32, device="cuda"))
    assert e.value.code == gpu_lib.SFD_E_INDEX
    with pytest.raises(gpu_lib.SfdError) as e:
        sk.append_csr(torch.tensor([0, 2, 1], dtype=torch.int64, device="cuda"),
                      torch.tensor([1, 2], dtype=torch.int32, device="cuda"),
                      torch.ones(2, dtype=torch.float32, device="cuda"))
    assert e.value.code == gpu_lib.SFD_E_ARG
    assert sk.stats() == s0
    assert torch.equal(sk.sketch(), before)
    with pytest.raises(gpu_lib.SfdError):
        gpu_lib.Sketch(10, 11)


@pytest.mark.parametrize("n,d,ell,seed", [(300, 60, 8, 0), (1000, 200, 20, 1), (700, 150, 50, 2), (1000, 400, 100, 3),
                                          (1000, 500, 200, 4)])
def test_fd_mode_matches_fd_oracle(gpu_lib, n, d, ell, seed):
    # FrequentDirections (Sec. 2.1) in batches of ell rows through the same DenseShrink kernels
    from oracle import FDBatchOracle

    st = small_random_csr(n, d, 6, seed, dist="lognormal")
    o = FDBatchOracle(d, ell)
    o.append_csr(st.indptr, st.indices, st.values)
    sk, B = _gpu_sketch(gpu_lib, st, ell, algorithm="fd")
    assert sk.stats()["flushes"] == o.flushes == n // ell
    assert sk.stats()["vs_calls"] == 0
    _parity(B, o.sketch())
    A = st.to_scipy()
    lmin, lmax = evaluate.cov_extremes(A, B)
    assert lmin >= -1e-5 * evaluate.fro2(A)
    assert lmax <= evaluate.fd_bound(A, ell, ell // 2) * (1 + 1e-4)


def test_sharded_merge_tree_matches_oracle(gpu_lib):
    # the multi-GPU design on one GPU: shards sketched independently, then a merge tree
    # (mergeability, Sec. 2.1); parity against the oracle run with the same sharding and tree
    st = small_random_csr(2400, 120, 10, 21, dist="lognormal")
    bounds = [0, 500, 1300, 1750, 2400]
    gs, os_ = [], []
    for k in range(4):
        sub = st.rows(bounds[k], bounds[k + 1])
        g = gpu_lib.Sketch(st.d, 16, stream_id=k)
        g.append_csr(*_dev(sub))
        gs.append(g)
        o = SFDOracle(st.d, 16, 0.25, 0, stream_id=k, unit_roundoff=U32)
        o.append_csr(sub.indptr, sub.indices, sub.values)
        os_.append(o)
    for a, b in [(0, 1), (2, 3), (0, 2)]:
        gs[a].merge(gs[b])
        os_[a].merge(os_[b])
    B = gs[0].sketch().cpu().numpy().astype(np.float64)
    _parity(B, os_[0].sketch())
    lmin, _ = evaluate.cov_extremes(st.to_scipy(), B)
    assert lmin >= -1e-5 * evaluate.fro2(st.to_scipy())


@pytest.mark.parametrize("n,d,ell,lam,seed", [
    (2500, 400, 100, 25, 6),  # ell = 100: 128-wide panels, 200 x 200 DenseShrink eigensolve
    (1800, 300, 65, 30, 7),   # ell = 65: the smallest ell on 128-wide panels, ragged tail
])
def test_wide_panel_streams_match_oracle(gpu_lib, n, d, ell, lam, seed):
    st = small_random_csr(n, d, lam, seed, dist="lognormal", dup_rate=0.02)
    o = _oracle(st, ell)
    sk, B = _gpu_sketch(gpu_lib, st, ell)
    assert sk.stats()["flushes"] == o.flushes >= 4
    _parity(B, o.sketch())
    assert sk.last_live == o.query()[1]


def test_wide_panel_large_buffer_matches_oracle(gpu_lib):
    # one 3,000-row buffer at ell = 100 with Zipf-long CSC columns, then a pending tail
    st = small_random_csr(4000, 3000, 40, 8, dist="lognormal")
    o = _oracle(st, 100)
    sk, B = _gpu_sketch(gpu_lib, st, 100)
    assert sk.stats()["flushes"] == o.flushes == 1
    _parity(B, o.sketch())


@pytest.mark.parametrize("n,d,ell,lam,seed", [
    (2000, 600, 150, 40, 9),    # 256-wide panels; two-pass Cholesky; 300 x 300 eigensolve (tridiagonal)
    (2400, 700, 200, 40, 10),   # ell = 200: 200 x 200 Jacobi with logged rotations, 400 x 400 tridiagonal
    (1800, 520, 256, 50, 11),   # the widest: both eigensolves tridiagonal (256 and 512)
])
def test_widest_panel_streams_match_oracle(gpu_lib, n, d, ell, lam, seed):
    st = small_random_csr(n, d, lam, seed, dist="lognormal", dup_rate=0.02 if ell == 150 else 0.0)
    o = _oracle(st, ell)
    sk, B = _gpu_sketch(gpu_lib, st, ell)
    assert sk.stats()["flushes"] == o.flushes == 3
    _parity(B, o.sketch())
    assert sk.last_live == o.query()[1]


def test_widest_panels_exact_buffers_and_ell_equal_d(gpu_lib):
    # ell = d = 200: every buffer (rows = d = ell) is kept exactly (dense rows on 256-wide
    # panels), the first fold is lossless and the later ones shrink a 400 x 400 stack
    st = small_random_csr(600, 200, 12, 12, dist="lognormal")
    o = _oracle(st, 200)
    sk, B = _gpu_sketch(gpu_lib, st, 200)
    assert sk.stats()["flushes"] == o.flushes == 3
    _parity(B, o.sketch())


def test_widest_panels_merge_and_verify_off(gpu_lib):
    # ell = 180 without VerifySpectral, sketched in two shards and merged (Sec. 2.1)
    st = small_random_csr(1800, 500, 30, 13, dist="lognormal")
    shards = [(0, 1100), (1100, 1800)]
    gs, os_ = [], []
    for k, (lo, hi) in enumerate(shards):
        sub = st.rows(lo, hi)
        g = gpu_lib.Sketch(st.d, 180, stream_id=k, verify=0)
        g.append_csr(*_dev(sub))
        gs.append(g)
        o = SFDOracle(st.d, 180, 0.25, 0, stream_id=k, unit_roundoff=U32, verify=False)
        o.append_csr(sub.indptr, sub.indices, sub.values)
        os_.append(o)
    gs[0].merge(gs[1])
    os_[0].merge(os_[1])
    B = gs[0].sketch().cpu().numpy().astype(np.float64)
    _parity(B, os_[0].sketch())
    assert gs[0].stats()["vs_calls"] == 0

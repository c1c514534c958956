"""BoostedSparseShrink's retry loop (Alg 4) on the GPU, through the C ABI.

The library's test hook SFD_OPT_TEST_ZERO_ROW zeroes row 0 of the start block G of
SimultaneousIteration (Alg 1) in each buffer's first attempt.  On the spiked stream every
buffer's dominant direction is e_0, which such a block never reaches, so VerifySpectral (Alg 6,
Lemma 3.1) rejects the first SparseShrink and the loop draws the next attempt's block.  The
oracle mirrors the hook (tests/planted.py, pinned on the CPU in test_oracle_stream.py).  q = 2 on
both sides: with many more steps the oracle's Householder QR would regrow e_0 from rounding noise,
while the GPU's CholeskyQR keeps the zero row exactly zero.

Checked: the attempt log (rejected, then accepted, per buffer), the persistent VerifySpectral
counter, the log-norms of both attempts, the sketch against the oracle's (relative Frobenius of
B^T B <= 1e-4 and every sigma_i^2), SFD_E_NOCONVERGE with the handle restored, and the batched
form's retry branch.
"""

import numpy as np
import pytest

from oracle import evaluate
from tests.parity import assert_sigma2_close
from tests.planted import ZeroRowOracle
from workloads import spiked_stream

pytestmark = pytest.mark.gpu

TOL = 1e-4
U32 = 2.0 ** -24
D, ELL, Q = 40, 8, 2


def _dev(st):
    import torch

    return tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (st.indptr, st.indices, st.values))


def _sketch(sfd, **kw):
    sk = sfd.Sketch(D, ELL, 0.25, 0, q=Q, **kw)
    sk.set_option(sfd.OPT_TEST_ZERO_ROW, 0)
    return sk


def _oracle(st, **kw):
    o = ZeroRowOracle(D, ELL, 0.25, 0, q=Q, unit_roundoff=U32, **kw)
    o.append_csr(st.indptr, st.indices, st.values)
    return o


def _np(B):
    return B.cpu().numpy().astype(np.float64)


def test_rejected_first_attempts_are_retried_like_the_oracle(gpu_lib):
    st = spiked_stream(100, D, 0)
    o = _oracle(st)
    sk = _sketch(gpu_lib)
    sk.append_csr(*_dev(st))
    s = sk.stats()
    att = [r for b in o.log for r in b["attempts"]]
    assert s["flushes"] == o.flushes == 2
    assert s["attempts"] == len(att) == 4
    assert s["vs_rejects"] == sum(not r["accepted"] for r in att) == 2
    assert s["vs_calls"] == o.vs_calls == 4
    # the last VerifySpectral call of the appends: buffer 1's accepted second attempt
    assert s["last_t"] == att[-1]["t"]
    assert abs(s["last_ln_norm"] - att[-1]["ln_norm"]) <= 1e-3 * abs(att[-1]["ln_norm"])
    # the query folds the pending 20 rows with the same reject-then-retry (purposes 2/3, counter 5, 6)
    B = _np(sk.sketch())
    rec = []
    Bo, live, calls = o.query(log=rec)
    assert [r["accepted"] for r in rec] == [False, True] and calls == 2
    s2 = sk.stats()
    assert s2["vs_rejects"] == 3 and s2["attempts"] == 6
    assert abs(s2["last_ln_norm"] - rec[-1]["ln_norm"]) <= 1e-3 * abs(rec[-1]["ln_norm"])
    assert evaluate.gram_distance(B, Bo) <= TOL
    assert_sigma2_close(B, Bo)
    assert sk.last_live == live


def test_exhausted_attempts_restore_the_handle(gpu_lib):
    # max_attempts = 1: the first flush's only attempt is rejected -> SFD_E_NOCONVERGE, and the
    # handle is as before the call (the stats' last_* figures give the rejected attempt)
    import torch

    st = spiked_stream(100, D, 0)
    o = _oracle(st)
    ref = _sketch(gpu_lib)
    ref.append_csr(*_dev(st))
    B_ref = ref.sketch()
    sk = _sketch(gpu_lib, max_attempts=1)
    pre = st.rows(0, 7)  # pending rows before the failing append
    sk.append_csr(*_dev(pre))
    s0 = sk.stats()
    B0 = sk.sketch().clone()
    rest = st.rows(7, 100)
    with pytest.raises(gpu_lib.SfdError) as e:
        sk.append_csr(*_dev(rest))
    assert e.value.code == gpu_lib.SFD_E_NOCONVERGE
    s1 = sk.stats()
    first = o.log[0]["attempts"][0]
    assert not first["accepted"]
    assert s1["last_t"] == first["t"]
    assert abs(s1["last_ln_norm"] - first["ln_norm"]) <= 1e-3 * abs(first["ln_norm"])
    for k in ("rows_seen", "nnz_seen", "flushes", "vs_calls", "attempts", "vs_rejects", "live_rows", "pending_rows",
              "pending_nnz"):
        assert s1[k] == s0[k], k
    # not an error state: queries and appends go on; the restored handle finishes exactly like one
    # that never failed (same kernels, same draws)
    assert torch.equal(sk.sketch(), B0)
    sk.set_option(gpu_lib.OPT_MAX_ATTEMPTS, 16)
    sk.append_csr(*_dev(rest))
    assert torch.equal(sk.sketch(), B_ref)
    assert sk.stats()["flushes"] == 2


def _concat(*parts):
    from workloads import CsrStream

    ptr = [np.zeros(1, np.int64)]
    base = 0
    for x in parts:
        ptr.append(x.indptr[1:] - x.indptr[0] + base)
        base += x.nnz
    return CsrStream(np.concatenate(ptr), np.concatenate([x.indices for x in parts]),
                     np.concatenate([x.values for x in parts]), parts[0].d, dict(name="concat"))


def test_exhausted_attempts_restore_pending_rows_of_a_host_block(gpu_lib):
    # a host block stages each full buffer through the pending buffer, so its second flush
    # overwrites the rows pending before the call: here the first flush (rows 0-39, no energy in
    # column 0) is accepted and folded into B, the second (rows 40-79, spiked) rejects every
    # attempt; B and the 5 pending rows are both restored
    import torch

    st = _concat(spiked_stream(40, D, 1, spike=0.0), spiked_stream(60, D, 2))
    ref = _sketch(gpu_lib)
    ref.append_csr(*_dev(st))
    B_ref = ref.sketch()
    sk = _sketch(gpu_lib)
    pre, rest = st.rows(0, 5), st.rows(5, 100)
    sk.append_csr(pre.indptr, pre.indices, pre.values)
    B0 = sk.sketch().clone()
    sk.set_option(gpu_lib.OPT_TEST_ZERO_ATTEMPTS, 16)  # every attempt planted: the loop gives up
    with pytest.raises(gpu_lib.SfdError) as e:
        sk.append_csr(rest.indptr, rest.indices, rest.values)
    assert e.value.code == gpu_lib.SFD_E_NOCONVERGE
    s = sk.stats()
    assert s["pending_rows"] == 5 and s["flushes"] == 0 and s["rows_seen"] == 5
    assert torch.equal(sk.sketch(), B0)
    sk.set_option(gpu_lib.OPT_TEST_ZERO_ATTEMPTS, 1)
    sk.append_csr(rest.indptr, rest.indices, rest.values)
    assert sk.stats()["flushes"] == 2
    assert torch.equal(sk.sketch(), B_ref)


def test_query_that_exhausts_its_attempts_changes_nothing(gpu_lib):
    import torch

    st = spiked_stream(30, D, 2)  # 30 rows < d: nothing flushes, the query folds m = 30 > ell rows
    sk = _sketch(gpu_lib, max_attempts=1)
    sk.append_csr(*_dev(st))
    s0 = sk.stats()
    with pytest.raises(gpu_lib.SfdError) as e:
        sk.sketch()
    assert e.value.code == gpu_lib.SFD_E_NOCONVERGE
    assert {k: v for k, v in sk.stats().items() if not k.startswith("last_")} == \
        {k: v for k, v in s0.items() if not k.startswith("last_")}
    sk.set_option(gpu_lib.OPT_MAX_ATTEMPTS, 2)
    B = sk.sketch()
    o = _oracle(st)
    rec = []
    Bo, _, _ = o.query(log=rec)
    assert [r["accepted"] for r in rec] == [False, True]
    assert evaluate.gram_distance(_np(B), Bo) <= TOL
    assert torch.equal(sk.sketch(), B)


def test_batched_retry_branch_matches_single_handles_and_the_oracle(gpu_lib):
    # three streams whose buffers all reject their first attempt: the lockstep group's verdict
    # marks them rejected and each retries on a lane (attempt 1, VerifySpectral counter + 1)
    import torch

    sts = [spiked_stream(100 + 10 * s, D, 10 + s) for s in range(3)]
    ptr = np.zeros(1 + sum(x.n for x in sts), dtype=np.int64)
    starts = np.zeros(4, dtype=np.int64)
    pos, base = 1, 0
    for i, x in enumerate(sts):
        ptr[pos:pos + x.n] = x.indptr[1:] + base
        pos += x.n
        base += x.nnz
        starts[i + 1] = starts[i] + x.n
    idx = np.concatenate([x.indices for x in sts])
    val = np.concatenate([x.values for x in sts])
    bat = gpu_lib.Batch(3, D, ELL)
    bat.set_option(gpu_lib.OPT_Q, Q)
    bat.set_option(gpu_lib.OPT_TEST_ZERO_ROW, 0)
    g = [torch.from_numpy(a).cuda() for a in (ptr, idx, val)]
    bat.append_csr(np.arange(3, dtype=np.int32), starts, *g)
    Bb = bat.sketch()
    for s, x in enumerate(sts):
        one = _sketch(gpu_lib, stream_id=s)
        one.append_csr(*_dev(x))
        assert torch.equal(one.sketch(), Bb[s])
        o = ZeroRowOracle(D, ELL, 0.25, 0, stream_id=s, q=Q, unit_roundoff=U32)
        o.append_csr(x.indptr, x.indices, x.values)
        st_b = bat.stats(s)
        rec = []
        o.query(log=rec)
        rejects = sum(not r["accepted"] for b in o.log for r in b["attempts"]) + sum(not r["accepted"] for r in rec)
        assert st_b["flushes"] == o.flushes >= 2
        # a query's VerifySpectral calls are not kept in the persistent counter (its rejects are counted)
        assert st_b["vs_calls"] == o.vs_calls and st_b["vs_rejects"] == rejects
        Bo = o.sketch()
        assert evaluate.gram_distance(_np(Bb[s]), Bo) <= TOL
        assert_sigma2_close(_np(Bb[s]), Bo)
    # every attempt planted: the batch reports SFD_E_NOCONVERGE and stays in its error state
    bat.reset()
    bat.set_option(gpu_lib.OPT_MAX_ATTEMPTS, 1)
    with pytest.raises(gpu_lib.SfdError) as e:
        bat.append_csr(np.arange(3, dtype=np.int32), starts, *g)
    assert e.value.code == gpu_lib.SFD_E_NOCONVERGE
    with pytest.raises(gpu_lib.SfdError) as e:
        bat.sketch()
    assert e.value.code == gpu_lib.SFD_E_STATE
    bat.reset()
    bat.set_option(gpu_lib.OPT_MAX_ATTEMPTS, 16)
    bat.append_csr(np.arange(3, dtype=np.int32), starts, *g)
    assert torch.equal(bat.sketch(), Bb)

"""Pins of the stream drivers: SparseFrequentDirections (Alg 2) and FrequentDirections (Sec. 2.1).

Pins: the FrequentDirections guarantee (Lemma 2.1 with alpha = 1), Theorem 3.1 for k < alpha ell,
Property 1 of the whole stream, exactness for n <= ell, a brute-force second oracle in d x d
covariance space, the flush rule on hand-computed streams, invariances, and mutation tests
that plant plausible mistakes in the oracle and check a pin catches each.
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle.shrink as osh
import oracle.stream as ost
from oracle import FDBatchOracle, FDOracle, SFDOracle, evaluate
from oracle.rng import PURPOSE_SI, PURPOSE_VS, sphere_vector, start_block
from oracle.shrink import ALPHA, si_iterations, vs_steps
from workloads import stream_1e4_d1e3, small_random_csr

pytestmark = pytest.mark.cpu


def _run_sfd(st, ell, **kw):
    o = SFDOracle(st.d, ell, kw.pop("eps", 0.25), kw.pop("seed", 0), **kw)
    o.append_csr(st.indptr, st.indices, st.values)
    return o


# ---------------------------------------------------------------------------- flush rule (Alg 2)
def _flush_sizes(indptr, d, ell):
    o = SFDOracle(d, ell, 0.25, 0)
    sizes = []
    orig = o._flush

    def spy():
        sizes.append(o.buf_rows)
        orig()

    o._flush = spy
    idx = np.concatenate([np.arange(k) % d for k in np.diff(indptr)]).astype(np.int32)
    o.append_csr(indptr, idx, np.ones(len(idx), np.float32))
    return sizes, o.buf_rows


def test_flush_rule_hand_computed():
    d, ell = 10, 2  # ell * d = 20
    # rows of 7 entries: 7, 14, 21 >= 20 -> flush after 3 rows
    sizes, pend = _flush_sizes(np.arange(8, dtype=np.int64) * 7, d, ell)
    assert sizes == [3, 3] and pend == 1
    # rows of 5 entries: 20 >= 20 reaches the budget exactly at row 4
    sizes, pend = _flush_sizes(np.arange(9, dtype=np.int64) * 5, d, ell)
    assert sizes == [4, 4] and pend == 0
    # rows of 1 entry: the rows(A') = d rule fires at 10 rows
    sizes, pend = _flush_sizes(np.arange(25, dtype=np.int64), d, ell)
    assert sizes == [10, 10] and pend == 4
    # empty rows count as rows
    sizes, pend = _flush_sizes(np.zeros(12, dtype=np.int64), d, ell)
    assert sizes == [10] and pend == 1


def test_flush_rule_independent_of_block_boundaries():
    st = small_random_csr(300, 40, 6, 3)
    whole = _run_sfd(st, 5)
    parts = SFDOracle(st.d, 5, 0.25, 0)
    for lo, hi in [(0, 1), (1, 50), (50, 51), (51, 200), (200, 300)]:
        sub = st.rows(lo, hi)
        parts.append_csr(sub.indptr, sub.indices, sub.values)
    assert [r["rows"] for r in parts.log] == [r["rows"] for r in whole.log]
    np.testing.assert_array_equal(parts.sketch(), whole.sketch())


# ---------------------------------------------------------------------------- FrequentDirections
@pytest.mark.parametrize("seed", [0, 1])
def test_fd_guarantee(seed):
    st = small_random_csr(200, 30, 5, seed)
    A = st.to_scipy()
    f = FDOracle(st.d, 8)
    f.append_csr(st.indptr, st.indices, st.values)
    B = f.sketch()
    lmin, lmax = evaluate.cov_extremes(A, B)
    assert lmin >= -1e-9 * evaluate.fro2(A)
    for k in range(8):
        assert lmax <= evaluate.fd_bound(A, 8, k) * (1 + 1e-9)


def test_fd_merge_guarantee():
    st = small_random_csr(300, 25, 5, 7)
    A = st.to_scipy()
    Bs = []
    for lo, hi in [(0, 100), (100, 200), (200, 300)]:
        f = FDOracle(st.d, 6)
        sub = st.rows(lo, hi)
        f.append_csr(sub.indptr, sub.indices, sub.values)
        Bs.append(f.sketch())
    f = FDOracle(st.d, 6)
    f.append_dense(np.vstack(Bs))
    B = f.sketch()
    _, lmax = evaluate.cov_extremes(A, B)
    for k in range(6):
        assert lmax <= evaluate.fd_bound(A, 6, k) * (1 + 1e-9)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fd_batch_guarantee(seed):
    # FD in batches of ell rows keeps Lemma 2.1's bound and B^T B <= A^T A
    st = small_random_csr(260, 30, 6, 10 + seed, dist="lognormal")
    A = st.to_scipy()
    f = FDBatchOracle(st.d, 8)
    f.append_csr(st.indptr, st.indices, st.values)
    assert f.flushes == 260 // 8
    assert all(r["attempts"] == [] for r in f.log)  # every flush is an exact fold
    B = f.sketch()
    lmin, lmax = evaluate.cov_extremes(A, B)
    assert lmin >= -1e-9 * evaluate.fro2(A)
    for k in range(8):
        assert lmax <= evaluate.fd_bound(A, 8, k) * (1 + 1e-9)


def test_fd_batch_agrees_with_row_at_a_time_fd_up_to_the_first_shrink():
    ell = 7
    st = small_random_csr(2 * ell, 40, 6, 3, dist="lognormal")
    fb = FDBatchOracle(st.d, ell)
    fb.append_csr(st.indptr, st.indices, st.values)
    f1 = FDOracle(st.d, ell)
    f1.append_csr(st.indptr, st.indices, st.values)
    B1, B2 = fb.sketch(), f1.sketch()
    np.testing.assert_allclose(B1.T @ B1, B2.T @ B2, atol=1e-9 * np.abs(B2.T @ B2).max())
    # and B^T B = A^T A while n <= ell
    sub = st.rows(0, ell)
    fe = FDBatchOracle(st.d, ell)
    fe.append_csr(sub.indptr, sub.indices, sub.values)
    A = sub.to_scipy().toarray()
    Be = fe.sketch()
    np.testing.assert_allclose(Be.T @ Be, A.T @ A, atol=1e-9 * np.abs(A.T @ A).max())


# ---------------------------------------------------------------------------- SparseFrequentDirections
def test_sfd_exact_when_n_at_most_ell():
    st = small_random_csr(7, 40, 5, 2)
    o = _run_sfd(st, 8)
    B = o.sketch()
    A = st.to_scipy().toarray()
    np.testing.assert_allclose(B.T @ B, A.T @ A, atol=1e-12 * np.abs(A.T @ A).max())


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sfd_property1_and_theorem(seed):
    """lambda_min(A^T A - B^T B) >= 0 always; ||A^T A - B^T B|| <= ||A - A_k||^2 / (alpha ell - k)
    for k < alpha ell (Theorem 3.1, which holds with probability 1 - delta: asserted on these seeds)."""
    st = small_random_csr(1500, 60, 8, seed, dist="lognormal")
    ell = 21  # alpha ell = 3.07
    o = _run_sfd(st, ell)
    assert o.flushes >= 5
    A = st.to_scipy()
    B = o.sketch()
    lmin, lmax = evaluate.cov_extremes(A, B)
    assert lmin >= -1e-9 * evaluate.fro2(A)
    for k in range(int(math.ceil(ALPHA * ell))):
        assert lmax <= evaluate.sfd_bound(A, ell, k)


def test_sfd_meets_fd_bound_on_the_1e4_row_stream():
    """The empirical target: SFD's covariance error under FrequentDirections' bound (k = 10)."""
    st = stream_1e4_d1e3()
    o = _run_sfd(st, 20)
    A = st.to_scipy()
    B = o.sketch()
    assert evaluate.cov_err(A, B) <= evaluate.fd_bound(A, 20, 10) / evaluate.fro2(A)
    assert o.flushes == 10 and all(len(r["attempts"]) == 1 for r in o.log)


def _brute_force_cov(st, ell, eps=0.25, seed=0, delta=0.01, q=None):
    """Second oracle in d x d covariance space: tracks M_B = B^T B only.

    Buffer: M_P = A'^T Pi_Y A' with Y = A' (A'^T A')^q G formed directly, B'^T B' = (M_P - lam_ell^2 I)_+;
    VerifySpectral from C = (A'^T A' - B'^T B') / (Delta/2) raised to the t-th power directly;
    DenseShrink: (M_B + M_B' - mu_ell I)_+ unless at most ell rows are live.
    """
    d = st.d
    A = st.to_scipy().toarray()
    MB = np.zeros((d, d))
    live = 0
    rows = []
    nnz = 0
    b = 0
    i = 0

    def psd(M):
        w, V = np.linalg.eigh((M + M.T) / 2)
        return (V * np.maximum(w, 0)) @ V.T, w[::-1]

    def fold(rows_, MB, live, purpose_g, purpose_x, i):
        Ab = A[rows_]
        m = len(rows_)
        if m <= ell:
            MR, radd = Ab.T @ Ab, m
        else:
            qq = q if q is not None else si_iterations(m, eps)
            for a in range(16):
                G = start_block(seed, 0, b, a, purpose_g, d, ell)
                Y = Ab @ np.linalg.matrix_power(Ab.T @ Ab, qq) @ G
                MP = Ab.T @ (Y @ np.linalg.pinv(Y)) @ Ab
                w = np.linalg.eigvalsh(MP)[::-1]
                MR, _ = psd(MP - w[ell - 1] * np.eye(d))
                S = np.trace(Ab.T @ Ab) - np.trace(MR)
                if S <= 64 * 2.0**-53 * ell * np.trace(Ab.T @ Ab):
                    break
                i += 1
                C = (Ab.T @ Ab - MR) / (S / (ALPHA * ell) / 2)
                x = sphere_vector(seed, 0, b, a, purpose_x, d)
                if np.linalg.norm(np.linalg.matrix_power(C, vs_steps(d, delta, i)) @ x) <= 1:
                    break
            radd = ell - 1
        tot = live + radd
        if tot <= ell:
            return MB + MR, tot, i
        _, mu = psd(MB + MR)
        MB2, _ = psd(MB + MR - mu[ell - 1] * np.eye(d))
        return MB2, ell - 1, i

    for r in range(st.n):
        rows.append(r)
        nnz += int(st.indptr[r + 1] - st.indptr[r])
        if nnz >= ell * d or len(rows) == d:
            MB, live, i = fold(rows, MB, live, PURPOSE_SI, PURPOSE_VS, i)
            rows, nnz, b = [], 0, b + 1
    MB, live, _ = fold(rows, MB, live, 2, 3, i)
    return MB


@pytest.mark.parametrize("n,d,ell,lam,q,seed", [(40, 8, 3, 2, 1, 0), (35, 6, 4, 3, 2, 1), (30, 8, 2, 1, 3, 2),
                                                 (23, 5, 4, 4, 2, 3)])
def test_sfd_matches_brute_force_covariance_oracle(n, d, ell, lam, q, seed):
    st = small_random_csr(n, d, lam, seed)
    o = _run_sfd(st, ell, q=q)
    B = o.sketch()
    MB = _brute_force_cov(st, ell, q=q)
    assert o.flushes >= 2
    np.testing.assert_allclose(B.T @ B, MB, atol=1e-7 * max(1.0, np.abs(MB).max()))


def test_query_is_non_destructive():
    st = small_random_csr(500, 40, 5, 4)
    a = SFDOracle(st.d, 6, 0.25, 1)
    b = SFDOracle(st.d, 6, 0.25, 1)
    for lo, hi in [(0, 130), (130, 377), (377, 500)]:
        sub = st.rows(lo, hi)
        a.append_csr(sub.indptr, sub.indices, sub.values)
        b.append_csr(sub.indptr, sub.indices, sub.values)
        q1 = a.sketch()
        q2 = a.sketch()
        np.testing.assert_array_equal(q1, q2)
    np.testing.assert_array_equal(a.sketch(), b.sketch())
    assert a.vs_calls == b.vs_calls and a.flushes == b.flushes


def test_within_buffer_row_permutation_invariance():
    st = small_random_csr(200, 50, 5, 8)  # d = 50 rows per buffer (nnz budget not reached)
    perm = np.concatenate([np.random.default_rng(0).permutation(50) + 50 * k for k in range(4)])
    lens = np.diff(st.indptr)
    idx = [st.indices[st.indptr[r]:st.indptr[r + 1]] for r in perm]
    val = [st.values[st.indptr[r]:st.indptr[r + 1]] for r in perm]
    indptr = np.zeros(201, np.int64)
    np.cumsum(lens[perm], out=indptr[1:])
    o1 = _run_sfd(st, 6)
    o2 = SFDOracle(50, 6, 0.25, 0)
    o2.append_csr(indptr, np.concatenate(idx), np.concatenate(val))
    assert [r["rows"] for r in o1.log] == [50] * 4
    assert evaluate.gram_distance(o1.sketch(), o2.sketch()) < 1e-9


def test_scale_equivariance():
    st = small_random_csr(300, 30, 5, 9)
    o1 = _run_sfd(st, 5)
    st2 = small_random_csr(300, 30, 5, 9)
    st2.values = (st2.values * 8.0).astype(np.float32)
    o2 = _run_sfd(st2, 5)
    assert evaluate.gram_distance(o2.sketch(), 8.0 * o1.sketch()) < 1e-10


def test_merge_obeys_guarantee_and_checks_shapes():
    st = small_random_csr(900, 40, 6, 10, dist="lognormal")
    A = st.to_scipy()
    ell = 21
    shards = []
    for k, (lo, hi) in enumerate([(0, 300), (300, 650), (650, 900)]):
        o = SFDOracle(st.d, ell, 0.25, 0, stream_id=k)
        sub = st.rows(lo, hi)
        o.append_csr(sub.indptr, sub.indices, sub.values)
        shards.append(o)
    src_before = shards[1].sketch()
    shards[0].merge(shards[1])
    shards[0].merge(shards[2])
    np.testing.assert_array_equal(shards[1].sketch(), src_before)
    B = shards[0].sketch()
    lmin, lmax = evaluate.cov_extremes(A, B)
    assert lmin >= -1e-9 * evaluate.fro2(A)
    for k in range(3):
        assert lmax <= evaluate.sfd_bound(A, ell, k)
    with pytest.raises(ValueError):
        shards[0].merge(SFDOracle(41, ell, 0.25, 0))


def test_rejects_bad_input_without_state_change():
    o = SFDOracle(10, 3, 0.25, 0)
    o.append_csr(np.array([0, 2]), np.array([1, 2], np.int32), np.ones(2, np.float32))
    with pytest.raises(IndexError):
        o.append_csr(np.array([0, 1, 2]), np.array([3, 10], np.int32), np.ones(2, np.float32))
    with pytest.raises(ValueError):
        o.append_csr(np.array([0, 2, 1]), np.array([3, 4], np.int32), np.ones(2, np.float32))
    assert o.buf_rows == 1 and o.buf_nnz == 2
    with pytest.raises(ValueError):
        SFDOracle(10, 11, 0.25, 0)


def test_duplicate_column_ids_are_summed():
    st = small_random_csr(120, 20, 4, 11, dup_rate=0.3)
    assert np.sum(np.diff(st.indices) == 0) > 10
    o = _run_sfd(st, 4)
    A = st.to_scipy()
    B = o.sketch()
    lmin, _ = evaluate.cov_extremes(A, B)
    assert lmin >= -1e-9 * evaluate.fro2(A)


# ---------------------------------------------------------------------------- mutation tests
def _pins_hold():
    """A handful of the pins above, as one boolean (used with a planted mistake)."""
    try:
        test_dense_shrink_pin()
        test_sfd_matches_brute_force_covariance_oracle(40, 8, 3, 2, 1, 0)
        st = small_random_csr(400, 30, 5, 1)
        o = _run_sfd(st, 6)
        A = st.to_scipy()
        lmin, _ = evaluate.cov_extremes(A, o.sketch())
        assert lmin >= -1e-9 * evaluate.fro2(A)
        test_flush_rule_hand_computed()
        # VerifySpectral's log norm against C^t x formed directly
        Av = small_random_csr(30, 12, 4, 5).to_scipy()
        Bv = np.random.default_rng(1).standard_normal((3, 12)) * 0.1
        C = ((Av.T @ Av).toarray() - Bv.T @ Bv) / 0.7
        x = sphere_vector(1, 0, 0, 0, 1, 12)
        _, ln = osh.verify_spectral(Av, Bv, 0.7, x, 9)
        assert math.isclose(ln, math.log(np.linalg.norm(np.linalg.matrix_power(C, 9) @ x)), rel_tol=1e-10)
    except AssertionError:
        return False
    return True


def test_dense_shrink_pin():
    C = np.random.default_rng(5).standard_normal((10, 8))
    B, _ = ost.dense_shrink(C, 4, 10)
    mu = np.linalg.eigvalsh(C.T @ C)[::-1]
    w, V = np.linalg.eigh(C.T @ C - mu[3] * np.eye(8))
    np.testing.assert_allclose(B.T @ B, (V * np.maximum(w, 0)) @ V.T, atol=1e-9)


def test_pins_hold_on_the_real_oracle():
    assert _pins_hold()


@pytest.mark.parametrize("mutation", ["no_shift", "plus_shift", "wrong_pivot", "si_one_short", "vs_full_delta",
                                      "flush_strict"])
def test_planted_mistakes_are_caught(monkeypatch, mutation):
    if mutation == "no_shift":
        monkeypatch.setattr(osh, "shrink_factors", lambda s, ell: s[:ell])
    elif mutation == "plus_shift":
        monkeypatch.setattr(osh, "shrink_factors",
                            lambda s, ell: np.sqrt(s[:ell] ** 2 + (s[ell - 1] ** 2 if len(s) >= ell else 0)))
    elif mutation == "wrong_pivot":
        def wp(s, ell):
            s2 = s[:ell] ** 2
            piv = s[ell] ** 2 if len(s) > ell else 0.0
            return np.sqrt(np.maximum(s2 - piv, 0))
        monkeypatch.setattr(osh, "shrink_factors", wp)
    elif mutation == "si_one_short":
        real = osh.simultaneous_iteration
        monkeypatch.setattr(osh, "simultaneous_iteration", lambda A, G, q: real(A, G, max(q - 1, 0)))
    elif mutation == "vs_full_delta":
        real_vs = osh.verify_spectral
        monkeypatch.setattr(osh, "verify_spectral", lambda A, B, h, x, t: real_vs(A, B, 2 * h, x, t))
    elif mutation == "flush_strict":
        # flushes one row late when nnz(A') reaches ell*d exactly (">" instead of ">=")
        orig_flush = ost.SFDOracle._flush

        def flush_late(self):
            if self.buf_nnz == self.ell * self.d:
                return
            return orig_flush(self)

        monkeypatch.setattr(ost.SFDOracle, "_flush", flush_late)
    assert not _pins_hold()


def test_planted_start_block_makes_every_buffer_reject_then_retry():
    # the scenario of the GPU retry tests (Alg 4's loop), pinned on the oracle: on the spiked
    # stream every buffer's dominant direction is e_0; with row 0 of attempt 0's start block zeroed
    # (and q = 2, too few steps for rounding noise to regrow e_0) VerifySpectral rejects (Lemma 3.1:
    # ||C|| >= 2 here), the next attempt's Gaussian block sees e_0 and is accepted
    from oracle import NoConvergence
    from tests.planted import ZeroRowOracle
    from workloads import spiked_stream

    st = spiked_stream(100, 40, 0)
    o = ZeroRowOracle(40, 8, 0.25, 0, q=2, unit_roundoff=2.0 ** -24)
    o.append_csr(st.indptr, st.indices, st.values)
    assert o.flushes == 2
    for b in o.log:
        assert [r["accepted"] for r in b["attempts"]] == [False, True]
        assert b["attempts"][0]["ln_norm"] > 5.0 and b["attempts"][1]["ln_norm"] < -10.0
    assert [r["vs_index"] for b in o.log for r in b["attempts"]] == [1, 2, 3, 4]
    rec = []
    B, live, calls = o.query(log=rec)
    assert [r["accepted"] for r in rec] == [False, True] and calls == 2
    # the accepted sketch keeps Property 1 on the whole stream
    A = st.to_scipy()
    lmin, _ = evaluate.cov_extremes(A, B)
    assert lmin >= -1e-9 * evaluate.fro2(A)
    # every attempt planted: the loop gives up
    bad = ZeroRowOracle(40, 8, 0.25, 0, q=2, max_attempts=3, zero_attempts=3, unit_roundoff=2.0 ** -24)
    with pytest.raises(NoConvergence):
        bad.append_csr(st.indptr, st.indices, st.values)

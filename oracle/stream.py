"""Stream drivers: SparseFrequentDirections (Alg 2, Sec. 3) and FrequentDirections (Sec. 2.1).

SparseFrequentDirections keeps a sketch B (ell x d, initially 0) and a buffer A' of whole rows.
After each appended row it tests nnz(A') >= ell*d or rows(A') = d; when either holds it
replaces A' by B' = BoostedSparseShrink(A', ell, delta) and sets B = DenseShrink([B; B'], ell).

Readings where the paper is silent (also listed in the repository's design notes):
* nnz(A') counts stored entries (explicit zeros and repeated column ids included).
* A buffer of m <= ell rows is kept exactly instead of being shrunk (SparseShrink needs
  ell <= m); mid-stream flushes always have m > ell unless d rows are dense, so this only
  matters for queries and tiny inputs, and it makes B^T B = A^T A for n <= ell.
* Structural live-row counts decide whether DenseShrink shrinks: a stack with at most ell
  live rows is kept exactly (shrinking it would subtract a positive lambda_ell^2 for nothing).
  SparseShrink and a shrinking DenseShrink leave ell - 1 live rows; an exact buffer leaves m.
* Alg 2 returns B without the rows still in A'.  A query folds the pending buffer into a copy
  of the state (random draws from purposes 2/3, VerifySpectral counter continued from i + 1
  but not stored), so querying does not change the stream.
* merge(dst, src) (mergeability, Sec. 2.1): dst.B = DenseShrink([query(dst); query(src)]);
  dst's buffer is consumed and its flush index advances; src is unchanged.
"""

from __future__ import annotations

import copy

import numpy as np
import scipy.sparse as sp

from .rng import (
    PURPOSE_QUERY_SI,
    PURPOSE_QUERY_VS,
    PURPOSE_SI,
    PURPOSE_VS,
    sphere_vector,
    start_block,
)
from .shrink import boosted_sparse_shrink, dense_shrink, si_iterations


def _check_csr(indptr, indices, values, d):
    indptr = np.asarray(indptr, dtype=np.int64)
    indices = np.asarray(indices, dtype=np.int64)
    values = np.asarray(values)
    if indptr.ndim != 1 or len(indptr) < 1:
        raise ValueError("indptr must have nrows + 1 entries")
    if np.any(np.diff(indptr) < 0):
        raise ValueError("indptr must be non-decreasing")
    lo, hi = int(indptr[0]), int(indptr[-1])
    if lo < 0 or hi > len(indices) or hi > len(values):
        raise ValueError("indptr points outside indices/values")
    idx = indices[lo:hi]
    if idx.size and (idx.min() < 0 or idx.max() >= d):
        raise IndexError("column index out of range")
    if np.any(np.diff(indptr) > d):
        raise ValueError("a row stores more than d entries")
    return indptr, indices, values


class SFDOracle:
    """SparseFrequentDirections (Alg 2) over one row stream, FP64 throughout.

    Parameters mirror the library's create call and options: d, ell, eps (accuracy of
    SimultaneousIteration, 1/4 in SparseShrink), seed and stream_id (random key), delta
    (failure probability of Alg 2), q (override of the power count), max_attempts (cap on
    the BoostedSparseShrink loop), verify (False runs SparseShrink alone, as the paper's
    experiments do, Sec. 4) and unit_roundoff (precision of the lossless-accept test).
    """

    def __init__(self, d, ell, eps=0.25, seed=0, stream_id=0, *, delta=0.01, q=None,
                 max_attempts=16, verify=True, unit_roundoff=2.0 ** -53, flush_rows=None, flush_nnz=None):
        if not (1 <= ell <= d):
            raise ValueError("need 1 <= ell <= d")
        if not (0.0 < eps < 1.0):
            raise ValueError("need 0 < eps < 1")
        self.d, self.ell, self.eps = int(d), int(ell), float(eps)
        self.seed, self.stream_id = int(seed), int(stream_id)
        self.delta, self.q_override = float(delta), q
        self.max_attempts, self.verify, self.unit_roundoff = int(max_attempts), bool(verify), float(unit_roundoff)
        # Alg 2's flush rule: rows(A') = d or nnz(A') >= ell*d (overridable, see FDBatchOracle)
        self.flush_rows = int(flush_rows) if flush_rows is not None else self.d
        self.flush_nnz = flush_nnz if flush_nnz is not None else self.ell * self.d
        self.B = np.zeros((self.ell, self.d))
        self.live = 0          # structural count of rows of B that may be non-zero
        self.flushes = 0       # b: completed flushes (buffer index of the pending buffer)
        self.vs_calls = 0      # i: persistent VerifySpectral counter (Alg 6)
        self.log: list[dict] = []
        self._clear_buffer()

    # -- buffer --------------------------------------------------------------------------
    def _clear_buffer(self):
        self._rows_idx: list[np.ndarray] = []
        self._rows_val: list[np.ndarray] = []
        self.buf_nnz = 0

    @property
    def buf_rows(self) -> int:
        return len(self._rows_idx)

    def _buffer_matrix(self) -> sp.csr_matrix:
        m = self.buf_rows
        lens = np.array([len(r) for r in self._rows_idx], dtype=np.int64)
        indptr = np.zeros(m + 1, dtype=np.int64)
        np.cumsum(lens, out=indptr[1:])
        idx = np.concatenate(self._rows_idx) if m else np.zeros(0, np.int64)
        val = np.concatenate(self._rows_val) if m else np.zeros(0)
        return sp.csr_matrix((val.astype(np.float64), idx, indptr), shape=(m, self.d))

    def append_csr(self, indptr, indices, values):
        """Append rows given in CSR form (indptr[0] may be non-zero); Alg 2's row loop."""
        indptr, indices, values = _check_csr(indptr, indices, values, self.d)
        full = self.flush_nnz
        n = len(indptr) - 1
        r = 0
        while r < n:
            # the first row at which nnz(A') >= ell*d or rows(A') = d holds after appending it
            lens = np.diff(indptr[r:])
            cum = self.buf_nnz + np.cumsum(lens)
            by_nnz = int(np.searchsorted(cum, full, side="left"))
            by_rows = self.flush_rows - self.buf_rows - 1
            cut = min(by_nnz, by_rows)
            last = min(cut, n - r - 1)
            for k in range(r, r + last + 1):
                a, b = indptr[k], indptr[k + 1]
                self._rows_idx.append(indices[a:b].astype(np.int64))
                self._rows_val.append(np.asarray(values[a:b], dtype=np.float64))
                self.buf_nnz += int(b - a)
            r += last + 1
            if last == cut:
                self._flush()

    # -- the buffer step ---------------------------------------------------------------------
    def draw_start_block(self, buffer_idx, attempt, purpose):
        """G ~ N(0,1)^{d x ell} of SimultaneousIteration (Alg 1) for attempt ``attempt`` of buffer
        ``buffer_idx`` (keyed as in ``oracle.rng``).  Tests override it to plant a start block."""
        return start_block(self.seed, self.stream_id, buffer_idx, attempt, purpose, self.d, self.ell)

    def _fold(self, B, live, buffer_idx, vs_start, purpose_G, purpose_x, log):
        """Fold the pending buffer into (B, live); returns (B, live, VerifySpectral calls made)."""
        m = self.buf_rows
        if m == 0:
            return B, live, 0
        A = self._buffer_matrix()
        calls = [0]
        if m <= self.ell:
            R = A.toarray()
            r_add = m
        else:
            q = self.q_override if self.q_override is not None else si_iterations(m, self.eps)

            def next_i():
                calls[0] += 1
                return vs_start + calls[0]

            R = boosted_sparse_shrink(
                A, self.ell,
                lambda a: self.draw_start_block(buffer_idx, a, purpose_G),
                lambda a: sphere_vector(self.seed, self.stream_id, buffer_idx, a, purpose_x, self.d),
                next_i, q=q, delta=self.delta, max_attempts=self.max_attempts, verify=self.verify,
                unit_roundoff=self.unit_roundoff, log=log)
            r_add = self.ell - 1
        stack = np.vstack([B, R])
        B2, live2 = dense_shrink(stack, self.ell, live + r_add)
        return B2, live2, calls[0]

    def _flush(self):
        rec: list[dict] = []
        self.B, self.live, calls = self._fold(self.B, self.live, self.flushes, self.vs_calls,
                                              PURPOSE_SI, PURPOSE_VS, rec)
        self.log.append({"buffer": self.flushes, "rows": self.buf_rows, "nnz": self.buf_nnz, "attempts": rec})
        self.vs_calls += calls
        self.flushes += 1
        self._clear_buffer()

    # -- query and merge ------------------------------------------------------------------
    def query(self, log=None):
        """B for everything appended so far (pending rows folded in a copy); returns (B, live, calls)."""
        return self._fold(self.B.copy(), self.live, self.flushes, self.vs_calls,
                          PURPOSE_QUERY_SI, PURPOSE_QUERY_VS, log)

    def sketch(self) -> np.ndarray:
        return self.query()[0]

    def merge(self, other: "SFDOracle"):
        """dst <- DenseShrink([query(dst); query(src)]) (mergeability, Sec. 2.1)."""
        if other.d != self.d or other.ell != self.ell:
            raise ValueError("merge needs equal d and ell")
        Bd, ld, calls = self.query()
        Bs, ls, _ = other.query()
        self.B, self.live = dense_shrink(np.vstack([Bd, Bs]), self.ell, ld + ls)
        self.vs_calls += calls
        self.flushes += 1
        self._clear_buffer()

    def copy(self) -> "SFDOracle":
        return copy.deepcopy(self)


class FDBatchOracle(SFDOracle):
    """FrequentDirections (Sec. 2.1) in batches of ell rows: the buffer is flushed every ell rows
    and, holding at most ell rows, is folded exactly, so the sketch changes only through
    DenseShrink (Alg 5) of [B; buffer] -- the paper's FD comparator with the stack's new rows
    arriving ell at a time instead of one at a time (it agrees with FDOracle up to its first
    shrink, at 2 ell rows)."""

    def __init__(self, d, ell, **kw):
        super().__init__(d, ell, flush_rows=ell, flush_nnz=float("inf"), **kw)


class FDOracle:
    """FrequentDirections with DenseShrink (Sec. 2.1): rows join the sketch until it holds 2*ell
    rows, then DenseShrink halves it.  The query applies DenseShrink to what is held."""

    def __init__(self, d, ell):
        self.d, self.ell = int(d), int(ell)
        self.stack = np.zeros((0, self.d))

    def append_dense(self, rows: np.ndarray):
        rows = np.atleast_2d(np.asarray(rows, dtype=np.float64))
        for row in rows:
            self.stack = np.vstack([self.stack, row[None, :]])
            if self.stack.shape[0] == 2 * self.ell:
                B, live = dense_shrink(self.stack, self.ell, self.stack.shape[0])
                self.stack = B[:live].copy()

    def append_csr(self, indptr, indices, values):
        indptr, indices, values = _check_csr(indptr, indices, values, self.d)
        n = len(indptr) - 1
        lo, hi = int(indptr[0]), int(indptr[-1])
        A = sp.csr_matrix((np.asarray(values[lo:hi], np.float64), indices[lo:hi], indptr - lo), shape=(n, self.d))
        for k in range(n):
            self.append_dense(A[k].toarray())

    def sketch(self) -> np.ndarray:
        B, _ = dense_shrink(self.stack, self.ell, self.stack.shape[0])
        return B

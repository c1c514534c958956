"""Synthetic sparse row streams (recipes in the repository's design notes).

Common recipe for the Zipf workloads:
* row i stores k_i ~ Poisson(lambda) entries (clamped to [0, d]);
* its columns are drawn one after another from a finite Zipf(s) law over d columns,
  P(j) proportional to (j+1)^-s (inverse CDF on an FP64 table), a draw equal to an earlier
  column of the same row is rejected (sampling without replacement);
* column ids then go through a fixed seeded permutation, so popularity is not tied to the
  index, and each row's ids are sorted (canonical CSR);
* values: a base distribution plus, where a config asks for it, the entries of a planted
  low-rank matrix U diag(sigma) V^T at the sampled positions.
Rows are generated in chunks of CHUNK rows, each from its own seeded numpy generator, so a
prefix of a stream is the same whatever the stream's length.  Values are returned as FP32,
the boundary's value type; the oracle reads the same FP32 numbers in FP64.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

CHUNK = 65536


@dataclass
class CsrStream:
    indptr: np.ndarray   # int64, n + 1
    indices: np.ndarray  # int32
    values: np.ndarray   # float32
    d: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return len(self.indptr) - 1

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1] - self.indptr[0])

    def rows(self, lo: int, hi: int) -> "CsrStream":
        """Rows [lo, hi) with a rebased indptr (copies)."""
        a, b = int(self.indptr[lo]), int(self.indptr[hi])
        return CsrStream(self.indptr[lo:hi + 1] - a, self.indices[a:b].copy(), self.values[a:b].copy(), self.d,
                         dict(self.meta, rows=(lo, hi)))

    def to_scipy(self):
        import scipy.sparse as sp
        a = int(self.indptr[0])
        return sp.csr_matrix((self.values.astype(np.float64), self.indices.astype(np.int64), self.indptr - a),
                             shape=(self.n, self.d))


def zipf_cdf(d: int, s: float) -> np.ndarray:
    """FP64 CDF of the finite Zipf(s) law on {0..d-1}, P(j) ~ (j+1)^-s."""
    w = np.arange(1, d + 1, dtype=np.float64) ** (-float(s))
    c = np.cumsum(w)
    return c / c[-1]


def _first_distinct(cand: np.ndarray, k: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """For each row of ``cand`` keep the first k[r] distinct values in draw order.

    Returns (mask of kept positions, whether the row had enough distinct values).
    """
    R, W = cand.shape
    order = np.argsort(cand, axis=1, kind="stable")
    srt = np.take_along_axis(cand, order, axis=1)
    first_sorted = np.ones((R, W), dtype=bool)
    first_sorted[:, 1:] = srt[:, 1:] != srt[:, :-1]
    first = np.zeros((R, W), dtype=bool)
    np.put_along_axis(first, order, first_sorted, axis=1)
    cnt = np.cumsum(first, axis=1)
    keep = first & (cnt <= k[:, None])
    enough = cnt[:, -1] >= k
    return keep, enough


def _rows_chunk(rng: np.random.Generator, rows: int, d: int, lam: float, cdf: np.ndarray, perm: np.ndarray | None):
    k = np.minimum(rng.poisson(lam, size=rows), d).astype(np.int64)
    cols = [None] * rows
    todo = np.arange(rows)
    pad = 16
    while todo.size:
        kk = k[todo]
        W = int(kk.max(initial=0)) + pad
        u = rng.random((todo.size, W))
        cand = np.minimum(np.searchsorted(cdf, u, side="right"), d - 1).astype(np.int64)
        keep, enough = _first_distinct(cand, kk)
        for j in np.nonzero(enough)[0]:
            cols[todo[j]] = cand[j][keep[j]]
        todo = todo[~enough]
        pad *= 2
    lens = k
    flat = np.concatenate(cols) if rows else np.zeros(0, np.int64)
    if perm is not None:
        flat = perm[flat]
    # sort each row's ids
    rowid = np.repeat(np.arange(rows), lens)
    o = np.lexsort((flat, rowid))
    flat = flat[o]
    return lens, flat.astype(np.int32)


def poisson_zipf_pattern(n: int, d: int, lam: float, s: float, seed_words, permute: bool = True):
    """Sparsity pattern of the Zipf workloads: (indptr int64, indices int32)."""
    cdf = zipf_cdf(d, s)
    perm = np.random.default_rng(list(seed_words) + [0xC01]).permutation(d) if permute else None
    lens_all, idx_all = [], []
    for c in range((n + CHUNK - 1) // CHUNK):
        rows = min(CHUNK, n - c * CHUNK)
        rng = np.random.default_rng(list(seed_words) + [c])
        lens, idx = _rows_chunk(rng, rows, d, lam, cdf, perm)
        lens_all.append(lens)
        idx_all.append(idx)
    lens = np.concatenate(lens_all) if lens_all else np.zeros(0, np.int64)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=indptr[1:])
    indices = np.concatenate(idx_all) if idx_all else np.zeros(0, np.int32)
    return indptr, indices


def _gaussian_orthonormal(rows: int, r: int, rng: np.random.Generator) -> np.ndarray:
    q, _ = np.linalg.qr(rng.standard_normal((rows, r)))
    return q


def _planted_at(indptr, indices, U_rows_fn, sigma, V, chunk=CHUNK):
    """Entries (U diag(sigma) V^T)_{ij} at the stored positions, FP64, row chunk by row chunk."""
    n = len(indptr) - 1
    out = np.empty(int(indptr[-1]), dtype=np.float64)
    for c in range(0, n, chunk):
        hi = min(n, c + chunk)
        a, b = int(indptr[c]), int(indptr[hi])
        U = U_rows_fn(c, hi) * sigma[None, :]
        rows = np.repeat(np.arange(hi - c), np.diff(indptr[c:hi + 1]))
        out[a:b] = np.einsum("er,er->e", U[rows], V[indices[a:b]])
    return out


def _chunk_gaussian_rows(seed_words, n_total, r):
    """Rows [lo, hi) of an n_total x r matrix of N(0, 1/n_total) entries, generated per chunk."""
    def rows_fn(lo, hi):
        out = np.empty((hi - lo, r))
        pos = lo
        while pos < hi:
            c = pos // CHUNK
            rng = np.random.default_rng(list(seed_words) + [0x5EED, c])
            block = rng.standard_normal((min(CHUNK, n_total - c * CHUNK), r)) / np.sqrt(n_total)
            a = pos - c * CHUNK
            b = min(block.shape[0], hi - c * CHUNK)
            out[pos - lo:pos - lo + (b - a)] = block[a:b]
            pos += b - a
        return out
    return rows_fn


def stream_1e4_d1e3(seed: int = 0, n: int = 10_000) -> CsrStream:
    """n=10,000, d=1,000, Poisson(10) entries per row, Zipf(1.1) columns; values = entries of a
    planted rank-10 U diag(sigma) V^T (U, V Gaussian then QR-orthonormalised, sigma_i = 2^-i)
    plus N(0, 0.1^2) noise (0.1 read as the standard deviation); ell = 20, k = 10."""
    d, lam, s, r = 1000, 10.0, 1.1, 10
    words = [seed, 1]
    indptr, indices = poisson_zipf_pattern(n, d, lam, s, words)
    rng = np.random.default_rng(words + [0xBA5E])
    U = _gaussian_orthonormal(n, r, rng)
    V = _gaussian_orthonormal(d, r, rng)
    sigma = 2.0 ** -np.arange(1, r + 1)
    planted = _planted_at(indptr, indices, lambda lo, hi: U[lo:hi], sigma, V)
    noise = np.random.default_rng(words + [0x401]).normal(0.0, 0.1, size=len(indices))
    vals = (planted + noise).astype(np.float32)
    return CsrStream(indptr, indices, vals, d, dict(name="stream_1e4_d1e3", ell=20, k=10, seed=seed,
                                                    planted_energy_share=float(np.sum(planted ** 2) / np.sum((planted + noise) ** 2))))


def stream_1e6_d1e5(seed: int = 0, n: int = 1_000_000) -> CsrStream:
    """n=1e6, d=1e5, Poisson(50) per row, Zipf(1.0) columns; values lognormal(0,1) plus a planted
    rank-20 component (sigma_i = 1/i) scaled to 30% of the expected energy at the sampled
    positions; ell = 50.  U is N(0, 1/n) per entry with n = 1e6 (near-orthonormal, generated per
    row chunk, so a shorter stream has the same rows of U); V is Gaussian then
    QR-orthonormalised.  Whole 65,536-row chunks of a shorter stream equal those of the full one."""
    d, lam, s, r = 100_000, 50.0, 1.0, 20
    return _lognormal_planted(seed, 2, n, d, lam, s, r, share=0.3, ell=50, name="stream_1e6_d1e5", n_total=1_000_000)


def _lognormal_planted(seed, cid, n, d, lam, s, r, share, ell, name, n_total):
    words = [seed] + (list(cid) if isinstance(cid, (list, tuple)) else [cid])
    indptr, indices = poisson_zipf_pattern(n, d, lam, s, words)
    base = np.empty(len(indices))
    for c in range(0, n, CHUNK):
        hi = min(n, c + CHUNK)
        a, b = int(indptr[c]), int(indptr[hi])
        base[a:b] = np.random.default_rng(words + [0x109, c // CHUNK]).lognormal(0.0, 1.0, size=b - a)
    vals = base
    meta = dict(name=name, ell=ell, k=10, seed=seed)
    if r:
        V = _gaussian_orthonormal(d, r, np.random.default_rng(words + [0xBA5E]))
        sigma = 1.0 / np.arange(1, r + 1)
        planted = _planted_at(indptr, indices, _chunk_gaussian_rows(words, n_total, r), sigma, V)
        # E[planted^2] per entry = sum(sigma^2) / (n_total * d); E[lognormal^2] = e^2
        e_base = np.exp(2.0)
        e_pl = float(np.sum(sigma ** 2)) / (n_total * d)
        c2 = share * e_base / ((1.0 - share) * e_pl)
        vals = base + np.sqrt(c2) * planted
        meta["planted_scale"] = float(np.sqrt(c2))
    return CsrStream(indptr, indices, vals.astype(np.float32), d, meta)


def stream_2e6_d5e4(seed: int = 0, n: int = 2_000_000) -> CsrStream:
    """n=2e6, d=5e4, Poisson(80), Zipf(1.1); N(0,1) values plus a planted rank-50 component with
    sigma_i = 1/i taken literally (unscaled, so its energy share is tiny); ell = 200."""
    d, lam, s, r = 50_000, 80.0, 1.1, 50
    words = [seed, 3]
    indptr, indices = poisson_zipf_pattern(n, d, lam, s, words)
    V = _gaussian_orthonormal(d, r, np.random.default_rng(words + [0xBA5E]))
    sigma = 1.0 / np.arange(1, r + 1)
    planted = _planted_at(indptr, indices, _chunk_gaussian_rows(words, 2_000_000, r), sigma, V)
    base = np.empty(len(indices))
    for c in range(0, n, CHUNK):
        hi = min(n, c + CHUNK)
        a, b = int(indptr[c]), int(indptr[hi])
        base[a:b] = np.random.default_rng(words + [0x401, c // CHUNK]).standard_normal(b - a)
    return CsrStream(indptr, indices, (base + planted).astype(np.float32), d,
                     dict(name="stream_2e6_d5e4", ell=200, k=10, seed=seed))


def batch_stream_d2e4(stream_id: int, seed: int = 0, n: int | None = None) -> CsrStream:
    """Stream s of the 4,096-stream batch: n_s = round(exp(U(ln 1e3, ln 1e5))) rows, d = 2e4,
    Poisson(30), Zipf(1.1), lognormal(0,1) values; ell = 32."""
    d, lam, s = 20_000, 30.0, 1.1
    if n is None:
        u = np.random.default_rng([seed, 4, 0x1E9]).random(4096)[stream_id]
        n = int(round(np.exp(np.log(1e3) + u * (np.log(1e5) - np.log(1e3)))))
    st = _lognormal_planted(seed, (4, 1000 + stream_id), n, d, lam, s, 0, 0.0, 32, "batch_stream_d2e4", n)
    st.meta["stream_id"] = stream_id
    return st


def paper_head_tail(n: int = 10_000, d: int = 1000, z: int = 100, seed: int = 0) -> CsrStream:
    """The paper's synthetic generator (Sec. 4, "Datasets"): each row gets exactly z distinct
    non-zeros of value +1 or -1; each placement picks the head (the first 1.5 z columns) with
    probability 0.9, else the tail, and a column uniformly inside it; a placement that repeats a
    column of the row is drawn again (rows are generated with vectorised draws: the first z
    distinct placements of each row's draw sequence)."""
    rng = np.random.default_rng([seed, 0x4EAD])
    head = min(int(1.5 * z), d)
    k = np.full(n, min(z, d), dtype=np.int64)
    cols = [None] * n
    todo = np.arange(n)
    W = 2 * z + 16
    while todo.size:
        R = todo.size
        in_head = rng.random((R, W)) < 0.9
        if head >= d:
            in_head[:] = True
        hc = rng.integers(0, head, size=(R, W))
        tc = rng.integers(head, d, size=(R, W)) if head < d else hc
        cand = np.where(in_head, hc, tc)
        keep, enough = _first_distinct(cand, k[todo])
        for j in np.nonzero(enough)[0]:
            cols[todo[j]] = np.sort(cand[j][keep[j]])
        todo = todo[~enough]
        W *= 2
    indptr = np.arange(n + 1, dtype=np.int64) * int(k[0])
    idx = np.concatenate(cols).astype(np.int32) if n else np.zeros(0, np.int32)
    vals = rng.choice(np.array([-1.0, 1.0], dtype=np.float32), size=len(idx))
    return CsrStream(indptr, idx, vals, d, dict(name="paper_head_tail", ell=50, k=10, seed=seed, z=z))


def spiked_stream(n: int, d: int, seed: int = 0, *, noise_nnz: int = 12, spike: float = 3.0,
                  noise: float = 0.3) -> CsrStream:
    """Rows that alternate between noise and a spike: even rows hold noise_nnz distinct columns of
    1 .. d - 1 with N(0, noise^2) values, odd rows the single entry (column 0, spike).  Column 0 then
    carries the dominant right singular direction e_0 of every buffer of consecutive rows, and
    nothing else touches it: a start block whose row 0 is zero misses it."""
    rng = np.random.default_rng([seed, 0x5B1E])
    idx, val, lens = [], [], []
    for r in range(n):
        if r % 2:
            idx.append(np.zeros(1, np.int64))
            val.append(np.full(1, spike))
        else:
            idx.append(np.sort(rng.choice(np.arange(1, d), size=noise_nnz, replace=False)))
            val.append(rng.standard_normal(noise_nnz) * noise)
        lens.append(len(idx[-1]))
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=indptr[1:])
    indices = np.concatenate(idx).astype(np.int32) if n else np.zeros(0, np.int32)
    values = np.concatenate(val).astype(np.float32) if n else np.zeros(0, np.float32)
    return CsrStream(indptr, indices, values, d, dict(name="spiked", seed=seed))


def small_random_csr(n: int, d: int, lam: float, seed: int, *, s: float = 1.1, dup_rate: float = 0.0,
                     empty_rate: float = 0.0, dist: str = "normal") -> CsrStream:
    """A small Zipf-Poisson stream for tests, with optional empty rows and repeated column ids."""
    rng = np.random.default_rng([seed, 0x7E57])
    indptr, indices = poisson_zipf_pattern(n, d, lam, s, [seed, 0x7E57], permute=True)
    lens = np.diff(indptr)
    if empty_rate > 0:
        keep_row = rng.random(n) >= empty_rate
        mask = np.repeat(keep_row, lens)
        lens = np.where(keep_row, lens, 0)
        indices = indices[mask]
    if dup_rate > 0 and len(indices):
        # repeat some entries of a row (same column id stored twice, adjacent)
        rows = np.repeat(np.arange(n), lens)
        dup = rng.random(len(indices)) < dup_rate
        indices = np.repeat(indices, 1 + dup.astype(np.int64))
        rows = np.repeat(rows, 1 + dup.astype(np.int64))
        lens = np.bincount(rows, minlength=n)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=indptr[1:])
    if dist == "normal":
        vals = rng.standard_normal(len(indices))
    elif dist == "lognormal":
        vals = rng.lognormal(0.0, 1.0, len(indices))
    else:
        vals = rng.choice([-1.0, 1.0], size=len(indices))
    return CsrStream(indptr, indices.astype(np.int32), vals.astype(np.float32), d, dict(name="small_random", seed=seed))

"""The seeded input generators (workloads/) against the recipe they implement: Poisson(lambda)
row lengths clamped to [0, d], column ids drawn from the finite Zipf(s) law by inverse CDF and
kept without replacement in draw order, a fixed permutation of the ids, ids sorted in a row.

Checked against closed forms rather than against the generators' own code: the Poisson mean and
variance, the Zipf probabilities of single-entry rows (chi-square), the popularity order under
the permutation, and the chunking properties the tests and the bench rely on.
"""

import math

import numpy as np
import pytest
import scipy.stats

from workloads.synthetic import CHUNK, poisson_zipf_pattern


def _check_rows(indptr, indices, d):
    assert indptr[0] == 0 and np.all(np.diff(indptr) >= 0)
    assert indices.min(initial=0) >= 0 and indices.max(initial=-1) < d
    rowid = np.repeat(np.arange(len(indptr) - 1), np.diff(indptr))
    same = rowid[1:] == rowid[:-1]
    assert np.all(np.diff(indices.astype(np.int64))[same] > 0)  # distinct and sorted in a row


def _zipf_p(d, s):
    w = np.arange(1, d + 1, dtype=np.float64) ** (-s)
    return w / w.sum()


def test_host_lengths_ids_and_popularity():
    # the 10^6-row stream's law (d = 1e5, Poisson(50), Zipf(1.0)) on 20,000 rows
    d, lam, s, words = 100_000, 50.0, 1.0, [7, 2]
    indptr, indices = poisson_zipf_pattern(20_000, d, lam, s, words)
    _check_rows(indptr, indices, d)
    lens = np.diff(indptr)
    se = math.sqrt(lam / lens.size)
    assert abs(lens.mean() - lam) < 6 * se
    assert abs(lens.var() / lam - 1) < 0.1
    # ids pass through the generator's fixed permutation: Zipf rank j is id perm[j], so the most
    # frequent ids are perm[0], perm[1], perm[2] in that order
    perm = np.random.default_rng(list(words) + [0xC01]).permutation(d)
    cnt = np.bincount(indices, minlength=d)
    assert list(np.argsort(-cnt, kind="stable")[:3]) == list(perm[:3])
    # rank 0 has P = 1 / H_d (1/12.09 at d = 1e5); a row of k distinct draws misses it with
    # probability at most (1 - p0)^k, so nearly every row holds it
    p0 = _zipf_p(d, s)[0]
    rows_with = cnt[perm[0]]
    bound_missing = np.sum((1 - p0) ** lens)
    assert lens.size - rows_with <= 2 * bound_missing + 10


def test_host_single_entry_rows_follow_the_zipf_law():
    # with lambda small most rows hold 0 or 1 entries; a 1-entry row's id is one inverse-CDF draw
    d, lam, s, words = 50, 0.05, 1.1, [11, 3]
    indptr, indices = poisson_zipf_pattern(200_000, d, lam, s, words)
    _check_rows(indptr, indices, d)
    lens = np.diff(indptr)
    assert abs(lens.mean() - lam) < 6 * math.sqrt(lam / lens.size)
    one = np.nonzero(lens == 1)[0]
    perm = np.random.default_rng(list(words) + [0xC01]).permutation(d)
    inv = np.empty(d, dtype=np.int64)
    inv[perm] = np.arange(d)
    ranks = inv[indices[indptr[one]]]
    obs = np.bincount(ranks, minlength=d)
    exp = _zipf_p(d, s) * one.size
    stat, p = scipy.stats.chisquare(obs, exp)
    assert p > 1e-4, (stat, p)


def test_host_whole_chunks_do_not_depend_on_the_length():
    # rows are generated in chunks of CHUNK rows, each from its own seeded generator: whole chunks
    # of a shorter stream equal the longer stream's, and every row length agrees
    a = poisson_zipf_pattern(CHUNK + 500, 1000, 10.0, 1.1, [3])
    b = poisson_zipf_pattern(CHUNK + 4000, 1000, 10.0, 1.1, [3])
    assert np.array_equal(a[0], b[0][:CHUNK + 501])
    nnz = int(a[0][CHUNK])
    assert np.array_equal(a[1][:nnz], b[1][:nnz])


def test_device_generator_draws_do_not_depend_on_chunking():
    # the counter-based generator keys every draw by (row key, counter, purpose): integer draws
    # are the same however rows are grouped, and so are the values on one device type
    import torch

    from workloads import device

    keys = device.row_keys(device.stream_key(5, 9), 3000, "cpu")
    whole = device.gen_csr(keys, 2000, 20.0, 1.1, 77, r=3, share=0.3, n_total=3000)
    parts = device.gen_csr(keys, 2000, 20.0, 1.1, 77, r=3, share=0.3, n_total=3000, chunk=700)
    for x, y in zip(whole, parts):
        assert torch.equal(x, y)
    ptr, idx, val = (t.numpy() for t in whole)
    _check_rows(ptr, idx, 2000)
    lens = np.diff(ptr)
    assert abs(lens.mean() - 20.0) < 6 * math.sqrt(20.0 / lens.size)
    assert abs(lens.var() / 20.0 - 1) < 0.15
    assert np.all(np.isfinite(val))
    # a prefix of the rows is generated identically on its own
    head = device.gen_csr(keys[:1000], 2000, 20.0, 1.1, 77, r=3, share=0.3, n_total=3000)
    n1 = int(head[0][-1])
    assert torch.equal(head[0], whole[0][:1001])
    assert torch.equal(head[1], whole[1][:n1]) and torch.equal(head[2], whole[2][:n1])


def _head_count_law(z, head, d, p_head=0.9):
    """Exact distribution of the number of head columns in a row of the paper's generator (Sec. 4,
    "Datasets"): a placement picks the head (first `head` columns) with probability p_head, else
    the tail, a column uniformly inside it, and is drawn again when the row already holds that
    column.  Conditioned on landing on a new column, the next new column is in the head with
    probability p_head (H - h)/H / (p_head (H - h)/H + (1 - p_head)(T - t)/T)."""
    H, T = head, d - head
    P = np.zeros(z + 1)
    P[0] = 1.0
    for step in range(z):
        Q = np.zeros(z + 1)
        for h in range(step + 1):
            if P[h] == 0.0:
                continue
            t = step - h
            a = p_head * (H - h) / H if H else 0.0
            b = (1 - p_head) * (T - t) / T if T else 0.0
            Q[h + 1] += P[h] * a / (a + b)
            Q[h] += P[h] * b / (a + b)
        P = Q
    return P


@pytest.mark.parametrize("d,z", [(1000, 5), (1000, 100), (1000, 500), (6000, 100)])
def test_paper_head_tail_follows_its_recipe(d, z):
    # the paper's synthetic rows (Sec. 4, "Datasets"): exactly z distinct non-zeros of value +-1,
    # head = the first 1.5 z columns, each placement in the head with probability 0.9, uniform
    # inside the chosen part, repeats of a column drawn again
    from workloads import paper_head_tail

    n = 10_000 if z <= 100 else 2_000
    st = paper_head_tail(n=n, d=d, z=z, seed=3)
    _check_rows(st.indptr, st.indices, d)
    assert np.all(np.diff(st.indptr) == z)
    assert set(np.unique(st.values)) == {-1.0, 1.0}
    plus = int(np.sum(st.values > 0))
    assert abs(plus - st.nnz / 2) < 6 * math.sqrt(st.nnz / 4)  # a fair sign
    head = int(1.5 * z)
    in_head = (st.indices < head).reshape(n, z).sum(axis=1)
    law = _head_count_law(z, head, d)
    support = np.nonzero(law * n >= 5)[0]  # chi-square over the cells with enough mass
    obs = np.array([np.sum(in_head == h) for h in support], dtype=np.float64)
    exp = law[support] * n
    obs = np.append(obs, n - obs.sum())
    exp = np.append(exp, n - exp.sum())
    keep = exp > 0
    stat, p = scipy.stats.chisquare(obs[keep], exp[keep] * obs[keep].sum() / exp[keep].sum())
    assert p > 1e-4, (stat, p, law[support][:5])
    # uniform inside the head and inside the tail
    cnt = np.bincount(st.indices, minlength=d).astype(np.float64)
    for part in (cnt[:head], cnt[head:]):
        if part.sum() > 20 * part.size:
            stat, p = scipy.stats.chisquare(part)
            assert p > 1e-4, (stat, p)

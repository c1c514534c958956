"""Zipf-Poisson row streams generated with torch, chunk by chunk, on the GPU (or the CPU).

For the workloads too large to build on the host (1e9 stored entries; 4,096 streams of 2.6e9
entries together).  Same recipe as ``synthetic.py`` (Poisson row lengths clamped to [0, d],
columns drawn from a finite Zipf(s) law by inverse CDF and kept without replacement in draw
order, a fixed permutation of the column ids, ids sorted inside a row, lognormal(0, 1) values
plus an optional planted low-rank component scaled to a share of the expected energy), but
every draw comes from a counter-based hash instead of numpy's generators:

* each row has a 64-bit key (``row_keys``); draw t of the row for purpose p is
  ``mix64(key + GOLDEN * (t + 1) + PURPOSE * p)`` with ``mix64`` the splitmix64 finaliser
  (Steele, Lea and Flood, OOPSLA 2014), so a row's draws do not depend on how rows are grouped
  into chunks or on the device;
* a uniform in (0, 1) is ((h >> 11) + 1/2) 2^-53 (exact in FP64); normals come from the
  Box-Muller transform on two uniforms.

Integer draws (row lengths, column ids, the permutation) are therefore identical on any
device; FP64 transcendental functions may differ in the last bit between devices, so values
are reproducible bit for bit on one device type.  Tests that compare with the oracle give it
the arrays generated here, copied to the host.

Input generation only: nothing here is part of the sketching method.
"""

from __future__ import annotations

import math

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
PURPOSE = 0xD1B54A32D192ED03
P_LEN, P_COL, P_VAL, P_VAL2, P_U, P_PERM, P_V = 1, 2, 3, 4, 5, 6, 7


def _s64(v: int) -> int:
    """An unsigned 64-bit constant as the signed value torch's int64 holds."""
    v &= MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


def _lsr(x, s: int):
    """Logical right shift of int64 tensors."""
    return (x >> s) & ((1 << (64 - s)) - 1)


def mix64(x):
    """splitmix64 finaliser on an int64 tensor (wrapping arithmetic)."""
    x = x ^ _lsr(x, 30)
    x = x * _s64(0xBF58476D1CE4E5B9)
    x = x ^ _lsr(x, 27)
    x = x * _s64(0x94D049BB133111EB)
    return x ^ _lsr(x, 31)


def _draw(keys, t, purpose: int):
    """Hash words for draw(s) t of rows keys (broadcasting)."""
    return mix64(keys + _s64(GOLDEN) * (t + 1) + _s64(PURPOSE * purpose))


def _unit(h):
    import torch

    return (_lsr(h, 11).to(torch.float64) + 0.5) * 2.0 ** -53


def _normal(keys, t, purpose: int):
    import torch

    u1 = _unit(_draw(keys, 2 * t, purpose))
    u2 = _unit(_draw(keys, 2 * t + 1, purpose))
    return torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * math.pi * u2)


def stream_key(*words: int) -> int:
    """A 64-bit key from small integers (seed, config, stream ...)."""
    import torch

    k = 0x243F6A8885A308D3
    for w in words:
        k = int(mix64(torch.tensor([_s64(k ^ (w & MASK64))], dtype=torch.int64))[0]) & MASK64
    return k


def row_keys(base: int, n: int, device):
    """Keys of rows 0..n-1 of a stream with key ``base``."""
    import torch

    return mix64(torch.arange(n, dtype=torch.int64, device=device) * _s64(GOLDEN) + _s64(base))


def zipf_cdf_t(d: int, s: float, device):
    import torch

    w = torch.arange(1, d + 1, dtype=torch.float64, device=device) ** (-float(s))
    c = torch.cumsum(w, 0)
    return c / c[-1]


def poisson_cdf_t(lam: float, device):
    import torch

    kmax = int(lam + 14 * math.sqrt(lam) + 30)
    k = np.arange(kmax + 1, dtype=np.float64)
    logp = -lam + k * math.log(lam) - np.array([math.lgamma(v + 1) for v in k])
    c = np.cumsum(np.exp(logp))
    return torch.from_numpy(c / c[-1]).to(device)


def column_permutation(key: int, d: int, device):
    """A fixed permutation of the d column ids (ranks of hashed ids)."""
    import torch

    h = mix64(torch.arange(d, dtype=torch.int64, device=device) + _s64(key * 31 + P_PERM))
    return torch.argsort(h, stable=True)


def gen_rows(keys, d: int, lam: float, cdf_zipf, cdf_pois, perm):
    """Sparsity pattern of the rows with the given keys: (lens int64, cols int64 sorted per row)."""
    import torch

    dev = keys.device
    R = keys.numel()
    lens = torch.searchsorted(cdf_pois, _unit(_draw(keys, torch.zeros_like(keys), P_LEN)), right=True)
    lens = lens.clamp(max=d).to(torch.int64)
    out_cols = torch.empty(0, dtype=torch.int64, device=dev)
    out_rows = torch.empty(0, dtype=torch.int64, device=dev)
    todo = torch.arange(R, device=dev)
    W = int(lens.max().item()) * 2 + 16 if R else 0
    while todo.numel():
        k = lens[todo]
        t = torch.arange(W, dtype=torch.int64, device=dev)
        u = _unit(_draw(keys[todo][:, None], t[None, :], P_COL))
        cand = torch.searchsorted(cdf_zipf, u, right=True).clamp(max=d - 1)
        srt, order = torch.sort(cand, dim=1, stable=True)
        first_sorted = torch.ones_like(srt, dtype=torch.bool)
        first_sorted[:, 1:] = srt[:, 1:] != srt[:, :-1]
        first = torch.zeros_like(first_sorted).scatter_(1, order, first_sorted)
        cnt = torch.cumsum(first.to(torch.int64), dim=1)
        keep = first & (cnt <= k[:, None])
        enough = cnt[:, -1] >= k
        ok = torch.nonzero(enough).flatten()
        kk = keep[ok]
        out_cols = torch.cat([out_cols, cand[ok][kk]])
        out_rows = torch.cat([out_rows, todo[ok][:, None].expand(-1, W)[kk]])
        todo = todo[~enough]
        W *= 2
    cols = perm[out_cols]
    o = torch.argsort(out_rows * d + cols)
    return lens, cols[o], out_rows[o]


def gen_csr(keys, d: int, lam: float, s: float, perm_key: int, *, r: int = 0, share: float | None = 0.0,
            n_total: int = 1, chunk: int = 1 << 17, base: str = "lognormal"):
    """CSR (indptr int64, indices int32, values float32) of the rows with the given keys, on
    their device.

    Values: lognormal(0, 1) (base="lognormal") or N(0, 1) (base="normal") plus, for r > 0, a
    planted rank-r component U diag(sigma) V^T at the stored positions with sigma_i = 1/i,
    U[i, :] ~ N(0, 1/n_total) per entry (near-orthonormal, keyed by row), V a Gaussian d x r
    block orthonormalised by CholeskyQR2 in FP64, scaled so its expected share of the energy is
    ``share`` (share=None: unscaled).
    """
    import torch

    device = keys.device
    n = keys.numel()
    cdf_z = zipf_cdf_t(d, s, device)
    cdf_p = poisson_cdf_t(lam, device)
    perm = column_permutation(perm_key, d, device)
    V = sigma = None
    scale = 0.0
    if r:
        vk = row_keys(stream_key(perm_key, P_V), d, device)
        G = torch.stack([_normal(vk, torch.full_like(vk, c), P_V) for c in range(r)], dim=1)
        for _ in range(2):  # CholeskyQR2; the r x r factorisation on the host
            Rm = torch.linalg.cholesky((G.T @ G).cpu())
            G = G @ torch.linalg.inv(Rm).T.to(device)
        V = G
        sigma = 1.0 / torch.arange(1, r + 1, dtype=torch.float64, device=device)
        e_pl = float((sigma ** 2).sum()) / (n_total * d)
        e_base = math.exp(2.0) if base == "lognormal" else 1.0
        scale = 1.0 if share is None else math.sqrt(share * e_base / ((1.0 - share) * e_pl))
    ptr_parts, idx_parts, val_parts = [torch.zeros(1, dtype=torch.int64, device=device)], [], []
    base_nnz = 0
    for c0 in range(0, n, chunk):
        ck = keys[c0:c0 + chunk]
        lens, cols, rows = gen_rows(ck, d, lam, cdf_z, cdf_p, perm)
        # position of each entry inside its row (the draw counter of its value)
        starts = torch.cumsum(lens, 0) - lens
        pos = torch.arange(cols.numel(), device=device) - starts[rows]
        vals = _normal(ck[rows], pos, P_VAL)
        if base == "lognormal":
            vals = torch.exp(vals)
        if r:
            U = torch.stack([_normal(ck, torch.full_like(ck, c), P_U) for c in range(r)], dim=1)
            U = U * (sigma[None, :] / math.sqrt(n_total))
            pl = torch.empty(cols.numel(), dtype=torch.float64, device=device)
            step = 1 << 20
            for a in range(0, cols.numel(), step):
                b = min(cols.numel(), a + step)
                pl[a:b] = (U[rows[a:b]] * V[cols[a:b]]).sum(dim=1)
            vals = vals + scale * pl
        ptr_parts.append(torch.cumsum(lens, 0) + base_nnz)
        base_nnz += int(lens.sum().item())
        idx_parts.append(cols.to(torch.int32))
        val_parts.append(vals.to(torch.float32))
    return torch.cat(ptr_parts), torch.cat(idx_parts), torch.cat(val_parts)


def stream_1e7_d1e6(device, seed: int = 0, n: int = 10_000_000):
    """n=1e7, d=1e6, Poisson(100), Zipf(1.0) columns, lognormal(0,1) values plus a planted
    rank-100 component (sigma_i = 1/i) scaled to 30% of the expected energy; ell = 100.
    Rows 0..n-1 of the 1e7-row stream (a prefix for n < 1e7)."""
    import torch

    key = stream_key(seed, 5)
    return gen_csr(row_keys(key, n, torch.device(device)), 1_000_000, 100.0, 1.0, key, r=100, share=0.3,
                   n_total=10_000_000)


def stream_2e6_d5e4(device, seed: int = 0, n: int = 2_000_000):
    """n=2e6, d=5e4, Poisson(80), Zipf(1.1) columns, N(0,1) values plus a planted rank-50
    component with sigma_i = 1/i taken literally (unscaled); ell = 200."""
    import torch

    key = stream_key(seed, 3)
    return gen_csr(row_keys(key, n, torch.device(device)), 50_000, 80.0, 1.1, key, r=50, share=None,
                   n_total=2_000_000, base="normal")


def batch_stream_lengths(seed: int = 0, streams: int = 4096) -> np.ndarray:
    """Row counts of the 4,096 batch streams: round(exp(U(ln 1e3, ln 1e5))), U keyed by stream."""
    import torch

    k = row_keys(stream_key(seed, 4, 0x1E9), streams, "cpu")
    u = _unit(_draw(k, torch.zeros_like(k), P_LEN)).numpy()
    return np.rint(np.exp(np.log(1e3) + u * (np.log(1e5) - np.log(1e3)))).astype(np.int64)


def batch_streams_d2e4(device, seed: int = 0, streams: int = 4096, first: int = 0):
    """Streams first .. first + streams - 1 of the batching workload, one after another:
    (indptr, indices, values, row starts (streams + 1, int64 numpy)).  Stream s: n_s rows,
    d = 2e4, Poisson(30), Zipf(1.1) columns, lognormal(0,1) values; ell = 32."""
    import torch

    device = torch.device(device)
    lens = batch_stream_lengths(seed, 4096)[first:first + streams]
    bases = torch.tensor([_s64(stream_key(seed, 4, 1000 + first + s)) for s in range(streams)], dtype=torch.int64,
                         device=device)
    lens_t = torch.from_numpy(lens).to(device)
    sid = torch.repeat_interleave(torch.arange(streams, device=device), lens_t)
    row0 = torch.repeat_interleave(torch.cumsum(lens_t, 0) - lens_t, lens_t)
    idx_in = torch.arange(sid.numel(), device=device) - row0
    keys = mix64(idx_in * _s64(GOLDEN) + bases[sid])
    ptr, idx, val = gen_csr(keys, 20_000, 30.0, 1.1, stream_key(seed, 4), chunk=1 << 20)
    starts = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    return ptr, idx, val, starts

"""The shrink operators of Sparse Frequent Directions, in FP64, step by step.

Algorithms (numbered in order of appearance in the paper):
  Alg 1 SimultaneousIteration      Sec. 2.2
  Alg 3 SparseShrink               Sec. 3
  Alg 4 BoostedSparseShrink        Sec. 3
  Alg 5 DenseShrink                Sec. 3
  Alg 6 VerifySpectral             Sec. 3.1

Readings where the paper is silent (each is listed in the design notes of the repository):
* q = ceil(ln(m/eps)/eps) for Alg 1 on an m-row input (the paper fixes only
  q = Theta(log(n/eps)/eps)); eps = 1/4 inside SparseShrink.
* SimultaneousIteration re-orthonormalises after every product (Householder QR).  In exact
  arithmetic the span is that of A (A^T A)^q G, which is all SparseShrink uses.
* VerifySpectral runs t = ceil(log2(d/delta_i)) power steps (constant c = 1, base 2) and
  evaluates ||C^t x|| <= 1 as a sum of logs of the normalised step norms.
* BoostedSparseShrink accepts without VerifySpectral when S = ||A'||_F^2 - ||B'||_F^2 is at
  rounding level (S <= 64 u ell ||A'||_F^2): then trace(A'^T A' - B'^T B') = S ~ 0 and the
  matrix is PSD (Property 1), so it is 0 and Property 2 holds for any Delta >= 0.  The unit
  roundoff u is that of the arithmetic whose decision is mirrored (FP64 by default).
* The retry loop of Alg 4 is capped (``max_attempts``); exhausting it raises NoConvergence.
* Zero singular values: the shrink factor sqrt(max(s_i^2 - s_l^2, 0)) / s_i is taken as 0.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

#: alpha of BoostedSparseShrink and Theorem 3.1 (Sec. 3, Alg 4)
ALPHA = 6.0 / 41.0


class NoConvergence(RuntimeError):
    """BoostedSparseShrink exhausted its attempts without VerifySpectral accepting."""


def si_iterations(m: int, eps: float) -> int:
    """q = ceil(ln(m/eps)/eps): the power count of SimultaneousIteration (Alg 1, q = Theta(log(n/eps)/eps)) on m rows."""
    return int(math.ceil(math.log(m / eps) / eps))


def vs_delta(delta: float, i: int) -> float:
    """delta_i = delta / (2 i^2) of the i-th VerifySpectral call (Alg 6); sum_i delta_i <= delta (Sec. 3.1)."""
    return delta / (2.0 * i * i)


def vs_steps(d: int, delta: float, i: int) -> int:
    """t = ceil(log2(d / delta_i)) power steps (Alg 6 with c = 1, log base 2)."""
    return int(math.ceil(math.log2(d / vs_delta(delta, i))))


def _orth(M: np.ndarray) -> np.ndarray:
    """GramSchmidt of Alg 1, as a Householder QR (reduced): orthonormal basis of the column span."""
    q, _ = np.linalg.qr(M, mode="reduced")
    return q


def simultaneous_iteration(A: sp.csr_matrix, G: np.ndarray, q: int) -> np.ndarray:
    """Alg 1: Z = GramSchmidt(A (A^T A)^q G) with the iterate orthonormalised after every product.

    A: m x d (sparse), G: d x k start block.  Returns Z, m x k with orthonormal columns.
    The products run in the order of the formula: q times X <- A^T (A X), then A X.
    """
    X = _orth(G)
    for _ in range(q):
        Y = _orth(A @ X)
        X = _orth(A.T @ Y)
    return _orth(A @ X)


def shrink_factors(sigma: np.ndarray, ell: int) -> np.ndarray:
    """Diagonal of sqrt(Lambda^2 - lambda_ell^2 I) (Alg 3 / Alg 5) for descending sigma, clamped at 0."""
    s2 = sigma[:ell] ** 2
    pivot = s2[ell - 1] if len(s2) >= ell else 0.0
    return np.sqrt(np.maximum(s2 - pivot, 0.0))


def sparse_shrink(A: sp.csr_matrix, G: np.ndarray, ell: int, q: int) -> dict:
    """Alg 3 SparseShrink on the m x d buffer A (ell <= m).

    Z = SimultaneousIteration(A, ell, 1/4); P = Z^T A; [H, Lambda, V] = svd(P, ell);
    B' = sqrt(Lambda^2 - lambda_ell^2 I) V^T.
    Returns B' (ell x d) and the intermediates the identities of Sec. 3.2 are stated on.
    """
    Z = simultaneous_iteration(A, G, q)
    P = np.asarray((A.T @ Z).T)  # ell x d
    H, lam, Vt = np.linalg.svd(P, full_matrices=False)
    lam_t = shrink_factors(lam, ell)
    Bp = lam_t[:, None] * Vt[:ell]
    return {"B": Bp, "Z": Z, "P": P, "lam": lam, "Vt": Vt[:ell], "q": q}


def dense_shrink(C: np.ndarray, ell: int, live_rows: int | None = None) -> tuple[np.ndarray, int]:
    """Alg 5 DenseShrink: [H, Lambda, V] = svd(C, ell); B = sqrt(Lambda^2 - lambda_ell^2 I) V^T.

    ``live_rows`` is the structural count of rows of C that may be non-zero.  When it is at most
    ell the stack is kept exactly (no shrink; the rows of Sigma V^T), which is what the stream
    needs when fewer than ell rows have been seen; otherwise the shrink of Alg 5 applies and the
    result has ell - 1 live rows.  Returns (B, live) with B of shape ell x d.
    """
    n, d = C.shape
    _, sig, Vt = np.linalg.svd(C, full_matrices=False)
    B = np.zeros((ell, d))
    k = min(ell, len(sig))
    if live_rows is not None and live_rows <= ell:
        B[:k] = sig[:k, None] * Vt[:k]
        return B, live_rows
    B[:k] = shrink_factors(sig, ell)[:k, None] * Vt[:k]
    return B, ell - 1


def verify_spectral(A: sp.csr_matrix, Bp: np.ndarray, half_delta: float, x: np.ndarray, t: int) -> tuple[bool, float]:
    """Alg 6 VerifySpectral on C = (A^T A - B'^T B') / (Delta / 2).

    Runs the power method from x for t steps and returns (||C^t x|| <= 1, ln ||C^t x||).
    Each step forms w = A^T (A y) - B'^T (B' y); the log of the product of the step norms
    divided by (Delta/2)^t is accumulated so nothing overflows.  A zero step vector means
    C^t x = 0, which passes.
    """
    y = x.copy()
    log_norm = 0.0
    log_half_delta = math.log(half_delta)
    for _ in range(t):
        w = A.T @ (A @ y) - Bp.T @ (Bp @ y)
        nw = float(np.linalg.norm(w))
        if nw == 0.0:
            return True, -math.inf
        log_norm += math.log(nw) - log_half_delta
        y = w / nw
    return log_norm <= 0.0, log_norm


def boosted_sparse_shrink(
    A: sp.csr_matrix,
    ell: int,
    draw_G,
    draw_x,
    next_vs_index,
    *,
    q: int,
    delta: float,
    max_attempts: int = 16,
    verify: bool = True,
    unit_roundoff: float = 2.0 ** -53,
    log: list | None = None,
) -> np.ndarray:
    """Alg 4 BoostedSparseShrink: repeat SparseShrink until VerifySpectral accepts.

    draw_G(attempt) -> d x ell start block; draw_x(attempt) -> unit vector in R^d;
    next_vs_index() -> the persistent VerifySpectral counter i after its increment (Alg 6).
    Delta = (||A'||_F^2 - ||B'||_F^2) / (alpha ell), alpha = 6/41; the verifier sees
    C = (A'^T A' - B'^T B') / (Delta/2).
    """
    d = A.shape[1]
    # stored duplicates of an entry add up (as they do in every product); ||A'||_F is the
    # norm of that summed matrix
    As = A.copy()
    As.sum_duplicates()
    fro_A = float(np.sum(As.data ** 2))
    for attempt in range(max_attempts):
        res = sparse_shrink(A, draw_G(attempt), ell, q)
        Bp = res["B"]
        fro_B = float(np.sum(Bp ** 2))
        S = fro_A - fro_B
        rec = {"attempt": attempt, "q": q, "S": S, "fro_A": fro_A, "lam_ell2": float(res["lam"][ell - 1] ** 2)}
        if S <= 64.0 * unit_roundoff * ell * fro_A:
            rec.update(accepted=True, reason="lossless")
            if log is not None:
                log.append(rec)
            return Bp
        if not verify:
            rec.update(accepted=True, reason="unverified")
            if log is not None:
                log.append(rec)
            return Bp
        Delta = S / (ALPHA * ell)
        i = next_vs_index()
        t = vs_steps(d, delta, i)
        ok, ln_norm = verify_spectral(A, Bp, Delta / 2.0, draw_x(attempt), t)
        rec.update(accepted=ok, reason="verified" if ok else "rejected", vs_index=i, t=t, ln_norm=ln_norm)
        if log is not None:
            log.append(rec)
        if ok:
            return Bp
    raise NoConvergence(f"BoostedSparseShrink: no accepted SparseShrink in {max_attempts} attempts")

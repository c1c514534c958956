"""Philox4x64-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11), written from its published definition with numpy uint64 arithmetic.

The paper draws its start block G from N(0,1) (Alg 1) and the VerifySpectral vector x
uniformly from the unit sphere (Alg 6) but fixes no generator.  A counter-based generator lets
the oracle and the GPU path draw the same numbers independently: each side implements this
one definition; the oracle's copy is pinned against ``numpy.random.Philox``.

Definition (4 words of 64 bits, key of 2 words, 10 rounds):

* round:  (hi0, lo0) = M0 * x0,  (hi1, lo1) = M1 * x2   (full 128-bit products)
          x <- (hi1 ^ x1 ^ k0,  lo1,  hi0 ^ x3 ^ k1,  lo0)
* key schedule: round r (0-based) uses (k0 + r*W0, k1 + r*W1) mod 2^64.
"""

from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
ROUNDS = 10

_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: np.uint64, b: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Full 128-bit product of the constant ``a`` and the uint64 array ``b``: (high, low)."""
    a_lo = a & _MASK32
    a_hi = a >> _S32
    b_lo = b & _MASK32
    b_hi = b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _MASK32) + (hl & _MASK32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    lo = a * b  # wraps mod 2^64
    return hi, lo


def philox4x64_10(counter, key) -> np.ndarray:
    """Apply the Philox4x64-10 bijection.

    counter: array-like of shape (4,) or (4, n), uint64 words (word 0 least significant).
    key:     two uint64 words.
    Returns a uint64 array of the same shape as ``counter``.
    """
    with np.errstate(over="ignore"):
        x = np.array(counter, dtype=np.uint64, copy=True)
        squeeze = x.ndim == 1
        if squeeze:
            x = x[:, None]
        k0 = np.uint64(key[0])
        k1 = np.uint64(key[1])
        x0, x1, x2, x3 = x[0], x[1], x[2], x[3]
        for _ in range(ROUNDS):
            hi0, lo0 = _mulhilo(M0, x0)
            hi1, lo1 = _mulhilo(M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
            k0 = k0 + W0
            k1 = k1 + W1
        out = np.stack([x0, x1, x2, x3])
    return out[:, 0] if squeeze else out


def philox_uniform01(words: np.ndarray) -> np.ndarray:
    """Map uint64 words to doubles in the open interval (0, 1): ((w >> 12) + 1/2) * 2^-52.

    The top 52 bits plus the half offset fit a double's 53-bit significand, so the map is exact
    (no rounding step for the two sides to disagree on) and keeps 0 and 1 out: log(u) is finite.
    """
    top = (np.asarray(words, dtype=np.uint64) >> np.uint64(12)).astype(np.float64)
    return (top + 0.5) * (2.0 ** -52)

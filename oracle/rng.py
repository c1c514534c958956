"""Random draws of the method, from a fixed counter schedule over Philox4x64-10.

The paper fixes only the distributions:
* SimultaneousIteration starts from G ~ N(0,1)^{d x k} (Alg 1);
* VerifySpectral picks x uniformly from the unit sphere in R^d (Alg 6).

Schedule (the same on the GPU side, which implements it independently):
* key     = (seed, stream_id)
* counter = (j, attempt, buffer, purpose), j = block index
* purpose: 0 = start block of a flushed buffer, 1 = VerifySpectral vector of a flushed buffer,
           2 / 3 = the same two draws for the pending buffer folded in by a query.
* element e of a row-major d x ell block (row = column id of A) comes from block e // 4, lane
  e % 4.  Each block's four words give four uniforms u0..u3 (see ``philox_uniform01``) and
  four normals by the Box-Muller transform on the pairs (u0, u1) and (u2, u3):
  sqrt(-2 ln u0) * cos(2 pi u1), sqrt(-2 ln u0) * sin(2 pi u1), and likewise for (u2, u3).
* x = g / ||g|| with g the first d normals of the VerifySpectral stream (a standard Gaussian
  vector normalised is uniform on the sphere).
"""

from __future__ import annotations

import numpy as np

from .philox import philox4x64_10, philox_uniform01

PURPOSE_SI = 0
PURPOSE_VS = 1
PURPOSE_QUERY_SI = 2
PURPOSE_QUERY_VS = 3


def normals(seed: int, stream_id: int, buffer_idx: int, attempt: int, purpose: int, count: int) -> np.ndarray:
    """The first ``count`` N(0,1) draws (FP64) of the stream keyed as in the module docstring."""
    nblocks = (count + 3) // 4
    ctr = np.empty((4, nblocks), dtype=np.uint64)
    ctr[0] = np.arange(nblocks, dtype=np.uint64)
    ctr[1] = np.uint64(attempt)
    ctr[2] = np.uint64(buffer_idx)
    ctr[3] = np.uint64(purpose)
    words = philox4x64_10(ctr, (np.uint64(seed), np.uint64(stream_id)))
    return box_muller(words).reshape(-1)[:count]


def box_muller(words: np.ndarray) -> np.ndarray:
    """Four N(0,1) draws per block of four Philox words (shape (4, n) -> (n, 4)).

    The words map to uniforms u0..u3 in (0, 1) (``philox_uniform01``); the Box-Muller transform
    takes the pairs (u0, u1) and (u2, u3): radius sqrt(-2 ln u0), angle 2 pi u1, giving
    (r cos, r sin), and the same for the second pair.
    """
    u = philox_uniform01(np.asarray(words, dtype=np.uint64).reshape(4, -1))
    r01 = np.sqrt(-2.0 * np.log(u[0]))
    r23 = np.sqrt(-2.0 * np.log(u[2]))
    t1 = 2.0 * np.pi * u[1]
    t3 = 2.0 * np.pi * u[3]
    z = np.empty((u.shape[1], 4), dtype=np.float64)
    z[:, 0] = r01 * np.cos(t1)
    z[:, 1] = r01 * np.sin(t1)
    z[:, 2] = r23 * np.cos(t3)
    z[:, 3] = r23 * np.sin(t3)
    return z


def start_block(seed: int, stream_id: int, buffer_idx: int, attempt: int, purpose: int, d: int, ell: int) -> np.ndarray:
    """G ~ N(0,1)^{d x ell} of SimultaneousIteration (Alg 1), row-major, FP64."""
    return normals(seed, stream_id, buffer_idx, attempt, purpose, d * ell).reshape(d, ell)


def sphere_vector(seed: int, stream_id: int, buffer_idx: int, attempt: int, purpose: int, d: int) -> np.ndarray:
    """x uniform on the unit sphere of R^d (Alg 6): a Gaussian vector divided by its norm."""
    g = normals(seed, stream_id, buffer_idx, attempt, purpose, d)
    return g / np.linalg.norm(g)

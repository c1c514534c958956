"""Pins of the oracle's random draws (Philox4x64-10, Box-Muller, sphere vector)."""

import numpy as np
import pytest
from scipy import stats

from oracle.philox import philox4x64_10, philox_uniform01
from oracle.rng import normals, sphere_vector, start_block

pytestmark = pytest.mark.cpu


def _numpy_block(key, counter):
    """Philox4x64-10 block at ``counter`` from numpy's implementation (a library routine).

    numpy advances its 256-bit counter before producing a block, so the block at c is the first
    output of a generator whose counter is c - 1.
    """
    c = 0
    for w in reversed(counter):
        c = (c << 64) | int(w)
    c = (c - 1) % (1 << 256)
    words = [(c >> (64 * i)) & ((1 << 64) - 1) for i in range(4)]
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(words, dtype=np.uint64))
    return bg.random_raw(4)


@pytest.mark.parametrize("key", [(0, 0), (1, 2), (2**64 - 1, 12345), (0xDEADBEEF, 7)])
@pytest.mark.parametrize("counter", [(0, 0, 0, 0), (1, 0, 0, 0), (5, 3, 2, 1), (2**64 - 1, 0, 9, 3), (17, 2**63, 1, 2)])
def test_philox_matches_numpy(key, counter):
    ours = philox4x64_10(np.array(counter, dtype=np.uint64), key)
    np.testing.assert_array_equal(ours, _numpy_block(key, counter))


def test_philox_vectorised_equals_scalar():
    rng = np.random.default_rng(3)
    ctr = rng.integers(0, 2**63, size=(4, 50), dtype=np.uint64)
    key = (11, 13)
    batch = philox4x64_10(ctr, key)
    for j in range(50):
        np.testing.assert_array_equal(batch[:, j], _numpy_block(key, ctr[:, j]))


def test_uniform_open_interval():
    w = np.array([0, 1, 2**12 - 1, 2**64 - 1, 2**63], dtype=np.uint64)
    u = philox_uniform01(w)
    assert np.all(u > 0) and np.all(u < 1)
    assert u[0] == 2.0**-53 and u[1] == u[0] and u[2] == u[0]
    assert u[3] == 1.0 - 2.0**-53
    assert u[4] == 0.5 + 2.0**-53


def test_normals_are_standard_gaussian():
    z = normals(7, 0, 0, 0, 0, 200_000)
    assert abs(z.mean()) < 0.01
    assert abs(z.var() - 1.0) < 0.01
    # Kolmogorov-Smirnov against N(0,1); each Box-Muller lane separately as well
    assert stats.kstest(z, "norm").pvalue > 1e-3
    for lane in range(4):
        assert stats.kstest(z[lane::4], "norm").pvalue > 1e-3
    # pairs from one block are uncorrelated
    assert abs(np.corrcoef(z[0::4], z[1::4])[0, 1]) < 0.02


def test_streams_differ_by_every_counter_word():
    base = normals(1, 2, 3, 4, 0, 64)
    for args in [(1, 2, 3, 5, 0), (1, 2, 4, 4, 0), (1, 2, 3, 4, 1), (1, 3, 3, 4, 0), (2, 2, 3, 4, 0)]:
        assert not np.allclose(base, normals(*args, 64))


def test_start_block_prefix_property():
    """Element e of the block depends only on e: a taller block extends a shorter one."""
    g1 = start_block(5, 0, 2, 1, 0, 10, 8)
    g2 = start_block(5, 0, 2, 1, 0, 37, 8)
    np.testing.assert_array_equal(g1, g2[:10])


def test_sphere_vector_uniform():
    d = 16
    xs = np.stack([sphere_vector(3, 0, b, 0, 1, d) for b in range(3000)])
    np.testing.assert_allclose(np.linalg.norm(xs, axis=1), 1.0, rtol=1e-14)
    # E[x] = 0 and E[x x^T] = I/d for the uniform law on the sphere
    assert np.abs(xs.mean(axis=0)).max() < 0.03
    np.testing.assert_allclose(xs.T @ xs / len(xs), np.eye(d) / d, atol=0.01)


def test_box_muller_exact_values_for_hand_picked_words():
    """Words whose uniforms have closed-form Box-Muller images, so the lane pairing (which uniform
    is the radius, which the angle), the cos/sin order and the uniform map are each pinned."""
    from oracle.rng import box_muller

    top = lambda k: np.uint64(k << 12)  # a word whose top 52 bits are k: u = (k + 1/2) 2^-52
    r_max = np.sqrt(106.0 * np.log(2.0))  # u = 2^-53 (k = 0): sqrt(-2 ln 2^-53)
    # radius word k = 0; angle words at u = 1/4 + 2^-53 (k = 2^50) and u = 1/2 + 2^-53 (k = 2^51)
    w = np.array([[top(0)], [top(1 << 50)], [top(0)], [top(1 << 51)]], dtype=np.uint64)
    z = box_muller(w)[0]
    eps = 2.0 * np.pi * 2.0 ** -53  # the angle's offset from pi/2 resp. pi
    # (the zeros of cos / sin are only zero to the rounding of 2 pi u: |z| <= 1e-14 r)
    assert abs(z[0]) <= 1e-14 * r_max                                       # cos(pi/2 + eps)
    np.testing.assert_allclose(z[1], r_max, rtol=1e-15)                     # sin(pi/2 + eps)
    np.testing.assert_allclose(z[2], -r_max, rtol=1e-15)                    # cos(pi + eps)
    assert abs(z[3]) <= 1e-14 * r_max                                       # sin(pi + eps)
    # radius word at u = 1 - 2^-53 (the largest word): r = sqrt(-2 ln(1 - 2^-53)) = 2^-26 (1 + ...)
    # angle word 0: u = 2^-53, cos = 1, sin = 2 pi 2^-53
    w = np.array([[np.uint64(2**64 - 1)], [np.uint64(0)], [np.uint64(2**64 - 1)], [top(3 << 50)]], dtype=np.uint64)
    z = box_muller(w)[0]
    np.testing.assert_allclose(z[0], 2.0 ** -26, rtol=1e-12)
    np.testing.assert_allclose(z[1], 2.0 ** -26 * eps, rtol=1e-12)
    assert abs(z[2]) <= 1e-14 * 2.0 ** -26                                 # cos(3 pi / 2 + eps)
    np.testing.assert_allclose(z[3], -(2.0 ** -26), rtol=1e-12)           # sin(3 pi / 2 + eps)
    # the start block is built from exactly these four lanes per Philox block, in this order
    from oracle.philox import philox4x64_10

    blk = philox4x64_10(np.array([0, 2, 3, 0], dtype=np.uint64), (5, 1))
    np.testing.assert_array_equal(start_block(5, 1, 3, 2, 0, 1, 4)[0], box_muller(blk[:, None])[0])

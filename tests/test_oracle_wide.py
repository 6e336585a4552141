"""Pins of the oracle's 64-bit keys (the wide records of the Experiments
section) and of its move counter (a swap is three moves, Experiments).

The 64-bit build is the same C source compiled for uint64 keys, so on keys
that fit in 32 bits it must take exactly the 32-bit build's steps: the same
order, the same comparison and move counts.  Against libraries: numpy.sort
for uint64, an independently written IEEE-754 totalOrder key for float64."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1804_10062_amd import inputs


def _total_order_f64(x: np.ndarray) -> np.ndarray:
    """Indices sorting float64 by totalOrder: sign-magnitude bits as a
    signed integer (negative values: -(magnitude) - 1)."""
    b = x.view(np.uint64)
    mag = (b & np.uint64(0x7FFFFFFFFFFFFFFF)).astype(object)
    neg = (b >> np.uint64(63)).astype(bool)
    key = [-(int(m)) - 1 if n else int(m) for m, n in zip(mag, neg)]
    return np.array(sorted(range(x.size), key=lambda i: key[i]), dtype=np.int64)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 17, 1000, 65537])
def test_u64_matches_numpy(n):
    rng = np.random.default_rng(n)
    for x in (rng.integers(0, 2 ** 64, n, dtype=np.uint64),
              rng.integers(0, 5, n).astype(np.uint64) << np.uint64(40),
              np.arange(n, dtype=np.uint64)[::-1].copy()):
        k, _, _ = oracle.sort(x)
        assert k.dtype == np.uint64
        np.testing.assert_array_equal(k, np.sort(x))


def test_f64_total_order_with_specials():
    rng = np.random.default_rng(5)
    x = rng.standard_normal(3000)
    x[:8] = [0.0, -0.0, np.inf, -np.inf, np.nan, -np.nan, 5e-324, -5e-324]
    k, _, _ = oracle.sort(x)
    want = x[_total_order_f64(x)]
    np.testing.assert_array_equal(k.view(np.uint64), want.view(np.uint64))


@pytest.mark.parametrize("kind", ["uniform", "sorted_swaps", "zipf", "reverse", "equal"])
def test_64_bit_build_takes_the_32_bit_steps(kind):
    """Keys below 2^32, zero-extended: identical order, payload order and
    counters (comparisons and moves) in both builds."""
    x = inputs.make_keys(kind, 20011, seed=7)
    v = np.arange(x.size, dtype=np.uint32)
    k32, v32, c32 = oracle.sort(x, v)
    k64, v64, c64 = oracle.sort(x.astype(np.uint64), v)
    np.testing.assert_array_equal(k64, k32.astype(np.uint64))
    np.testing.assert_array_equal(v64, v32)
    assert c64 == c32
    kx32, _, cx32 = oracle.sort_x(x, x_thresh=100)
    kx64, _, cx64 = oracle.sort_x(x.astype(np.uint64), x_thresh=100)
    np.testing.assert_array_equal(kx64, kx32.astype(np.uint64))
    assert cx64 == cx32


def test_f64_of_f32_values_takes_the_f32_steps():
    """float32 values widened to float64 keep their order, so the binary64
    build must compare and move exactly as the binary32 build."""
    x = inputs.normal_f32(12345, seed=3)
    k32, _, c32 = oracle.sort(x)
    k64, _, c64 = oracle.sort(x.astype(np.float64))
    np.testing.assert_array_equal(k64, k32.astype(np.float64))
    assert c64 == c32


def test_all_permutations_u64_high_bits():
    """Keys that differ only above bit 32 sort correctly (the comparison
    really uses all 64 bits)."""
    for n in range(0, 8):
        for perm in itertools.permutations(range(n)):
            x = (np.array(perm, dtype=np.uint64) << np.uint64(33)) | np.uint64(7)
            k, _, _ = oracle.sort(x)
            assert (k >> np.uint64(33)).tolist() == list(range(n))


def test_segments_u64():
    rng = np.random.default_rng(9)
    lens = np.array([0, 1, 2, 50, 3001, 7], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    x = rng.integers(0, 2 ** 64, int(off[-1]), dtype=np.uint64)
    k, _, _ = oracle.sort_segments(x, off)
    for j in range(lens.size):
        a, b = int(off[j]), int(off[j + 1])
        np.testing.assert_array_equal(k[a:b], np.sort(x[a:b]))


def test_move_counter_swap_is_three_moves():
    """Experiments section: a swap of two elements counts as three moves.
    msort of one element into a target cell is exactly one swap; a merge of
    one run1 element into an empty run2 is one exchange: also three moves."""
    x = np.array([5, 9], dtype=np.uint32)
    k, _, c = oracle.msort(x, 0, 1, 1)
    assert k.tolist() == [9, 5] and c.moves == 3 and c.comparisons == 0
    k, _, c = oracle.merge(np.array([4, 8], dtype=np.uint32), 0, 1, 1, 2)
    assert k[1] == 4 and c.moves == 3 and c.comparisons == 0

"""Host-side checks of the number-theoretic facts the key/payload base case
relies on, emulated in numpy (no device code runs here):

* an element with bit 52 set, the key in bits 13..44 and a tile index below
  2^13 in bits 0..12 is a positive normal double, and its order as a double
  is the lexicographic order of (key, index);
* complementing bits 0..44 reverses that order and keeps every element a
  positive normal double;
* with the elements of the lanes whose mask bit is set negated, the double
  minimum of the own element and the negated partner is the smaller element
  in the lower lane and the negated larger one in the upper lane."""
import numpy as np

IBITS = 13
FLIP = (1 << (32 + IBITS)) - 1
EXP1 = 1 << 52
SIGN = 1 << 63


def encode(keys: np.ndarray, idx: np.ndarray) -> np.ndarray:
    return (np.uint64(EXP1) | (keys.astype(np.uint64) << np.uint64(IBITS))
            | idx.astype(np.uint64))


def as_double(bits: np.ndarray) -> np.ndarray:
    return bits.view(np.float64)


def _sample(n: int, seed: int):
    rng = np.random.default_rng(seed)
    # keys from the whole range with the extremes and many ties
    keys = rng.integers(0, 1 << 32, n, dtype=np.uint64)
    keys[: n // 4] = rng.choice(np.array([0, 1, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFE,
                                          0xFFFFFFFF], dtype=np.uint64), n // 4)
    idx = rng.integers(0, 1 << IBITS, n, dtype=np.uint64)
    return keys, idx


def test_encoding_is_positive_normal_and_ordered():
    keys, idx = _sample(200000, 1)
    e = encode(keys, idx)
    d = as_double(e)
    assert np.all(np.isfinite(d)) and np.all(d > 0)
    assert np.all(np.abs(d) >= np.finfo(np.float64).tiny)  # normal, not subnormal
    # order as doubles == lexicographic (key, index) order == integer order
    by_double = np.argsort(d, kind="stable")
    by_pair = np.lexsort((idx, keys))
    assert np.array_equal(e[by_double], e[by_pair])
    assert np.array_equal(np.sort(e), e[by_pair])
    # key and index are recovered from the element
    assert np.array_equal((e >> np.uint64(IBITS)) & np.uint64(0xFFFFFFFF), keys)
    assert np.array_equal(e & np.uint64((1 << IBITS) - 1), idx)


def test_padding_sorts_after_every_real_element_of_the_tile():
    # padding of tile position i: key 0xFFFFFFFF with index i >= the real length
    n_real = 5000
    keys = np.full(n_real, 0xFFFFFFFF, dtype=np.uint64)
    real = encode(keys, np.arange(n_real, dtype=np.uint64))
    pad = encode(np.full(8192 - n_real, 0xFFFFFFFF, dtype=np.uint64),
                 np.arange(n_real, 8192, dtype=np.uint64))
    assert as_double(real).max() < as_double(pad).min()


def test_complement_reverses_the_order():
    keys, idx = _sample(100000, 2)
    e = np.unique(encode(keys, idx))  # a tile's elements are distinct (own indices)
    c = e ^ np.uint64(FLIP)
    dc = as_double(c)
    assert np.all(np.isfinite(dc)) and np.all(dc >= np.finfo(np.float64).tiny)
    order = np.argsort(as_double(e), kind="stable")
    assert np.all(np.diff(dc[order]) < 0)  # strictly reversed (elements are distinct)
    assert np.array_equal(c ^ np.uint64(FLIP), e)


def test_signed_minimum_keeps_each_lanes_side():
    keys, idx = _sample(100000, 3)
    e = encode(keys, idx)
    x, y = e[0::2], e[1::2]  # x in the lower lane, y in the upper lane
    lo_own = as_double(x)
    hi_own = as_double(y ^ np.uint64(SIGN))  # upper lane holds its element negated
    # each lane reads the partner's register as it is and negates it
    lower_kept = np.minimum(lo_own, -hi_own)
    upper_kept = np.minimum(hi_own, -lo_own)
    want_min = np.minimum(as_double(x), as_double(y))
    want_max = np.maximum(as_double(x), as_double(y))
    assert np.array_equal(lower_kept, want_min)
    assert np.array_equal(-upper_kept, want_max)
    # bit-exact: the kept values are the inputs' bit patterns, sign restored
    assert np.array_equal(lower_kept.view(np.uint64), np.minimum(x, y))
    assert np.array_equal(upper_kept.view(np.uint64) ^ np.uint64(SIGN), np.maximum(x, y))

"""The pass structure of the in-place bitonic network that finishes the
loop's last ranges (the library's final X), simulated on the CPU.

The library sorts tiles of T = 2^lt keys with the base case and then runs,
for every stage k > lt, a mirror step (position i against i ^ (2^k - 1))
together with the first (up to four) half-cleaner steps 2^(k-2) .. in one
pass, the further half-cleaner steps down to T four at a time, and the steps
below T inside the tiles, all ascending; positions at or past the range's
end act as +infinity.  This file replays exactly that sequence of
compare-exchanges with numpy and checks that it sorts ranges of any
length, including every 0-1 input of small lengths (the 0-1 principle: a
comparator network that sorts all 0-1 inputs sorts every input).
"""
import itertools
import math

import numpy as np
import pytest


def network_passes(K: int, lt: int):
    """(kind, k, lo, hi) in launch order, as the library builds them."""
    out = []
    for k in range(lt + 1, K + 1):
        hi = k - 2
        if hi < lt:
            out.append(("mirror", k, 0, 0))
        else:
            out.append(("mirror_columns", k, max(lt, hi - 3), hi))
            hi -= 4
        while hi >= lt:
            out.append(("columns", k, max(lt, hi - 3), hi))
            hi -= 4
        out.append(("tile", k, 0, 0))
    return out


def _cmpx(x: np.ndarray, i: np.ndarray, p: np.ndarray) -> None:
    """Ascending compare-exchange of the pairs (i, p), i < p; pairs whose
    upper position lies outside the range are left alone (+infinity)."""
    ok = p < x.size
    i, p = i[ok], p[ok]
    a, b = x[i].copy(), x[p].copy()
    sw = b < a
    x[i[sw]], x[p[sw]] = b[sw], a[sw]


def _half_cleaner(x: np.ndarray, j: int) -> None:
    n = x.size
    i = np.arange(n)
    i = i[(i & j) == 0]
    _cmpx(x, i, i + j)


def run_network(keys, lt: int) -> np.ndarray:
    x = np.array(keys, copy=True)
    m, T = x.size, 1 << lt
    for t0 in range(0, m, T):  # the base case
        x[t0:t0 + T] = np.sort(x[t0:t0 + T])
    if m <= T:
        return x
    K = math.ceil(math.log2(m))
    for kind, k, lo, hi in network_passes(K, lt):
        if kind in ("mirror", "mirror_columns"):
            i = np.arange(m)
            i = i[(i >> (k - 1)) & 1 == 0]
            _cmpx(x, i, i ^ ((1 << k) - 1))
        if kind in ("columns", "mirror_columns"):
            for s in range(hi, lo - 1, -1):
                _half_cleaner(x, 1 << s)
        else:
            for s in range(lt - 1, -1, -1):
                _half_cleaner(x, 1 << s)
    return x


def test_pass_order_covers_every_step_once():
    """Stage k: one mirror step first, then the half-cleaners 2^(k-2) ..
    2^0, each exactly once and in decreasing order; the mirror shares a pass
    with the first of them whenever one lies above the tile."""
    lt = 4
    for K in range(lt + 1, 14):
        for k in range(lt + 1, K + 1):
            steps = []
            kinds = [kind for kind, kk, *_ in network_passes(K, lt) if kk == k]
            assert kinds[0] == ("mirror" if k - 2 < lt else "mirror_columns")
            assert kinds.count("mirror") + kinds.count("mirror_columns") == 1
            for kind, kk, lo, hi in network_passes(K, lt):
                if kk != k:
                    continue
                if kind in ("columns", "mirror_columns"):
                    assert 1 <= hi - lo + 1 <= 4 and lo >= lt
                    steps += list(range(hi, lo - 1, -1))
                elif kind == "tile":
                    steps += list(range(lt - 1, -1, -1))
            assert steps == list(range(k - 2, -1, -1))


@pytest.mark.parametrize("lt", [1, 2, 3])
def test_all_zero_one_inputs(lt):
    for n in range(1, 13):
        for bits in itertools.product((0, 1), repeat=n):
            x = np.array(bits, dtype=np.uint8)
            assert np.array_equal(run_network(x, lt), np.sort(x)), (lt, bits)


@pytest.mark.parametrize("lt", [2, 4, 6])
def test_random_lengths(lt):
    rng = np.random.default_rng(lt)
    for m in list(range(1, 70)) + [int(v) for v in rng.integers(70, 5000, 40)] + [1 << 12, (1 << 12) + 1, (1 << 12) - 1]:
        x = rng.integers(0, 1 << 32, m, dtype=np.uint64).astype(np.uint32)
        assert np.array_equal(run_network(x, lt), np.sort(x)), m
        y = rng.integers(0, 3, m).astype(np.uint32)  # many equal keys
        assert np.array_equal(run_network(y, lt), np.sort(y)), m


def test_reverse_and_sorted():
    for m in (257, 1000, 4096, 4097):
        x = np.arange(m, dtype=np.uint32)[::-1]
        assert np.array_equal(run_network(x, 4), np.arange(m, dtype=np.uint32))
        assert np.array_equal(run_network(np.arange(m, dtype=np.uint32), 4),
                              np.arange(m, dtype=np.uint32))

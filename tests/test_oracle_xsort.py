"""Pins of the oracle's QuickMergeXsort (Sec. "QuickMergeXsort") and of its
X = CleverQuicksort (median-of-3 Quicksort, Introduction).

The chain: (1) brute force over every permutation of up to 8 elements gives
averages equal to exact average-case recurrences, written here from the
proofs (pivot rank k with probability (k-1)(n-k)/C(n,3), n comparisons per
partition of n >= 3 elements, both sides random; msort hands ranges shorter
than X_THRESH to X); (2) the recurrences, evaluated at large n, approach
the paper's constants: (12/7) ln 2 ~ 1.188 for X and (1 + alpha)/2 ~ 1.094
for Mergesort with X called at sqrt(n) elements (Theorem "Average-Case
QuickMergeXsort", beta = 1/2); (3) the oracle's own counts over random
permutations grow with those slopes; (4) X_THRESH = 2 is QuickMergesort.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from tests.test_oracle_pins import _merge_avg, qms_recurrence

ALPHA = 12.0 / 7.0 * math.log(2.0)  # CleverQuicksort's leading constant


def cqs_recurrence(N):
    """Average comparisons of median-of-3 Quicksort: Q(n) = n + 2 / C(n,3) *
    sum_j j (n-1-j) Q(j) for n >= 3 (pivot rank k = j + 1 leaves sides j and
    n-1-j; both recursions contribute the same sum), Q(2) = 1.  Prefix sums
    of j Q(j) and j^2 Q(j) make it linear in N."""
    Q = np.zeros(N + 1)
    if N >= 2:
        Q[2] = 1.0
    s1 = 2.0 * Q[2]      # sum_{j<n} j Q(j) at n = 3
    s2 = 4.0 * Q[2]      # sum_{j<n} j^2 Q(j) at n = 3
    for n in range(3, N + 1):
        Q[n] = n + 2.0 * ((n - 1) * s1 - s2) / math.comb(n, 3)
        s1 += n * Q[n]
        s2 += n * n * Q[n]
    return Q


def msort_x_avg(m, xt, Q, memo):
    """Average comparisons of Fig. 2's msort on m random elements with X
    below xt: X's average when m < xt, else the two halves (q = m/2) and the
    merge of runs of q and m - q."""
    if m < xt:
        return Q[m]
    if m in memo:
        return memo[m]
    q = m // 2
    v = msort_x_avg(q, xt, Q, memo) + msort_x_avg(m - q, xt, Q, memo) + _merge_avg(q, m - q)
    memo[m] = v
    return v


def out_x_avg(m, xt, Q, memo):
    """Fig. 2's out on m elements: msort of both halves and one merge."""
    if m < 2:
        return 0.0
    q = m // 2
    return (msort_x_avg(m - q, xt, Q, memo) + msort_x_avg(q, xt, Q, memo)
            + _merge_avg(m - q, q))


def qmxs_recurrence(N, xt):
    """T(n) = n + sum_k P(k) [ out(smaller side) + T(larger side) ] with the
    side test of the QuickMergesort loop, T(2) = 1."""
    Q = cqs_recurrence(max(N, xt))
    memo = {}
    O = np.array([out_x_avg(m, xt, Q, memo) for m in range(N + 1)])
    T = np.zeros(N + 1)
    if N >= 2:
        T[2] = 1.0
    for n in range(3, N + 1):
        k = np.arange(1, n + 1)
        p = (k - 1) * (n - k) / math.comb(n, 3)
        left, right = k - 1, n - k
        val = np.where(left < n // 2, O[left] + T[right], O[right] + T[left])
        T[n] = n + float((p * val).sum())
    return T


def test_cqs_recurrence_prefix_sums_match_direct_sum():
    Q = cqs_recurrence(200)
    for n in (3, 4, 7, 50, 63, 64, 65, 200):
        k = np.arange(1, n + 1)
        p = (k - 1) * (n - k) / math.comb(n, 3)
        direct = n + float((p * (Q[k - 1] + Q[n - k])).sum())
        assert abs(direct - Q[n]) < 1e-9 * n, n


def test_clever_quicksort_all_permutations_exact_average():
    Q = cqs_recurrence(8)
    for n in range(0, 9):
        total = count = 0
        for perm in itertools.permutations(range(n)):
            s, _, c = oracle.clever_quicksort(np.array(perm, dtype=np.uint32))
            assert s.tolist() == list(range(n)), perm
            total += c.comparisons
            count += 1
        assert abs(total / count - Q[n]) < 1e-9, (n, total / count, Q[n])


@pytest.mark.parametrize("xt", [3, 4, 5, 9])
def test_quickmergexsort_all_permutations_exact_average(xt):
    T = qmxs_recurrence(8, xt)
    for n in range(2, 9):
        total = count = 0
        for perm in itertools.permutations(range(n)):
            s, _, c = oracle.sort_x(np.array(perm, dtype=np.uint32), x_thresh=xt)
            assert s.tolist() == list(range(n)), perm
            total += c.comparisons
            count += 1
        assert abs(total / count - T[n]) < 1e-9, (xt, n, total / count, T[n])


@pytest.mark.parametrize("xt", [2, 3, 5, 9])
def test_msort_with_x_all_permutations_exact_average(xt):
    """msort of 8 elements into 8 buffer cells, over all 8! orders: the
    average equals the msort recurrence with X below xt (xt = 9: X sorts
    the whole range; 5: X on two halves of 4; 3: on pairs; 2: Mergesort),
    and the buffer elements end up where the data were."""
    Q = cqs_recurrence(16)
    m = 8
    total = count = 0
    buf = np.arange(100, 100 + m, dtype=np.uint32)
    for perm in itertools.permutations(range(m)):
        a = np.concatenate([np.array(perm, dtype=np.uint32), buf])
        k, _, c = oracle.msort_x(a, 0, m, m, xt)
        assert k[m:].tolist() == list(range(m)), perm
        assert sorted(k[:m].tolist()) == buf.tolist()
        total += c.comparisons
        count += 1
    assert abs(total / count - msort_x_avg(m, xt, Q, {})) < 1e-9


def test_msort_x_distinguishes_x_from_mergesort():
    """The enumeration above separates X from Mergesort: on 8 elements, X on
    the whole range (xt = 9) or on halves of 4 (xt = 5) costs more on average
    than Mergesort (xt = 2; xt = 3 hands X only pairs, one comparison each,
    the same as Mergesort)."""
    Q = cqs_recurrence(16)
    v = {xt: msort_x_avg(8, xt, Q, {}) for xt in (2, 3, 5, 9)}
    assert v[2] == v[3] < v[5] < v[9], v


def test_threshold_2_recurrence_is_quickmergesort():
    """With X_THRESH = 2 the X recurrence collapses onto Theorem 1's."""
    assert np.allclose(qmxs_recurrence(60, 2)[2:], qms_recurrence(60)[2:], rtol=1e-12)


def test_cqs_leading_constant():
    """Introduction: CleverQuicksort averages (12/7) ln 2 n lg n + O(n); the
    doubling difference (Q(2n) - 2 Q(n)) / (2n) isolates the constant."""
    n = 1 << 18
    Q = cqs_recurrence(2 * n)
    assert abs((Q[2 * n] - 2 * Q[n]) / (2 * n) - ALPHA) < 2e-3


def test_mergexsort_at_sqrt_n_leading_constant():
    """Proof of Theorem "Average-Case QuickMergeXsort": Mergesort with X at
    ceil(n^beta) elements averages (alpha beta + 1 - beta) n lg n + O(n); at
    beta = 1/2 and n = 4^k the O(n) term is c n, so (M(4n) - 4 M(n)) / (8n)
    is the constant (1 + alpha) / 2 ~ 1.094."""
    n = 4 ** 10
    Q = cqs_recurrence(2 * int(math.isqrt(4 * n)) + 2)
    m1 = msort_x_avg(n, int(math.isqrt(n)), Q, {})
    m4 = msort_x_avg(4 * n, int(math.isqrt(4 * n)), Q, {})
    assert abs((m4 - 4 * m1) / (8 * n) - (1 + ALPHA) / 2) < 0.01


def _slopes(ns, runs, seed):
    """Least-squares slope of mean comparisons / n against lg n."""
    rng = np.random.default_rng(seed)
    ys = {"cqs": [], "qms": [], "qmqs": []}
    for n in ns:
        acc = dict.fromkeys(ys, 0)
        for _ in range(runs):
            x = rng.permutation(n).astype(np.uint32)
            acc["cqs"] += oracle.clever_quicksort(x)[2].comparisons
            acc["qms"] += oracle.sort(x)[2].comparisons
            acc["qmqs"] += oracle.sort_x(x)[2].comparisons
        for k in ys:
            ys[k].append(acc[k] / runs / n)
    return {k: float(np.polyfit(np.log2(ns), v, 1)[0]) for k, v in ys.items()}


def test_oracle_counts_grow_with_the_papers_constants():
    """The oracle itself, averaged over random permutations of n = 4^5..4^8:
    CleverQuicksort ~ 1.188 n lg n; QuickMergesort ~ 1.0 n lg n (Theorem 1);
    QuickMergeXsort with X at sqrt(n) between them, near 1.094 (at these
    sizes X's blocks hold 16..128 keys and the measured slope sits about
    0.02 below the asymptotic constant)."""
    s = _slopes([4 ** k for k in range(5, 9)], 64, 20)
    assert abs(s["cqs"] - ALPHA) < 0.03, s
    assert abs(s["qms"] - 1.0) < 0.04, s
    assert 1.044 < s["qmqs"] < 1.124, s
    assert s["qms"] + 0.03 < s["qmqs"] < s["cqs"] - 0.03, s


def test_threshold_2_is_quickmergesort_bit_for_bit():
    rng = np.random.default_rng(3)
    cases = [rng.integers(0, 2 ** 32, 1000, dtype=np.uint64).astype(np.uint32),
             rng.integers(0, 4, 777).astype(np.uint32),
             np.arange(500, dtype=np.uint32)[::-1].copy(),
             rng.standard_normal(333).astype(np.float32)]
    for x in cases:
        v = np.arange(x.size, dtype=np.uint32)
        a = oracle.sort(x, v)
        b = oracle.sort_x(x, v, x_thresh=2)
        assert a[0].view(np.uint32).tolist() == b[0].view(np.uint32).tolist()
        assert a[1].tolist() == b[1].tolist()
        assert a[2] == b[2]


@pytest.mark.parametrize("xt", [3, 5, 17, 64, None, 10 ** 6])
def test_sort_x_sorts_any_threshold(xt):
    rng = np.random.default_rng(xt or 0)
    for x in (rng.integers(0, 2 ** 32, 3001, dtype=np.uint64).astype(np.uint32),
              rng.integers(0, 3, 2000).astype(np.uint32),
              np.zeros(100, dtype=np.uint32),
              np.arange(1500, dtype=np.uint32)):
        v = np.arange(x.size, dtype=np.uint32)
        k, vv, _ = oracle.sort_x(x, v, x_thresh=xt)
        assert k.tolist() == np.sort(x).tolist()
        # payloads travel with their keys: (key, payload) pairs are preserved
        assert sorted(zip(k.tolist(), vv.tolist())) == sorted(zip(x.tolist(), v.tolist()))
    f = rng.standard_normal(999).astype(np.float32)
    f[:4] = [0.0, -0.0, np.inf, -np.inf]
    k, _, _ = oracle.sort_x(f, x_thresh=xt)
    order = np.argsort(np.where(f.view(np.uint32) >= 2 ** 31, ~f.view(np.uint32),
                                f.view(np.uint32) | np.uint32(2 ** 31)), kind="stable")
    assert k.view(np.uint32).tolist() == f[order].view(np.uint32).tolist()

"""The worst-case pivot of HybridQuickMergesort on the GPU (through the C ABI).

Sec. "Worst-Case Efficient QuickMergeSort": after a round whose pivot fell
outside [n/16, 15n/16], the next pivot is the median of the n/3 medians of
three (MoMQuickMergesort's pivot), then median-of-3 again.  The pivot the GPU
selects (qms_mom_pivot, the kernels the sort uses) must equal the oracle's bit
for bit; inside a sort, every such round must split with the guarantee of the
section (at least 2 floor(s/6) keys on each side of the pivot), and the sorted
output must still equal the oracle's.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1804_10062_amd import inputs, qms  # noqa: E402
from tests.gpu_helpers import to_device, to_host  # noqa: E402

pytestmark = pytest.mark.gpu
needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")


def _pivot_parity(x):
    got = qms.qms_mom_pivot(to_device(x))
    assert got == oracle.mom_pivot(x), (x.size, got, oracle.mom_pivot(x))


@needs_gpu
@pytest.mark.parametrize("n", [3, 4, 5, 6, 7, 100, 8191, 24575, 24576, 24577, 100003, 1 << 20])
def test_mom_pivot_uniform_sizes(n):
    _pivot_parity(inputs.uniform_u32(n, seed=n))


@needs_gpu
@pytest.mark.parametrize("kind", ["sorted", "reverse", "sorted_swaps", "zipf", "equal"])
def test_mom_pivot_structured(kind):
    _pivot_parity(inputs.make_keys(kind, 300007, seed=5))


@needs_gpu
def test_mom_pivot_few_values_and_extremes():
    rng = np.random.default_rng(3)
    _pivot_parity(rng.integers(0, 3, 99999).astype(np.uint32))
    _pivot_parity(rng.choice(np.array([0, 1, 0xFFFFFFFE, 0xFFFFFFFF], dtype=np.uint32), 50001))


@needs_gpu
def test_mom_pivot_f32():
    _pivot_parity(inputs.normal_f32(123457, seed=8))
    specials = np.array([0.0, -0.0, np.inf, -np.inf, 1e-45, -1e-45, 3.4e38, -3.4e38],
                        dtype=np.float32)
    rng = np.random.default_rng(4)
    _pivot_parity(rng.permutation(np.tile(specials, 1001)))


@needs_gpu
def test_mom_pivot_full_size_2_26():
    _pivot_parity(inputs.uniform_u32(1 << 26, seed=2))


def _wide_to_device(x):
    if x.dtype == np.float64:
        return torch.from_numpy(np.ascontiguousarray(x)).cuda()
    return torch.from_numpy(np.ascontiguousarray(x).view(np.int64)).cuda()


@needs_gpu
@pytest.mark.parametrize("n", [3, 7, 100, 8191, 24577, 100003, 1 << 20])
def test_mom_pivot_u64(n):
    """64-bit keys: eight 8-bit digit passes of the select, bit-exact with the
    oracle's 64-bit build (keys spread over all 64 bits, and keys that differ
    only in the upper word)."""
    rng = np.random.default_rng(n)
    x = rng.integers(0, 2 ** 64, n, dtype=np.uint64)
    assert qms.qms_mom_pivot(_wide_to_device(x)) == oracle.mom_pivot(x)
    hi = rng.integers(0, 5, n, dtype=np.uint64) << np.uint64(40)
    y = hi | np.uint64(7)
    assert qms.qms_mom_pivot(_wide_to_device(y)) == oracle.mom_pivot(y)


@needs_gpu
def test_mom_pivot_f64():
    rng = np.random.default_rng(9)
    x = rng.standard_normal(200003)
    assert qms.qms_mom_pivot(_wide_to_device(x)) == oracle.mom_pivot(x)
    specials = np.array([0.0, -0.0, np.inf, -np.inf, 5e-324, -5e-324, 1.7e308, -1.7e308],
                        dtype=np.float64)
    y = rng.permutation(np.tile(specials, 1001))
    assert qms.qms_mom_pivot(_wide_to_device(y)) == oracle.mom_pivot(y)


@needs_gpu
def test_mom_pivot_log_order_is_the_integer_pivot():
    """Under the logarithm comparison the order is the integers' own, so the
    pivot is the plain uint32 one."""
    x = inputs.uniform_u32(100003, seed=12)
    got = qms.qms_mom_pivot(to_device(x), dtype=qms.QMS_U32_LOG)
    assert got == oracle.mom_pivot(x)


@needs_gpu
def test_mom_pivot_rejects_short_input():
    t = to_device(np.array([1, 2], dtype=np.uint32))
    with pytest.raises(qms.QmsError):
        qms.qms_mom_pivot(t)


def _bad_first_round(n, seed):
    """Distinct keys whose median-of-3 sample (first, middle, last) holds the
    three smallest keys: the first round splits off a single key."""
    x = np.random.default_rng(seed).permutation(n).astype(np.int64) + 3
    x[0], x[n // 2], x[n - 1] = 0, 1, 2
    return x.astype(np.uint32)


@needs_gpu
@pytest.mark.parametrize("n", [100003, 1 << 20])
def test_hqms_round_after_bad_split(n):
    x = _bad_first_round(n, seed=n)
    t = to_device(x)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_host(t), np.sort(x))
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(to_host(t), want)
    sched = qms.qms_last_schedule()
    assert sched[0][5] == 0 and min(sched[0][1], sched[0][3]) * 16 < sched[0][0]
    assert sched[1][5] == 1, sched[:3]
    prev_bad = False
    for (s, lt, eq, gt, levels, rule) in sched:
        # the rule follows the previous round's balance
        assert rule == (1 if prev_bad else 0)
        if rule == 1:
            # distinct keys: the pivot itself is the only key equal to it
            assert lt + eq >= 2 * (s // 6) - 1 and gt + eq >= 2 * (s // 6) - 1, (s, lt, eq, gt)
        prev_bad = min(lt, gt) * 16 < s


@needs_gpu
@pytest.mark.parametrize("kind", ["organ_pipe", "sawtooth", "interleaved"])
def test_hqms_structured_rules(kind):
    n = 1 << 21
    i = np.arange(n, dtype=np.int64)
    if kind == "organ_pipe":
        x = np.minimum(i, n - 1 - i)
    elif kind == "sawtooth":
        x = i % 1000
    else:
        x = np.where(i % 2 == 0, i, n - i)
    x = (x * 16).astype(np.uint32)
    t = to_device(x)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(to_host(t), want)
    prev_bad = False
    for (s, lt, eq, gt, levels, rule) in qms.qms_last_schedule():
        assert rule == (1 if prev_bad else 0)
        prev_bad = min(lt, gt) * 16 < s

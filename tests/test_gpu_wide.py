"""64-bit keys on the GPU (the wide records of the Experiments section):
uint64 and float64 (IEEE-754 total order) through qms_sort and
qms_sort_batch, bit-exact with the oracle's 64-bit build."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1804_10062_amd import autotune, inputs, qms  # noqa: E402

pytestmark = pytest.mark.gpu
needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")


@pytest.fixture(autouse=True)
def _restore_defaults():
    yield
    if torch.cuda.is_available():
        autotune.reset_tuning()


def dev64(x: np.ndarray) -> torch.Tensor:
    if x.dtype == np.float64:
        return torch.from_numpy(np.ascontiguousarray(x)).cuda()
    assert x.dtype == np.uint64
    return torch.from_numpy(np.ascontiguousarray(x).view(np.int64)).cuda()


def host64(t: torch.Tensor) -> np.ndarray:
    a = t.cpu().numpy()
    return a if a.dtype == np.float64 else a.view(np.uint64)


def u64_keys(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).integers(0, 2 ** 64, n, dtype=np.uint64)


@needs_gpu
@pytest.mark.parametrize("n", [0, 1, 2, 3, 100, 8191, 8192, 8193, 65537, 300007, 1 << 20])
def test_u64_matches_oracle(n):
    x = u64_keys(n, seed=n % 101)
    t = dev64(x)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(host64(t), want)


@needs_gpu
@pytest.mark.parametrize("kind", ["sorted", "reverse", "sorted_swaps", "zipf", "equal"])
def test_u64_structured_and_high_bits(kind):
    """Structured 32-bit inputs moved into the high word, with random low
    words, and keys that differ only above bit 32."""
    base = inputs.make_keys(kind, 200003, seed=4).astype(np.uint64)
    lo = np.random.default_rng(1).integers(0, 16, base.size).astype(np.uint64)
    for x in (base << np.uint64(32) | lo, base << np.uint64(32)):
        t = dev64(x)
        qms.qms_sort(t)
        torch.cuda.synchronize()
        want, _, _ = oracle.sort(x, counted=False)
        np.testing.assert_array_equal(host64(t), want)


@needs_gpu
@pytest.mark.parametrize("n", [5, 9000, 262147])
def test_f64_total_order(n):
    x = np.random.default_rng(n).standard_normal(n)
    x[:5] = [0.0, -0.0, np.inf, -np.inf, np.nan][:min(5, n)]
    if n > 8:
        x[5:9] = [-np.nan, 5e-324, -5e-324, 1e308]
    t = dev64(x)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(host64(t).view(np.uint64), want.view(np.uint64))


@needs_gpu
@pytest.mark.parametrize("tuning", [(4, 4096, 16384, 16384), (2, 8192, 32768, 2048),
                                    (4, 4096, 16384, 4096)])
def test_u64_tunings(tuning):
    """64-bit sorts run on runs of at most 8,192 keys whatever base_tile the
    tuning names (2-way or 4-way passes as merge_ways says)."""
    qms.qms_set_tuning(*tuning)
    x = u64_keys(400009, seed=3)
    t = dev64(x)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(host64(t), want)
    import math
    r0 = min(8192, tuning[3])
    for s, c_lt, c_eq, c_gt, L, _ in qms.qms_last_schedule():
        m = min(c_lt, c_gt)
        assert L == (0 if m <= r0 else math.ceil(math.log2(math.ceil(m / r0))))


@needs_gpu
def test_u64_median_of_medians_round():
    """First, middle and last keys are the three smallest: the median-of-3
    pivot is the second smallest key, the round is unbalanced, and the next
    round takes the median-of-medians pivot (8 digit passes for 64 bits)."""
    n = 300001
    x = u64_keys(n, seed=8) | np.uint64(1 << 40)
    x[0], x[n // 2], x[n - 1] = 1, 2, 3
    t = dev64(x)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(host64(t), want)
    sched = qms.qms_last_schedule()
    assert sched[1][5] == 1, sched[:3]
    s, c_lt, c_eq, c_gt, _, _ = sched[1]
    assert min(c_lt, c_gt) >= 2 * (s // 6) - 1


@needs_gpu
@pytest.mark.parametrize("dtype", [np.uint64, np.float64])
def test_batch_64_bit(dtype):
    lens = inputs.log_uniform_lengths(300, seed=11, lo_exp=3, hi_exp=16)
    lens[:5] = [0, 1, 2, 8192, 8193]
    off = inputs.offsets_from_lengths(lens)
    n = int(off[-1])
    x = u64_keys(n, seed=12) if dtype == np.uint64 else np.random.default_rng(12).standard_normal(n)
    t = dev64(x)
    ot = torch.from_numpy(off.view(np.int64)).cuda()
    qms.qms_sort_batch(t, ot, host_offsets=off)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort_segments(x, off)
    np.testing.assert_array_equal(host64(t).view(np.uint64), want.view(np.uint64))


@needs_gpu
def test_u64_2e24_against_oracle():
    x = u64_keys(1 << 24, seed=2)
    t = dev64(x)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(host64(t), want)


def _u64_sorted(t: torch.Tensor) -> bool:
    """Non-decreasing as unsigned 64-bit: compare (high word, low word)."""
    hi = (t >> 32) & 0xFFFFFFFF
    lo = t & 0xFFFFFFFF
    a_hi, b_hi, a_lo, b_lo = hi[:-1], hi[1:], lo[:-1], lo[1:]
    return bool(((a_hi < b_hi) | ((a_hi == b_hi) & (a_lo <= b_lo))).all().item())


def _hash64(t: torch.Tensor) -> tuple:
    """Order-independent sums of mixed 64-bit words (int64 arithmetic wraps)."""
    out = []
    for a, b in ((-7046029254386353131, -4658895280553007687),
                 (-7723592293110705685, -2978262305473349485)):
        h = t * a
        h = h ^ ((h >> 29) & ((1 << 35) - 1))
        h = h * b
        out.append(int(h.sum().item()))
    return tuple(out)


@needs_gpu
def test_u64_2e27_full_size_properties():
    """2^27 64-bit keys (1 GiB): sorted as unsigned, same multiset, and
    sampled ranks by the counting definition."""
    n = 1 << 27
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    t = torch.randint(-2 ** 63, 2 ** 63 - 1, (n,), dtype=torch.int64, device="cuda",
                      generator=g)
    h_in = _hash64(t)
    x_in = t.cpu().numpy().view(np.uint64)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    assert _u64_sorted(t)
    assert _hash64(t) == h_in
    # sampled outputs against the input by the counting definition of rank
    tu = t.cpu().numpy().view(np.uint64)
    for k in (0, 1, n // 3, n // 2, n - 2, n - 1):
        v = tu[k]
        assert np.count_nonzero(x_in < v) <= k < np.count_nonzero(x_in <= v)


@needs_gpu
@pytest.mark.parametrize("kind", ["u64", "f64", "u64_few"])
@pytest.mark.parametrize("n", [2, 3, 2047, 2048, 2049, 100003, 1 << 20])
def test_64_bit_pairs(kind, n):
    """64-bit keys with uint32 payloads (payload = original index): keys
    bit-exact with the oracle's 64-bit build, payloads the exact permutation
    that carries every key to its place."""
    rng = np.random.default_rng(n % 997)
    if kind == "f64":
        x = rng.standard_normal(n)
    elif kind == "u64_few":  # many equal keys
        x = rng.integers(0, 5, n, dtype=np.uint64) << np.uint64(40)
    else:
        x = rng.integers(0, 2 ** 64, n, dtype=np.uint64)
    t = dev64(x)
    v = torch.arange(n, dtype=torch.int32, device="cuda")
    qms.qms_sort_pairs(t, v)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    got = host64(t)
    np.testing.assert_array_equal(got, want)
    vo = v.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(vo), np.arange(n))
    np.testing.assert_array_equal(x[vo], got)


@needs_gpu
def test_64_bit_pairs_batch():
    lens = inputs.log_uniform_lengths(120, seed=61, lo_exp=0, hi_exp=17)
    off = inputs.offsets_from_lengths(lens)
    n = int(off[-1])
    x = np.random.default_rng(62).integers(0, 2 ** 64, n, dtype=np.uint64)
    t = dev64(x)
    v = torch.arange(n, dtype=torch.int32, device="cuda")
    ot = torch.from_numpy(off.view(np.int64)).cuda()
    qms.qms_sort_batch(t, ot, vals=v, host_offsets=off)
    qms.qms_batch_check()
    want, _, _ = oracle.sort_segments(x, off)
    got = host64(t)
    np.testing.assert_array_equal(got, want)
    vo = v.cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(x[vo], got)
    for j in range(lens.size):
        a, b = int(off[j]), int(off[j + 1])
        assert np.array_equal(np.sort(vo[a:b]), np.arange(a, b))


@needs_gpu
def test_64_bit_rejections():
    # 4-byte aligned but not 8-byte aligned 64-bit keys
    buf = torch.zeros(130, dtype=torch.int32, device="cuda")
    lib = qms.load_library()
    rc = lib.qms_sort(buf.data_ptr() + 4, 64, qms.QMS_U64, None)
    assert rc == -2  # QMS_ERR_ALIGN
    out = ctypes.c_uint64()
    rc = lib.qms_mom_pivot(buf.data_ptr() + 4, 64, qms.QMS_U64, ctypes.byref(out), None)
    assert rc == -2


@needs_gpu
def test_u64_automatic_run_width():
    """With the automatic X_THRESH, 64-bit keys mergesort from runs of 2,048
    keys (their network costs more per level than a merge level); keys stay
    bit-exact with the oracle."""
    import math
    defaults = qms.qms_get_tuning()
    qms.qms_set_tuning(4, 4096, 16384, 0, 8192)
    try:
        x = u64_keys(1 << 20, seed=12)
        t = dev64(x)
        qms.qms_sort(t)
        torch.cuda.synchronize()
        want, _, _ = oracle.sort(x, counted=False)
        np.testing.assert_array_equal(host64(t), want)
        sched = qms.qms_last_schedule()
        assert len(sched) >= 1
        for s, c_lt, c_eq, c_gt, L, _ in sched:
            m = min(c_lt, c_gt)
            assert L == (0 if m <= 2048 else math.ceil(math.log2(math.ceil(m / 2048)))), (s, m, L)
    finally:
        qms.qms_set_tuning(*(defaults[f] for f in autotune.FIELDS))

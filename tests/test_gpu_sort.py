"""Parity of the HIP QuickMergesort (through the C ABI) with the CPU oracle.

Keys: the sorted permutation is unique, so the device output must equal the
oracle's output bit for bit.  Pairs: payload order among equal keys is not
unique; keys must equal the oracle's and the pairs invariants must hold.
At 2^26 / 2^28 keys the oracle is too slow to run whole inside a test, so
the device output is checked by properties that hold at any size
(sortedness plus an order-independent multiset hash of input and output),
and sampled output ranks are checked against the oracle's counting
definition of an order statistic.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1804_10062_amd import inputs, qms  # noqa: E402
from tests.gpu_helpers import (as_u64, check_pairs_exact, is_sorted,  # noqa: E402
                               multiset_hash, to_device, to_host)

pytestmark = pytest.mark.gpu

needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")


def _sort_and_compare(x: np.ndarray):
    t = to_device(x)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    got = to_host(t)
    want, _, _ = oracle.sort(x, counted=False)
    assert got.dtype == want.dtype
    np.testing.assert_array_equal(got.view(np.uint32), want.view(np.uint32))


SIZES = [0, 1, 2, 3, 17, 255, 4095, 4096, 4097, 8191, 8192, 8193, 12345, 16383, 16384,
         16385, 32769, 40000, 65543, 1 << 17, 300007]


@needs_gpu
@pytest.mark.parametrize("n", SIZES)
def test_uniform_u32_sizes(n):
    _sort_and_compare(inputs.uniform_u32(n, seed=100 + n))


@needs_gpu
@pytest.mark.parametrize("kind", ["sorted", "reverse", "sorted_swaps", "zipf", "equal"])
@pytest.mark.parametrize("n", [5000, 70001, 1 << 19])
def test_structured_u32(kind, n):
    _sort_and_compare(inputs.make_keys(kind, n, seed=7))


@needs_gpu
def test_config0_uniform_2_20_seed1():
    """One array of 2^20 uniform u32 keys, seed 1: bit-exact with the oracle."""
    _sort_and_compare(inputs.uniform_u32(1 << 20, seed=1))


@needs_gpu
@pytest.mark.parametrize("n", [100, 4097, 99991, 1 << 20])
def test_f32_normal(n):
    _sort_and_compare(inputs.normal_f32(n, seed=n))


@needs_gpu
def test_f32_uniform_with_duplicates():
    _sort_and_compare(inputs.uniform_f32(200003, seed=3))


@needs_gpu
def test_f32_special_values():
    specials = np.array([0.0, -0.0, 1.0, -1.0, np.inf, -np.inf, 1e-45, -1e-45,
                         3.4e38, -3.4e38], dtype=np.float32).view(np.uint32)
    nan_bits = np.array([0x7FC00000, 0xFFC00000, 0x7F800001, 0xFF800001], dtype=np.uint32)
    rng = np.random.default_rng(1)
    x = np.concatenate([np.tile(specials, 700), np.tile(nan_bits, 300),
                        inputs.normal_f32(6000, seed=4).view(np.uint32)])
    x = x[rng.permutation(x.size)].view(np.float32)
    _sort_and_compare(x)


@needs_gpu
@pytest.mark.parametrize("n", [2, 4096, 4097, 12347, 65536 + 77, 300007])
def test_few_distinct_values(n):
    rng = np.random.default_rng(n)
    _sort_and_compare(rng.integers(0, 3, n, dtype=np.uint64).astype(np.uint32))


@needs_gpu
def test_extreme_u32_values():
    rng = np.random.default_rng(2)
    x = rng.choice(np.array([0, 1, 0xFFFFFFFE, 0xFFFFFFFF], dtype=np.uint32), 50000)
    _sort_and_compare(x)


@needs_gpu
@pytest.mark.parametrize("kind,n", [("zipf", 300007), ("uniform", 65543), ("equal", 9000),
                                    ("uniform_f32", 123457), ("uniform", 8191),
                                    ("uniform", 8193), ("sorted_swaps", 70001)])
def test_pairs(kind, n):
    _pairs_and_compare(inputs.make_keys(kind, n, seed=4))


def _pairs_and_compare(k: np.ndarray):
    """Sort k with payload = index: keys bit-exact with the oracle, payloads
    a permutation that carries every key to its place."""
    n = k.size
    kt = to_device(k)
    k_in = kt.clone()
    vt = torch.arange(n, dtype=torch.int32, device="cuda")
    qms.qms_sort_pairs(kt, vt)
    torch.cuda.synchronize()
    check_pairs_exact(k_in, kt, vt)
    want, _, _ = oracle.sort(k, counted=False)
    np.testing.assert_array_equal(to_host(kt).view(np.uint32), want.view(np.uint32))


@needs_gpu
@pytest.mark.parametrize("n", [8191, 8193, 50001])
def test_pairs_extreme_keys(n):
    """Pairs whose keys sit at the ends and the middle of the unsigned order
    (the largest equals the base case's padding key), with ragged tails of
    the 8,192-pair base tile."""
    rng = np.random.default_rng(n)
    vals = np.array([0, 1, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFE, 0xFFFFFFFF], dtype=np.uint32)
    _pairs_and_compare(rng.choice(vals, n))


@needs_gpu
def test_pairs_f32_special_values():
    """f32 pairs over zeros of both signs, infinities, denormals, the largest
    finite values and NaN bit patterns, among normal keys."""
    specials = np.array([0.0, -0.0, 1.0, -1.0, np.inf, -np.inf, 1e-45, -1e-45,
                         3.4e38, -3.4e38], dtype=np.float32).view(np.uint32)
    nan_bits = np.array([0x7FC00000, 0xFFC00000, 0x7F800001, 0xFF800001], dtype=np.uint32)
    rng = np.random.default_rng(5)
    x = np.concatenate([np.tile(specials, 900), np.tile(nan_bits, 400),
                        inputs.normal_f32(7001, seed=6).view(np.uint32)])
    _pairs_and_compare(x[rng.permutation(x.size)].view(np.float32))


@needs_gpu
def test_sort_on_side_stream_and_schedule_log():
    x = inputs.uniform_u32(1 << 18, seed=9)
    t = to_device(x)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        qms.qms_sort(t, stream=s)
    s.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(to_host(t), want)
    sched = qms.qms_last_schedule()
    assert len(sched) > 0
    lo_hi = 1 << 18
    for (s_, lt, eq, gt, levels, rule) in sched:
        # eq == 0: the pivot-equal keys stayed in the ">= p" side (then lt > 0)
        assert s_ == lo_hi and lt + eq + gt == s_ and (eq >= 1 or lt >= 1)
        lo_hi = max(lt, gt)
    assert lo_hi <= qms.qms_get_tiles()["base_tile"]


@needs_gpu
def test_uniform_2_24_exact():
    _sort_and_compare(inputs.uniform_u32(1 << 24, seed=24))


_ORACLE_2_28 = {}


def _oracle_2_28(kind: str, seed: int):
    """Input and oracle output of a 2^28-key workload, computed once per
    module (about 25 s of oracle time for the uniform input)."""
    if kind not in _ORACLE_2_28:
        x = inputs.make_keys(kind, 1 << 28, seed=seed)
        want, _, _ = oracle.sort(x, counted=False)
        _ORACLE_2_28[kind] = (x, want)
    return _ORACLE_2_28[kind]


def _full_size_exact(kind: str, seed: int):
    x, want = _oracle_2_28(kind, seed)
    t = to_device(x)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    got = to_host(t)
    del t
    np.testing.assert_array_equal(got, want)


@needs_gpu
@pytest.mark.parametrize("kind,seed", [("uniform", 2), ("sorted_swaps", 3), ("reverse", 0)])
def test_config1_2_28(kind, seed):
    """2^28 u32 keys (1 GiB), three distributions, every element against the
    oracle; the QuickMergesort loop down to the base tile."""
    _full_size_exact(kind, seed)


@needs_gpu
@pytest.mark.final_path
@pytest.mark.parametrize("kind,seed", [("uniform", 2), ("sorted_swaps", 3), ("reverse", 0)])
def test_config1_2_28_library_defaults(kind, seed):
    """The same at the library's default tuning (the tuning the headline
    measurement runs)."""
    from paper_1804_10062_amd import autotune
    autotune.reset_tuning()
    _full_size_exact(kind, seed)


@needs_gpu
def test_config2_pairs_zipf_2_26():
    """2^26 (key, payload = index) pairs, Zipf(1.1) keys over [0, 2^10)."""
    n = 1 << 26
    k = inputs.zipf_u32(n, seed=4)
    kt = to_device(k)
    k_in = kt.clone()
    vt = torch.arange(n, dtype=torch.int32, device="cuda")
    h_in = multiset_hash(k_in, vt)
    qms.qms_sort_pairs(kt, vt)
    torch.cuda.synchronize()
    check_pairs_exact(k_in, kt, vt)
    assert multiset_hash(kt, vt) == h_in
    # keys against the oracle's sort of the same keys
    want, _, _ = oracle.sort(k, counted=False)
    np.testing.assert_array_equal(to_host(kt), want)


def _structured(kind, n):
    i = np.arange(n, dtype=np.int64)
    if kind == "organ_pipe":
        x = np.minimum(i, n - 1 - i)
    elif kind == "sawtooth":
        x = i % 1000
    elif kind == "reverse_blocks":
        x = (n - 1 - i) // 7
    elif kind == "interleaved":
        x = np.where(i % 2 == 0, i, n - i)
    elif kind == "one_different":
        x = np.zeros(n, dtype=np.int64)
        x[n // 3] = 5
    else:
        raise ValueError(kind)
    return (x * 16).astype(np.uint32)


@needs_gpu
@pytest.mark.parametrize("kind", ["organ_pipe", "sawtooth", "reverse_blocks", "interleaved",
                                  "one_different"])
@pytest.mark.parametrize("n", [100003, 1 << 21])
def test_structured_inputs_bounded_rounds(kind, n):
    """Sorted correctly, and the round count stays logarithmic: after a round
    whose smaller side holds less than 1/16 of the range, the next pivot is a
    sample median."""
    x = _structured(kind, n)
    _sort_and_compare(x)
    rounds = len(qms.qms_last_schedule())
    assert rounds <= 8 * int(np.log2(max(2, n // 16384))) + 16, rounds


@needs_gpu
@pytest.mark.parametrize("n", [1 << 22])
def test_reverse_rounds(n):
    x = inputs.reverse_u32(n)
    _sort_and_compare(x)
    assert len(qms.qms_last_schedule()) <= 40


def _sliced(t: torch.Tensor, step: int = 1 << 28):
    return [t[a:a + step] for a in range(0, t.numel(), step)]


def _sliced_hash(t: torch.Tensor) -> tuple:
    """multiset_hash summed over slices (its terms are sums mod 2^64)."""
    acc = [0, 0]
    for part in _sliced(t):
        for q, v in enumerate(multiset_hash(part)):
            acc[q] = (acc[q] + v) % (1 << 64)
    return tuple(acc)


def _sliced_sorted(t: torch.Tensor, step: int = 1 << 28) -> bool:
    parts = _sliced(t, step)
    if not all(is_sorted(p) for p in parts):
        return False
    return all(int(as_u64(parts[i][-1:]).item()) <= int(as_u64(parts[i + 1][:1]).item())
               for i in range(len(parts) - 1))


@needs_gpu
def test_array_above_2_31_keys():
    """2^31 + 2^20 + 7 uint32 keys (8.6 GB) from the device's seeded
    generator.  Its first partition rounds use more than half of the per-64
    counts, and the scan gives each of its workgroups several chunks of
    tiles.  (A round beyond the per-64 counts, which locates its chunk
    boundaries by walking whole tiles, is the first round of the 2^32 + 2^20
    keys of test_gpu_huge.py.)  Checks that hold at any size: sorted, same
    multiset (both computed in slices)."""
    n = (1 << 31) + (1 << 20) + 7
    gen = torch.Generator(device="cuda")
    gen.manual_seed(31)
    t = torch.randint(-(1 << 31), 1 << 31, (n,), dtype=torch.int32, device="cuda", generator=gen)
    h_in = _sliced_hash(t)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    assert _sliced_sorted(t)
    assert _sliced_hash(t) == h_in

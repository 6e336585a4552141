"""QuickMergeXsort's threshold on the GPU (Sec. "QuickMergeXsort"): the
Mergesort of every round stops at runs of base_tile keys (X_THRESH), which
the base case X sorts; base_tile is a run-time tunable.  Whatever the
threshold, the sorted output is the oracle's bit for bit, and the merge
levels of each round follow from it: L = ceil(lg(m / base_tile)) for the
m keys Mergesorted."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1804_10062_amd import autotune, inputs, qms  # noqa: E402
from tests.gpu_helpers import check_pairs_exact, to_device, to_host  # noqa: E402

pytestmark = pytest.mark.gpu
needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")

THRESHOLDS = (2048, 4096, 8192, 16384)


@pytest.fixture(autouse=True)
def _restore_defaults():
    yield
    if torch.cuda.is_available():
        autotune.reset_tuning()


def _levels(m: int, r0: int) -> int:
    return 0 if m <= r0 else math.ceil(math.log2(math.ceil(m / r0)))


@needs_gpu
@pytest.mark.parametrize("ways", [4, 2])
@pytest.mark.parametrize("t0", THRESHOLDS)
@pytest.mark.parametrize("n", [2049, 3 * 4096 + 17, 16385, 65537, 300007, 1 << 20])
def test_threshold_sort_matches_oracle(t0, ways, n):
    qms.qms_set_tuning(ways, 4096, 16384, t0)
    x = inputs.uniform_u32(n, seed=n % 97 + t0)
    t = to_device(x)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(to_host(t), want)
    # every round Mergesorts its smaller side in L levels of the threshold's runs
    for s, c_lt, c_eq, c_gt, L, _ in qms.qms_last_schedule():
        assert L == _levels(min(c_lt, c_gt), t0), (s, c_lt, c_eq, c_gt, L, t0)


@needs_gpu
@pytest.mark.parametrize("ways", [4, 2])
@pytest.mark.parametrize("n", [16385, 100003, 1 << 20, 3000017])
def test_automatic_threshold(ways, n):
    """base_tile 0: runs of 16,384 keys, or of 8,192 when a 4-way sort's
    level count would otherwise be odd (every pass then merges four runs)."""
    qms.qms_set_tuning(ways, 4096, 16384, 0)
    assert qms.qms_get_tuning()["base_tile"] == 0
    x = inputs.uniform_u32(n, seed=n % 89)
    t = to_device(x)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(to_host(t), want)
    for s, c_lt, c_eq, c_gt, L, _ in qms.qms_last_schedule():
        m = min(c_lt, c_gt)
        l16 = _levels(m, 16384)
        expect = _levels(m, 8192) if (ways == 4 and l16 % 2 == 1) else l16
        assert L == expect, (m, L, expect)
        if ways == 4:
            assert L % 2 == 0


@needs_gpu
@pytest.mark.parametrize("t0", THRESHOLDS)
@pytest.mark.parametrize("kind", ["sorted", "reverse", "sorted_swaps", "zipf", "equal"])
def test_threshold_structured_inputs(t0, kind):
    qms.qms_set_tuning(4, 4096, 16384, t0)
    x = inputs.make_keys(kind, 200003, seed=5)
    t = to_device(x)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(to_host(t), want)


@needs_gpu
@pytest.mark.parametrize("t0", THRESHOLDS)
def test_threshold_f32_total_order(t0):
    qms.qms_set_tuning(4, 4096, 16384, t0)
    x = inputs.normal_f32(150001, seed=t0)
    x[:6] = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, -np.nan], dtype=np.float32)
    t = to_device(x)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(to_host(t).view(np.uint32), want.view(np.uint32))


@needs_gpu
@pytest.mark.parametrize("t0", THRESHOLDS)
def test_threshold_pairs(t0):
    """Key/payload sorts run at most 8,192-key runs: keys bit-exact, every
    payload the original index of its key."""
    qms.qms_set_tuning(2, 4096, 16384, t0)
    k = inputs.make_keys("zipf", 250007, seed=t0)
    kt = to_device(k)
    k_in = kt.clone()
    vt = torch.arange(k.size, dtype=torch.int32, device="cuda")
    qms.qms_sort_pairs(kt, vt)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(k, counted=False)
    np.testing.assert_array_equal(to_host(kt), want)
    check_pairs_exact(k_in, kt, vt)
    for s, c_lt, c_eq, c_gt, L, _ in qms.qms_last_schedule():
        assert L == _levels(min(c_lt, c_gt), min(t0, 8192))


@needs_gpu
@pytest.mark.parametrize("t0", [2048, 8192])
def test_threshold_batch(t0):
    qms.qms_set_tuning(4, 4096, 16384, t0)
    lens = inputs.log_uniform_lengths(400, seed=t0, lo_exp=6, hi_exp=17)
    lens[:4] = [0, 1, t0, t0 + 1]
    off = inputs.offsets_from_lengths(lens)
    x = inputs.uniform_u32(int(off[-1]), seed=3)
    t = to_device(x)
    ot = torch.from_numpy(off.view(np.int64)).cuda()
    qms.qms_sort_batch(t, ot, host_offsets=off)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort_segments(x, off)
    np.testing.assert_array_equal(to_host(t), want)


@needs_gpu
def test_threshold_2e24_against_oracle():
    """A larger sort (many rounds, long Mergesorts) at a small threshold."""
    qms.qms_set_tuning(4, 4096, 16384, 4096)
    x = inputs.uniform_u32(1 << 24, seed=2)
    t = to_device(x)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(to_host(t), want)

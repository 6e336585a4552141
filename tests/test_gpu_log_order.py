"""QMS_U32_LOG: uint32 keys under the expensive comparison of the paper's
Experiments section (the logarithm of each key, evaluated inside every
comparison).  log is strictly increasing and double precision separates
the logarithms of distinct keys below 2^32, so the expected output is the
oracle's plain uint32 sort, bit for bit; only the cost of each comparison
changes (partition, merges, base case and the final network all compare
through it)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1804_10062_amd import autotune, inputs, qms  # noqa: E402
from tests.gpu_helpers import to_device, to_host  # noqa: E402

pytestmark = pytest.mark.gpu
needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")


@pytest.fixture(autouse=True)
def _defaults():
    if torch.cuda.is_available():
        autotune.reset_tuning()
    yield
    if torch.cuda.is_available():
        autotune.reset_tuning()


def _keys(kind: str, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    if kind == "permutation":  # the paper's inputs: a random order of 1..n
        return (rng.permutation(n) + 1).astype(np.uint32)
    x = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    x[: min(n, 3)] = np.array([0, 0xFFFFFFFF, 1], dtype=np.uint32)[: min(n, 3)]
    return x


@needs_gpu
@pytest.mark.parametrize("kind", ["permutation", "uniform"])
@pytest.mark.parametrize("n", [2, 3, 1000, 16384, 16385, 100003, (1 << 20) + 5])
def test_log_order_matches_integer_sort(kind, n):
    x = _keys(kind, n, n % 97)
    t = to_device(x)
    qms.qms_sort(t, dtype=qms.QMS_U32_LOG)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(to_host(t), want)


@needs_gpu
@pytest.mark.parametrize("base_tile", [2048, 8192])
@pytest.mark.parametrize("ways", [4, 2])
def test_log_order_tunings(base_tile, ways):
    qms.qms_set_tuning(ways, 4096, 16384, base_tile, 1 << 20)
    x = _keys("permutation", 3_000_017, base_tile + ways)
    t = to_device(x)
    qms.qms_sort(t, dtype=qms.QMS_U32_LOG)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(to_host(t), want)


@needs_gpu
def test_log_order_batch():
    lens = inputs.log_uniform_lengths(300, seed=12, lo_exp=0, hi_exp=18)
    off = inputs.offsets_from_lengths(lens)
    x = _keys("uniform", int(off[-1]), 13)
    t = to_device(x)
    ot = torch.from_numpy(off.view(np.int64)).cuda()
    qms.qms_sort_batch(t, ot, host_offsets=off, dtype=qms.QMS_U32_LOG)
    qms.qms_batch_check()
    want, _, _ = oracle.sort_segments(x, off)
    np.testing.assert_array_equal(to_host(t), want)


@needs_gpu
def test_log_order_rejects_payloads():
    x = to_device(_keys("uniform", 100, 1))
    v = torch.arange(100, dtype=torch.int32, device="cuda")
    with pytest.raises(qms.QmsError):
        qms.qms_sort_pairs(x, v, dtype=qms.QMS_U32_LOG)
    off = np.array([0, 100], dtype=np.uint64)
    ot = torch.from_numpy(off.view(np.int64)).cuda()
    with pytest.raises(qms.QmsError):
        qms.qms_sort_batch(x, ot, vals=v, host_offsets=off, dtype=qms.QMS_U32_LOG)

"""Seeded random cases across the run-time tunings: key type, distribution,
size, merge arity, partition tile, chunk span, X_THRESH and the final
threshold drawn per case; single arrays and batches.  Every output must be
the oracle's bit for bit (pairs: keys exact, payloads a permutation that
travels with its keys)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1804_10062_amd import autotune, inputs, qms  # noqa: E402
from tests.gpu_helpers import check_pairs_exact, to_device, to_host  # noqa: E402

pytestmark = pytest.mark.gpu
needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")
KINDS = ["uniform", "sorted_swaps", "reverse", "sorted", "zipf", "equal"]


@pytest.fixture(autouse=True)
def _restore_defaults():
    yield
    if torch.cuda.is_available():
        autotune.reset_tuning()


def _random_tuning(rng):
    tp = int(rng.choice([4096, 8192, 16384, 65536]))
    span = int(max(tp, rng.choice([4096, 8192, 16384, 32768, 1 << 20])))
    return (int(rng.choice([4, 2])), tp, span, int(rng.choice([0, 2048, 4096, 8192, 16384])),
            int(rng.choice([8192, 1 << 16, 1 << 20, 1 << 22, 1 << 24])))


@needs_gpu
@pytest.mark.parametrize("case", range(48))
def test_random_single_array(case):
    rng = np.random.default_rng(1000 + case)
    tune = _random_tuning(rng)
    qms.qms_set_tuning(*tune)
    n = int(2 ** rng.uniform(0, 22))
    kind = str(rng.choice(KINDS))
    ty = str(rng.choice(["u32", "f32", "pairs", "u64"]))
    seed = int(rng.integers(1 << 30))
    if ty == "u64":
        x = np.random.default_rng(seed).integers(0, 2 ** 64, n, dtype=np.uint64)
        if kind == "equal":
            x[:] = 12345
        t = torch.from_numpy(x.view(np.int64)).cuda()
        qms.qms_sort(t)
        torch.cuda.synchronize()
        want, _, _ = oracle.sort(x, counted=False)
        np.testing.assert_array_equal(t.cpu().numpy().view(np.uint64), want)
        return
    if ty == "f32":
        x = inputs.normal_f32(n, seed=seed)
        t = to_device(x)
        qms.qms_sort(t)
        torch.cuda.synchronize()
        want, _, _ = oracle.sort(x, counted=False)
        np.testing.assert_array_equal(to_host(t).view(np.uint32), want.view(np.uint32))
        return
    x = inputs.make_keys(kind, n, seed=seed)
    t = to_device(x)
    if ty == "pairs":
        k_in = t.clone()
        v = torch.arange(n, dtype=torch.int32, device="cuda")
        qms.qms_sort_pairs(t, v)
        torch.cuda.synchronize()
        check_pairs_exact(k_in, t, v)
    else:
        qms.qms_sort(t)
        torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(to_host(t), want)


@needs_gpu
@pytest.mark.parametrize("case", range(8))
def test_random_batch(case):
    rng = np.random.default_rng(2000 + case)
    qms.qms_set_tuning(*_random_tuning(rng))
    count = int(rng.integers(1, 300))
    lens = (2 ** rng.uniform(0, float(rng.uniform(8, 20)), count)).astype(np.int64)
    lens[rng.random(count) < 0.05] = 0
    off = inputs.offsets_from_lengths(lens)
    n = int(off[-1])
    ty = str(rng.choice(["u32", "f32", "pairs", "u64"]))
    seed = int(rng.integers(1 << 30))
    ot = torch.from_numpy(off.view(np.int64)).cuda()
    if ty == "u64":
        x = np.random.default_rng(seed).integers(0, 2 ** 40, n, dtype=np.uint64)
        t = torch.from_numpy(x.view(np.int64)).cuda()
        qms.qms_sort_batch(t, ot, host_offsets=off)
        torch.cuda.synchronize()
        want, _, _ = oracle.sort_segments(x, off)
        np.testing.assert_array_equal(t.cpu().numpy().view(np.uint64), want)
        return
    if ty == "f32":
        x = inputs.normal_f32(n, seed=seed)
        t = to_device(x)
        qms.qms_sort_batch(t, ot, host_offsets=off)
        torch.cuda.synchronize()
        want, _, _ = oracle.sort_segments(x, off)
        np.testing.assert_array_equal(to_host(t).view(np.uint32), want.view(np.uint32))
        return
    x = inputs.zipf_u32(n, seed=seed) if rng.random() < 0.5 else inputs.uniform_u32(n, seed=seed)
    t = to_device(x)
    v = torch.arange(n, dtype=torch.int32, device="cuda") if ty == "pairs" else None
    qms.qms_sort_batch(t, ot, vals=v, host_offsets=off)
    torch.cuda.synchronize()
    got = to_host(t)
    want, _, _ = oracle.sort_segments(x, off)
    np.testing.assert_array_equal(got, want)
    if v is not None:
        idx = v.cpu().numpy().view(np.int32).astype(np.int64)
        seg = np.repeat(np.arange(count), lens)
        np.testing.assert_array_equal(np.sort(idx), np.arange(n))  # a permutation
        np.testing.assert_array_equal(seg[idx], seg)               # within its segment
        np.testing.assert_array_equal(x[idx], got)                 # with its key

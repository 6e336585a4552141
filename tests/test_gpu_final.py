"""The loop's last range: a range that a partition round leaves with at
most final_tile keys leaves the QuickMergesort loop and is sorted in place
by X, a bitonic network (QuickXsort with X at the loop level; final_tile
8192 runs the paper's loop to the base tile).  Every input array above the
base tile is partitioned at least once.  Results must be the oracle's bit
for bit, whatever path a range takes."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1804_10062_amd import autotune, inputs, qms  # noqa: E402
from tests.gpu_helpers import check_pairs_exact, to_device, to_host  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.final_path]
needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")


@pytest.fixture(autouse=True)
def _defaults():
    if torch.cuda.is_available():
        autotune.reset_tuning()
    yield
    if torch.cuda.is_available():
        autotune.reset_tuning()


def _check_rounds(n: int, tf: int):
    """The first round partitions the whole array (above the base tile);
    later rounds run only while the range exceeds final_tile."""
    sched = qms.qms_last_schedule()
    if n <= qms.qms_get_tiles()["base_tile"]:
        assert sched == [], sched[:2]
        return
    assert len(sched) >= 1 and sched[0][0] == n
    for s, *_ in sched[1:]:
        assert s > tf


@needs_gpu
@pytest.mark.parametrize("ways", [4, 2])
@pytest.mark.parametrize("tf", [1 << 16, 1 << 20, 1 << 22])
@pytest.mark.parametrize("n", [8193, 16385, 100003, 1 << 20, (1 << 22) + 1])
def test_final_sort_matches_oracle(ways, tf, n):
    qms.qms_set_tuning(ways, 4096, 16384, 0, tf)
    x = inputs.uniform_u32(n, seed=n % 71 + tf % 13)
    t = to_device(x)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(to_host(t), want)
    _check_rounds(n, tf)


@needs_gpu
@pytest.mark.parametrize("kind", ["sorted", "reverse", "sorted_swaps", "zipf", "equal"])
def test_final_structured(kind):
    x = inputs.make_keys(kind, 700001, seed=6)
    t = to_device(x)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(to_host(t), want)


@needs_gpu
@pytest.mark.parametrize("base_tile", [0, 16384, 4096])
def test_final_f32_and_pairs(base_tile):
    qms.qms_set_tuning(4, 4096, 16384, base_tile, 1 << 20)
    x = inputs.normal_f32(300007, seed=base_tile)
    x[:4] = np.array([0.0, -0.0, np.inf, -np.nan], dtype=np.float32)
    t = to_device(x)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(to_host(t).view(np.uint32), want.view(np.uint32))
    k = inputs.make_keys("zipf", 600011, seed=base_tile + 1)
    kt = to_device(k)
    k_in = kt.clone()
    vt = torch.arange(k.size, dtype=torch.int32, device="cuda")
    qms.qms_sort_pairs(kt, vt)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(k, counted=False)
    np.testing.assert_array_equal(to_host(kt), want)
    check_pairs_exact(k_in, kt, vt)


@needs_gpu
@pytest.mark.parametrize("n", [9000, 1 << 20, (1 << 21) + 3])
def test_final_64_bit(n):
    qms.qms_set_tuning(4, 4096, 16384, 0, 1 << 20)
    x = np.random.default_rng(n).integers(0, 2 ** 64, n, dtype=np.uint64)
    t = torch.from_numpy(x.view(np.int64)).cuda()
    qms.qms_sort(t)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(t.cpu().numpy().view(np.uint64), want)
    f = np.random.default_rng(n + 1).standard_normal(n)
    tf = torch.from_numpy(f).cuda()
    qms.qms_sort(tf)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(f, counted=False)
    np.testing.assert_array_equal(tf.cpu().numpy().view(np.uint64), want.view(np.uint64))


@needs_gpu
def test_final_batch_of_every_size_class():
    """Segments of every size class (empty, one key, one tile, just above a
    tile, several ~2^22) in one batch."""
    qms.qms_set_tuning(4, 4096, 16384, 0, 1 << 22)
    lens = np.concatenate([
        # after their first partition the larger sides (at least half of
        # each) are buffered finals: 9 x 2M > 2^24
        np.full(9, (1 << 22) - 7, dtype=np.int64),
        np.array([0, 1, 2, 8192, 16384, 16385, (1 << 22) + 9], dtype=np.int64),
        inputs.log_uniform_lengths(200, seed=4, lo_exp=6, hi_exp=18).astype(np.int64)])
    off = inputs.offsets_from_lengths(lens)
    x = inputs.uniform_u32(int(off[-1]), seed=8)
    t = to_device(x)
    ot = torch.from_numpy(off.view(np.int64)).cuda()
    qms.qms_sort_batch(t, ot, host_offsets=off)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort_segments(x, off)
    np.testing.assert_array_equal(to_host(t), want)


@needs_gpu
def test_final_path_is_the_default_and_large_sorts_use_both():
    """Defaults: a range of 2^24 + 1 keys is partitioned until it fits the
    final threshold, then finished in place by the network."""
    tf = qms.qms_get_tuning()["final_tile"] or (1 << 24)  # 0: automatic, 2^24 for uint32
    n = (1 << 24) + 1
    x = inputs.uniform_u32(n, seed=3)
    t = to_device(x)
    qms.qms_sort(t)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    np.testing.assert_array_equal(to_host(t), want)
    sched = qms.qms_last_schedule()
    assert len(sched) >= 1
    assert all(s > tf for s, *_ in sched)


@needs_gpu
def test_final_only_rounds_back_to_back():
    """Twelve arrays of almost 2^22 keys sorted twice in a row (the second
    call reuses the state of the first)."""
    qms.qms_set_tuning(4, 4096, 16384, 0, 1 << 22)
    lens = np.concatenate([np.full(12, (1 << 22) - 5, dtype=np.int64),
                           np.array([3, 9000, 20000], dtype=np.int64)])
    off = inputs.offsets_from_lengths(lens)
    x = inputs.uniform_u32(int(off[-1]), seed=21)
    t = to_device(x)
    ot = torch.from_numpy(off.view(np.int64)).cuda()
    for _ in range(2):  # twice: the second call reuses the arenas of the first
        t.copy_(to_device(x))
        qms.qms_sort_batch(t, ot, host_offsets=off)
        torch.cuda.synchronize()
    want, _, _ = oracle.sort_segments(x, off)
    np.testing.assert_array_equal(to_host(t), want)


@needs_gpu
@pytest.mark.parametrize("dt", ["u32", "f32", "u64"])
def test_final_network_many_ranges_in_one_round(dt):
    """The request server sorts many arrays per host-driven round, so one
    round's network serves ranges of different lengths (different stage
    counts) through its task tables."""
    import time
    lens = [16385, 20000, 40000, 65536, 65537, 100000, 300001, (1 << 20) + 1, 3000000, 1 << 21]
    rng = np.random.default_rng(len(lens))
    xs, ts = [], []
    for n in lens:
        if dt == "u32":
            x = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
            t = torch.from_numpy(x.view(np.int32)).cuda()
        elif dt == "f32":
            x = rng.standard_normal(n).astype(np.float32)
            t = torch.from_numpy(x).cuda()
        else:
            x = rng.integers(0, 2 ** 64, n, dtype=np.uint64)
            t = torch.from_numpy(x.view(np.int64)).cuda()
        xs.append(x)
        ts.append(t)
    torch.cuda.synchronize()
    qms.qms_set_tuning(4, 4096, 16384, 0, 1 << 22)
    with qms.Server(hbm_budget_bytes=1 << 33) as srv:
        tickets = [srv.submit(t) for t in ts]
        t_end = time.time() + 120
        for tk in tickets:
            while srv.poll(tk)[0] != qms.QMS_OK:
                assert time.time() < t_end, "request not done"
                time.sleep(0.001)
    for x, t in zip(xs, ts):
        want, _, _ = oracle.sort(x, counted=False)
        got = t.cpu().numpy().view(want.dtype)
        np.testing.assert_array_equal(got.view(np.uint8), want.view(np.uint8))


@needs_gpu
@pytest.mark.parametrize("kind,n", [
    ("u32", 3_000_017),                    # below the exit size: one round, then the network
    ("u32", (1 << 24) + (1 << 22) + 3),    # above 2^24: several device-planned rounds
    ("u64", (1 << 23) + 12_345),           # 64-bit keys leave at 2^23
    ("log", (1 << 22) + 5),                # the logarithm order leaves at 2^22
])
def test_qms_sort_captured_at_the_default_exit_size(kind, n):
    """qms_sort under stream capture with the library defaults: the device
    plans the rounds down to the automatic exit size of the key type and the
    network sorts what is left; every replay is the oracle's sort bit for
    bit, with eager work between replays."""
    rng = np.random.default_rng(n)
    if kind == "u64":
        x = rng.integers(0, 2 ** 64, n, dtype=np.uint64)
        src = torch.from_numpy(x.view(np.int64)).cuda()
        dt = qms.QMS_U64
    else:
        x = inputs.uniform_u32(n, seed=n % 11)
        src = to_device(x)
        dt = qms.QMS_U32_LOG if kind == "log" else qms.QMS_U32
    s = torch.cuda.Stream()
    work = src.clone()
    with torch.cuda.stream(s):
        qms.qms_sort(work, stream=s, dtype=dt)  # outside the capture: the stream's workspace
    s.synchronize()
    want, _, _ = oracle.sort(x, counted=False)
    # the eager call (host-planned rounds, the same defaults) is the oracle's too
    np.testing.assert_array_equal(work.cpu().numpy().view(np.uint8), want.view(np.uint8))
    g = torch.cuda.CUDAGraph()
    work.copy_(src)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        qms.qms_sort(work, stream=s, dtype=dt)
    for _ in range(2):
        work.copy_(src)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = work.cpu().numpy()
        np.testing.assert_array_equal(got.view(np.uint8), want.view(np.uint8))
        _ = (src.float() * 2).sum().item()  # eager work between replays
    with torch.cuda.stream(s):
        qms.qms_batch_check(stream=s)
    del g


@needs_gpu
def test_server_batches_at_the_automatic_exit_size():
    """The server sorts each batch of requests in one host-driven loop; with
    the automatic exit size a batch whose requests still in the loop hold
    enough keys together leaves it earlier than one array would (here about
    80 requests of 2^20 keys per key type: the exit falls to 2^20 or below).
    Mixed uint32 and float32 requests, a few small ones among them, each
    bit-exact with the oracle."""
    import time
    rng = np.random.default_rng(2024)
    sizes = (1 << 20) + rng.integers(0, 4096, 164)
    sizes[:4] = [3, 16385, 5000, 300001]
    xs, ts = [], []
    for j, n in enumerate(sizes):
        if j % 2:
            x = rng.standard_normal(int(n)).astype(np.float32)
            t = torch.from_numpy(x).cuda()
        else:
            x = rng.integers(0, 1 << 32, int(n), dtype=np.uint64).astype(np.uint32)
            t = torch.from_numpy(x.view(np.int32)).cuda()
        xs.append(x)
        ts.append(t)
    torch.cuda.synchronize()
    assert qms.qms_get_tuning()["final_tile"] == 0
    with qms.Server(hbm_budget_bytes=1 << 33) as srv:
        tickets = [srv.submit(t) for t in ts]
        t_end = time.time() + 120
        for tk in tickets:
            while srv.poll(tk)[0] != qms.QMS_OK:
                assert time.time() < t_end, "request not done"
                time.sleep(0.001)
    for x, t in zip(xs, ts):
        want, _, _ = oracle.sort(x, counted=False)
        got = t.cpu().numpy().view(want.dtype)
        np.testing.assert_array_equal(got.view(np.uint8), want.view(np.uint8))


@needs_gpu
@pytest.mark.parametrize("kind", ["u32", "u64"])
def test_server_large_batches(kind):
    """Server batches of about 100 large requests (2^21 keys, or 2^20 for
    64-bit keys) with small ones among them, at the library defaults: the
    batch's automatic exit falls to 2^20 keys or below.  Each request
    bit-exact with the oracle."""
    import time
    rng = np.random.default_rng(7 if kind == "u32" else 8)
    big = (1 << 21) if kind == "u32" else (1 << 20)
    sizes = list(big + rng.integers(0, 4096, 100)) + list(rng.integers(2, 20000, 60)) + [2, 3, 16385]
    xs, ts = [], []
    for n in sizes:
        if kind == "u32":
            x = rng.integers(0, 1 << 32, int(n), dtype=np.uint64).astype(np.uint32)
            t = torch.from_numpy(x.view(np.int32)).cuda()
        else:
            x = rng.integers(0, 2 ** 64, int(n), dtype=np.uint64)
            t = torch.from_numpy(x.view(np.int64)).cuda()
        xs.append(x)
        ts.append(t)
    torch.cuda.synchronize()
    assert qms.qms_get_tuning()["final_tile"] == 0
    with qms.Server(hbm_budget_bytes=1 << 34) as srv:
        tickets = [srv.submit(t) for t in ts]
        t_end = time.time() + 150
        for tk in tickets:
            while srv.poll(tk)[0] != qms.QMS_OK:
                assert time.time() < t_end, "request not done"
                time.sleep(0.001)
        assert srv.stats()["batches"] >= 1
    for x, t in zip(xs, ts):
        want, _, _ = oracle.sort(x, counted=False)
        got = t.cpu().numpy().view(want.dtype)
        np.testing.assert_array_equal(got.view(np.uint8), want.view(np.uint8))

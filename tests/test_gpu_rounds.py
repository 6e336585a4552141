"""qms_sort_batch with its rounds planned on the device: bit-exact with the
oracle per segment for every key type, asynchronous (the call returns before
the GPU has run the batch), and capturable in a HIP graph whose replays each
sort a fresh copy of the batch exactly as the eager call does."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1804_10062_amd import inputs, qms  # noqa: E402
from tests.gpu_helpers import (segment_ids, segment_multiset_hash,  # noqa: E402
                               segments_sorted, to_device, to_host)

pytestmark = pytest.mark.gpu
needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")


def _lengths(count, seed, lo_exp, hi_exp, extra=()):
    L = inputs.log_uniform_lengths(count, seed=seed, lo_exp=lo_exp, hi_exp=hi_exp)
    L = np.concatenate([L, np.array(extra, dtype=np.int64)])
    return L[np.random.default_rng(seed).permutation(L.size)]


def _dev(x: np.ndarray) -> torch.Tensor:
    if x.dtype == np.uint64:
        return torch.from_numpy(np.ascontiguousarray(x).view(np.int64)).cuda()
    if x.dtype == np.float64:
        return torch.from_numpy(np.ascontiguousarray(x)).cuda()
    return to_device(x)


def _host(t: torch.Tensor, like: np.ndarray) -> np.ndarray:
    a = t.cpu().numpy()
    return a.view(like.dtype) if a.dtype != like.dtype else a


def _keys(kind: str, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    if kind == "u32":
        return inputs.uniform_u32(n, seed=seed)
    if kind == "f32":
        return inputs.normal_f32(n, seed=seed)
    if kind == "u64":
        return rng.integers(0, 2 ** 64, n, dtype=np.uint64)
    if kind == "f64":
        return rng.standard_normal(n)
    raise ValueError(kind)


@needs_gpu
@pytest.mark.parametrize("kind", ["u32", "f32", "u64", "f64"])
def test_device_rounds_match_oracle(kind):
    lens = _lengths(400, seed=31, lo_exp=0, hi_exp=19,
                    extra=(0, 1, 2, 8191, 8192, 8193, 16384, 16385, 1 << 20))
    off = inputs.offsets_from_lengths(lens)
    x = _keys(kind, int(off[-1]), seed=32)
    kt = _dev(x)
    ot = torch.from_numpy(off.view(np.int64)).cuda()
    qms.qms_sort_batch(kt, ot, host_offsets=off)
    qms.qms_batch_check()
    want, _, _ = oracle.sort_segments(x, off)
    np.testing.assert_array_equal(_host(kt, x), want)


@needs_gpu
@pytest.mark.parametrize("merge_ways,base_tile", [(4, 0), (2, 0), (4, 4096), (2, 8192)])
def test_device_rounds_tunings_and_pairs(merge_ways, base_tile):
    """Key/payload pairs (payload = index) and every merge arity / run width:
    keys exact, payloads the exact permutation carrying their keys."""
    from paper_1804_10062_amd import autotune
    lens = _lengths(150, seed=33, lo_exp=0, hi_exp=18, extra=(0, 1, 9000, 300001))
    off = inputs.offsets_from_lengths(lens)
    n = int(off[-1])
    x = inputs.zipf_u32(n, seed=34)
    try:
        qms.qms_set_tuning(merge_ways, 4096, 16384, base_tile)
        kt = to_device(x)
        vt = torch.arange(n, dtype=torch.int32, device="cuda")
        ot = torch.from_numpy(off.view(np.int64)).cuda()
        qms.qms_sort_batch(kt, ot, vals=vt, host_offsets=off)
        qms.qms_batch_check()
    finally:
        autotune.reset_tuning()
    want, _, _ = oracle.sort_segments(x, off)
    ko = to_host(kt)
    np.testing.assert_array_equal(ko, want)
    vo = to_host(vt).astype(np.int64)
    # payload = original index: each carries its key, and stays in its segment
    np.testing.assert_array_equal(x[vo], ko)
    for j in range(lens.size):
        a, b = int(off[j]), int(off[j + 1])
        assert np.array_equal(np.sort(vo[a:b]), np.arange(a, b))


@needs_gpu
@pytest.mark.parametrize("kind", ["sorted_swaps", "reverse", "zipf", "equal", "sorted"])
def test_device_rounds_structured(kind):
    """Structured inputs take the median-of-medians pivot after unbalanced
    rounds; every segment still finishes inside the schedule."""
    parts = [inputs.make_keys(kind, int(n), seed=35 + i)
             for i, n in enumerate((1 << 20, 300007, 70001, 16385, 5000, 3))]
    lens = np.array([p.size for p in parts], dtype=np.int64)
    off = inputs.offsets_from_lengths(lens)
    x = np.concatenate(parts)
    kt = to_device(x)
    ot = torch.from_numpy(off.view(np.int64)).cuda()
    qms.qms_sort_batch(kt, ot, host_offsets=off)
    qms.qms_batch_check()
    want, _, _ = oracle.sort_segments(x, off)
    np.testing.assert_array_equal(to_host(kt), want)


@needs_gpu
def test_device_rounds_return_before_the_gpu_finishes():
    """The call enqueues the whole batch and returns: an event recorded right
    after it has not completed yet (the GPU still sorts), and the result is
    complete after a synchronisation."""
    lens = _lengths(2000, seed=36, lo_exp=12, hi_exp=20)
    off = inputs.offsets_from_lengths(lens)
    x = inputs.uniform_u32(int(off[-1]), seed=37)
    kt = to_device(x)
    ot = torch.from_numpy(off.view(np.int64)).cuda()
    s = torch.cuda.current_stream()
    # warm-up (allocates this stream's workspace)
    warm = kt[: int(off[3])].clone()
    qms.qms_sort_batch(warm, ot[:4], host_offsets=off[:4])
    torch.cuda.synchronize()
    qms.qms_sort_batch(kt, ot, host_offsets=off)
    ev = torch.cuda.Event()
    ev.record(s)
    pending = not ev.query()
    torch.cuda.synchronize()
    assert pending, "qms_sort_batch waited for the GPU"
    qms.qms_batch_check()
    assert segments_sorted(kt, ot)
    want, _, _ = oracle.sort_segments(x, off)
    np.testing.assert_array_equal(to_host(kt), want)


def _capture_and_replay(src, ot, off, replays=3):
    """Capture qms_sort_batch on `work` (a fresh copy of src before every
    replay), replay it several times with eager work in between, and return
    the result of each replay."""
    s = torch.cuda.Stream()
    work = src.clone()
    with torch.cuda.stream(s):
        qms.qms_sort_batch(work, ot, host_offsets=off)  # warm-up: workspace of s
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    work.copy_(src)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        qms.qms_sort_batch(work, ot, host_offsets=off)
    outs = []
    for _ in range(replays):
        work.copy_(src)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        outs.append(work.clone())
        _ = (src.float() * 2).sum().item()  # eager work between replays
    with torch.cuda.stream(s):
        qms.qms_batch_check(stream=s)
    return outs


@needs_gpu
def test_graph_capture_replays_exact():
    lens = _lengths(500, seed=38, lo_exp=0, hi_exp=19, extra=(0, 1, 16385))
    off = inputs.offsets_from_lengths(lens)
    x = inputs.normal_f32(int(off[-1]), seed=39)
    src = to_device(x)
    ot = torch.from_numpy(off.view(np.int64)).cuda()
    outs = _capture_and_replay(src, ot, off)
    want, _, _ = oracle.sort_segments(x, off)
    for o in outs:
        np.testing.assert_array_equal(to_host(o).view(np.uint32), want.view(np.uint32))


@needs_gpu
def test_graph_capture_20000_arrays():
    """The 20,000-array float32 workload (lengths log-uniform in [2^6, 2^20],
    seed 5) captured once and replayed: every segment sorted with its own
    multiset in every replay, 256 segments (the longest among them) against
    the oracle."""
    lens = inputs.log_uniform_lengths(20000, seed=5, lo_exp=6, hi_exp=20)
    off = inputs.offsets_from_lengths(lens)
    n = int(off[-1])
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    src = torch.randn(n, generator=gen, device="cuda", dtype=torch.float32)
    src[src == 0] = 0.0
    ot = torch.from_numpy(off.view(np.int64)).cuda()
    seg = segment_ids(ot, n)
    h_in = segment_multiset_hash(src, seg)
    rng = np.random.default_rng(1)
    picks = sorted(set(rng.choice(lens.size, 255, replace=False).tolist()) | {int(np.argmax(lens))})
    before = {j: src[int(off[j]):int(off[j + 1])].cpu().numpy() for j in picks}
    outs = _capture_and_replay(src, ot, off, replays=2)
    wants = {j: oracle.sort(before[j], counted=False)[0] for j in picks}
    for o in outs:
        assert segments_sorted(o, ot)
        assert segment_multiset_hash(o, seg) == h_in
        for j in picks:
            got = o[int(off[j]):int(off[j + 1])].cpu().numpy()
            np.testing.assert_array_equal(got.view(np.uint32), wants[j].view(np.uint32))


@needs_gpu
@pytest.mark.parametrize("kind", ["u32", "f32", "pairs", "u64"])
@pytest.mark.parametrize("n", [5000, 16385, 1_000_003])
def test_qms_sort_captured_in_a_graph(kind, n):
    """qms_sort and qms_sort_pairs under stream capture: the rounds are
    planned on the device (nothing read back), the graph replays bit-exact
    with the oracle, with eager work between replays."""
    rng = np.random.default_rng(n)
    if kind == "f32":
        x = inputs.normal_f32(n, seed=n % 7)
        src = to_device(x)
    elif kind == "u64":
        x = rng.integers(0, 2 ** 64, n, dtype=np.uint64)
        src = torch.from_numpy(x.view(np.int64)).cuda()
    else:
        x = inputs.uniform_u32(n, seed=n % 7) if kind == "u32" else inputs.make_keys("zipf", n, seed=3)
        src = to_device(x)
    pairs = kind == "pairs"
    s = torch.cuda.Stream()
    work = src.clone()
    vals = torch.arange(n, dtype=torch.int32, device="cuda") if pairs else None

    def run():
        if pairs:
            qms.qms_sort_pairs(work, vals, stream=s)
        else:
            qms.qms_sort(work, stream=s)

    with torch.cuda.stream(s):
        run()  # warm-up outside the capture: the stream's workspace
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    work.copy_(src)
    if pairs:
        vals.copy_(torch.arange(n, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        run()
    want, _, _ = oracle.sort(x, counted=False)
    for _ in range(3):
        work.copy_(src)
        if pairs:
            vals.copy_(torch.arange(n, dtype=torch.int32, device="cuda"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = work.cpu().numpy()
        np.testing.assert_array_equal(got.view(np.uint8), want.view(np.uint8))
        if pairs:
            vo = vals.cpu().numpy().astype(np.int64)
            assert np.array_equal(np.sort(vo), np.arange(n))
            np.testing.assert_array_equal(x[vo], want)
        _ = (src.float() * 2).sum().item()  # eager work between replays
    with torch.cuda.stream(s):
        qms.qms_batch_check(stream=s)
